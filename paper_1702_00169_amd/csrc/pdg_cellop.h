// Cell solves of the axis-aligned transport (shared by the sweep kernels and
// the fused relaxation + sweep kernel): y = A^{-1} B f for one cell of a
// chain, in downwind-local node order, in the arithmetic of the precision.
#pragma once

#include "pdg_device.h"

namespace pdg {
namespace {

// Cell solve y = A^{-1} B f in the precision of the policy.
template <int PREC, int NP>
struct CellOp {
  using Rt = typename Pol<PREC>::Rt;
  Rt m[NP][NP];
  Rt g[NP];
  Rt a, theta;
  __device__ void load(const OpEntry &op) {
#pragma unroll
    for (int i = 0; i < NP; ++i) {
#pragma unroll
      for (int j = 0; j < NP; ++j) m[i][j] = (PREC == kF32) ? (Rt)op.M32[i * NP + j] : (Rt)op.M[i * NP + j];
      g[i] = (PREC == kF32) ? (Rt)op.g32[i] : (Rt)op.g[i];
    }
    a = (PREC == kF32) ? (Rt)op.a32 : (Rt)op.a;
    theta = (Rt)op.theta;
  }
  __device__ void solve(const Rt (&f)[NP], Rt (&y)[NP], double &, double &) const {
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      Rt acc = m[i][0] * f[0];
#pragma unroll
      for (int j = 1; j < NP; ++j) acc = fma(m[i][j], f[j], acc);
      y[i] = acc;
    }
  }
};

// binary32 cell solve with one binary64 residual correction:
//   r = B f (fp64);  y1 = A32^{-1} r (fp32);  rho = r - A y1 (fp64);
//   y = y1 + A32^{-1} rho (fp32 correction added in fp64).
template <int NP>
struct CellOp<kRefine, NP> {
  using Rt = double;
  double bm[NP][NP];
  double am[NP][NP];
  float ai[NP][NP];
  double g[NP];
  double a, theta;
  __device__ void load(const OpEntry &op) {
#pragma unroll
    for (int i = 0; i < NP; ++i) {
#pragma unroll
      for (int j = 0; j < NP; ++j) {
        bm[i][j] = op.B[i * NP + j];
        am[i][j] = op.A[i * NP + j];
        ai[i][j] = op.Ainv32[i * NP + j];
      }
      g[i] = op.g[i];
    }
    a = op.a;
    theta = op.theta;
  }
  __device__ void solve(const double (&f)[NP], double (&y)[NP], double &cmax, double &ymax) const {
    double r[NP];
    float r32[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      double acc = bm[i][0] * f[0];
#pragma unroll
      for (int j = 1; j < NP; ++j) acc = fma(bm[i][j], f[j], acc);
      r[i] = acc;
      r32[i] = (float)acc;
    }
    float y1[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      float acc = ai[i][0] * r32[0];
#pragma unroll
      for (int j = 1; j < NP; ++j) acc = fmaf(ai[i][j], r32[j], acc);
      y1[i] = acc;
    }
    float rho32[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      double acc = r[i];
#pragma unroll
      for (int j = 0; j < NP; ++j) acc = fma(-am[i][j], (double)y1[j], acc);
      rho32[i] = (float)acc;
    }
#pragma unroll
    for (int i = 0; i < NP; ++i) {
      float acc = ai[i][0] * rho32[0];
#pragma unroll
      for (int j = 1; j < NP; ++j) acc = fmaf(ai[i][j], rho32[j], acc);
      y[i] = (double)y1[i] + (double)acc;
      cmax = fmax(cmax, fabs((double)acc));
      ymax = fmax(ymax, fabs(y[i]));
    }
  }
};

// The 48-bit state keeps the arithmetic of binary32 + refinement.
template <int NP>
struct CellOp<kP48, NP> : CellOp<kRefine, NP> {};

}  // namespace
}  // namespace pdg
