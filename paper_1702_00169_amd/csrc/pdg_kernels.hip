// gfx950 kernels of the PDG transport sweep and relaxation.
//
// Transport (Sec. 4.1-4.2 of the paper, eq. transport_cn).  For an
// axis-aligned velocity v = +-|v| e_a on a uniform Cartesian mesh, the cell
// block Gamma_{L<-L} of eq. DG_reduit is the one-dimensional upwind operator
// along axis a, repeated for every transverse node, and Gamma_{L<-R} couples
// only the inflow node of a line to the outflow node of the upwind cell on the
// same line.  The implicit step therefore splits into independent chains: a
// line of n_a cells along axis a, each holding NP = d+1 nodes.  In downwind
// order (local node 0 = inflow, NP-1 = outflow) cell l of a chain solves
//
//   A x_l = B f_l + c0 u_l e_0,   u_l = theta x_{l-1,out} + (1-theta) f_{l-1,out}
//
// (u_0 from the inflow data fb), i.e. x_l = M f_l + g u_l with M = A^{-1} B,
// g = c0 A^{-1} e_0.  The scalar u obeys the affine recurrence
//
//   u_{l+1} = a u_l + (theta (M f_l)_out + (1-theta) f_{l,out}),  a = theta g_out,
//
// so a chain can be cut into segments that are solved in parallel: every
// thread owns S consecutive cells of one chain, computes M f for them and the
// affine map (alpha, beta) taking its inflow u to its outflow u, the maps of
// the segments before it are composed in order (a sequential combine over at
// most kBlock/C segments), and the thread finishes its cells with the exact
// inflow.  The result is the block-triangular solve of the paper, with the
// rounding order of the combine instead of cell after cell.
//
// Two thread mappings share that arithmetic:
//  * chains along a strided axis (y, z): a group of C consecutive chains
//    reads consecutive addresses, so each thread loads its S cells directly
//    from HBM (C lanes per 8-byte row, fully coalesced) and the segment maps
//    are combined through LDS;
//  * chains along the contiguous axis x: one cell per thread with lanes in
//    downwind order along the rows, so loads and stores are contiguous row
//    segments; the segment maps (one cell each) are combined by a segmented
//    Kogge-Stone scan inside each wave and a carry across waves and chunks.
//
// Relaxation (eq. collision_cn, Sec. 4.4): one thread per node reads the nv x m
// values of that node (node-major layout: coalesced across threads), forms
// w with a compensated (Neumaier) sum in a fixed velocity order, evaluates
// f^eq(w) and applies f += omega (f^eq - f).
#include <float.h>
#include <math.h>

#include <algorithm>

#include "pdg_internal.h"

#ifndef PDG_NONTEMPORAL
#define PDG_NONTEMPORAL 0
#endif

namespace pdg {
namespace {

// State traffic: every value is read once and written once per kernel, so
// the loads and stores may carry the streaming (non-temporal) hint.
template <class T>
__device__ __forceinline__ T ld_state(const T *p) {
#if PDG_NONTEMPORAL
  return __builtin_nontemporal_load(p);
#else
  return *p;
#endif
}
template <class T>
__device__ __forceinline__ void st_state(T *p, T v) {
#if PDG_NONTEMPORAL
  __builtin_nontemporal_store(v, p);
#else
  *p = v;
#endif
}

template <int PREC>
struct Pol;
template <>
struct Pol<kF64> {
  using St = double;  // state
  using Rt = double;  // recurrence / arithmetic
};
template <>
struct Pol<kF32> {
  using St = float;
  using Rt = float;
};
template <>
struct Pol<kRefine> {
  using St = double;
  using Rt = double;
};

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

// Chains along the contiguous axis: one cell per thread, lanes in downwind
// order over the item's rows (rows of one family are contiguous in memory,
// so every load and store is a coalesced row segment).  The inflow values
// obey u_{l+1} = a u_l + beta_l with beta_l = theta (M f_l)_out +
// (1 - theta) f_{l,out}; the chain head absorbs its boundary inflow
// (beta += a u_b).  A segmented inclusive scan I_l = u_{l+1} runs inside each
// wave (Kogge-Stone with the powers a^(2^s)), then across the four waves
// and across 256-cell chunks through a carry.
template <int PREC, int NP>
__device__ __forceinline__ void sweep_rows(const SweepItem &it, const SweepDesc &d, const CellOp<PREC, NP> &op,
                                           typename Pol<PREC>::St *__restrict__ f,
                                           const double *__restrict__ fb_old, const double *__restrict__ fb_new,
                                           typename Pol<PREC>::Rt (*wtot)[4], int (*wopen)[4], double &cmax,
                                           double &ymax) {
  using St = typename Pol<PREC>::St;
  using Rt = typename Pol<PREC>::Rt;
  constexpr int KCH = 4;  // 256-cell chunks whose loads are issued together
  const Rt theta = op.theta;
  const Rt omt = (Rt)1 - theta;
  const Rt a = op.a;
  Rt apow[7];  // a^(2^s)
  apow[0] = a;
#pragma unroll
  for (int s = 1; s < 7; ++s) apow[s] = apow[s - 1] * apow[s - 1];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int wv = t >> 6;
  const int n = d.n_a;
  const int total = it.count * n;  // < 2^16 (host), so the float quotient below is exact
  const float inv_n = 1.0f / (float)n;
  const bool rev = d.cell_step < 0;
  const int64_t rowbase = it.base + d.plane0 + (int64_t)it.tau0 * d.hi_stride;
  // a^(lane+1) by binary powering: weight of the wave's carry at this lane
  Rt alane = 1;
  {
    const int e = lane + 1;
#pragma unroll
    for (int s = 0; s < 7; ++s)
      if (e & (1 << s)) alane *= apow[s];
  }
  Rt carry = 0;  // I of the last element of the previous chunk
  int par = 0;
  for (int c0 = 0; c0 < total; c0 += KCH * kBlock) {
    // issue the loads of KCH chunks before any of them is used
    Rt fv[KCH][NP];
    int pidx[KCH], row[KCH], pos[KCH];
#pragma unroll
    for (int k = 0; k < KCH; ++k) {
      const int e = c0 + k * kBlock + t;
      const bool valid = e < total;
      const int pi = rev ? total - 1 - e : e;  // physical flat index (row-major rows x n)
      const int r = valid ? (int)(((float)pi + 0.5f) * inv_n) : 0;
      const int x = pi - r * n;
      pidx[k] = valid ? pi : -1;
      row[k] = r;
      pos[k] = rev ? n - 1 - x : x;  // downwind position in the chain
#pragma unroll
      for (int q = 0; q < NP; ++q) fv[k][q] = valid ? (Rt)ld_state(f + rowbase + q * d.plane_step + pi) : (Rt)0;
    }
#pragma unroll
    for (int k = 0; k < KCH; ++k, par ^= 1) {
      if (c0 + k * kBlock >= total) break;  // uniform across the block
      const bool valid = pidx[k] >= 0;
      const int l = pos[k];
      const int r = row[k];
      Rt y[NP];
      op.solve(fv[k], y, cmax, ymax);
      const Rt fo = fv[k][NP - 1];
      Rt beta = valid ? theta * y[NP - 1] + omt * fo : (Rt)0;
      Rt ub = 0;
      if (valid && l == 0) {
        ub = theta * (Rt)fb_new[it.fb + r] + omt * (Rt)fb_old[it.fb + r];
        beta = fma(a, ub, beta);
      }
      // segmented scan inside the wave
      const int kw = l < lane ? l : lane;  // lanes back to the segment start within the wave
      Rt I = beta;
#pragma unroll
      for (int s = 0; s < 6; ++s) {
        const int dd = 1 << s;
        const Rt up = __shfl_up(I, dd, 64);
        if (kw >= dd) I = fma(apow[s], up, I);
      }
      if (lane == 63) {
        wtot[par][wv] = I;
        wopen[par][wv] = (l > 63) ? 1 : 0;  // segment reaches back before the wave
      }
      __syncthreads();
      // carry into each wave, then into the next chunk
      Rt cin = carry;
      Rt cw = carry;
#pragma unroll
      for (int w = 0; w < 4; ++w) {
        if (w == wv) cin = cw;
        cw = wopen[par][w] ? fma(apow[6], cw, wtot[par][w]) : wtot[par][w];
      }
      if (l > lane) I = fma(alane, cin, I);
      const Rt prev = __shfl_up(I, 1, 64);
      const Rt u = (l == 0) ? ub : (lane > 0 ? prev : cin);
      if (valid) {
#pragma unroll
        for (int q = 0; q < NP; ++q) st_state(f + rowbase + q * d.plane_step + pidx[k], (St)fma(op.g[q], u, y[q]));
      }
      carry = cw;
    }
  }
}

template <int PREC, int NP, int SMAX>
__global__ __launch_bounds__(kBlock) void sweep_kernel(const SweepItem *__restrict__ items,
                                                      const SweepDesc *__restrict__ descs,
                                                      const OpEntry *__restrict__ ops, int dt_idx,
                                                      typename Pol<PREC>::St *__restrict__ f,
                                                      const double *__restrict__ fb_old,
                                                      const double *__restrict__ fb_new,
                                                      double *__restrict__ stats) {
  using St = typename Pol<PREC>::St;
  using Rt = typename Pol<PREC>::Rt;
  __shared__ Rt xa[2][kBlock];
  __shared__ Rt xb[2][kBlock];
  const SweepItem it = items[blockIdx.x];
  const SweepDesc d = descs[it.desc];
  CellOp<PREC, NP> op;
  op.load(ops[d.op + dt_idx]);
  const Rt theta = op.theta;
  const Rt omt = (Rt)1 - theta;

  const int t = threadIdx.x;
  double cmax = 0.0, ymax = 0.0;

  if (it.xk) {
    __shared__ Rt wtot[2][4];
    __shared__ int wopen[2][4];
    sweep_rows<PREC, NP>(it, d, op, f, fb_old, fb_new, wtot, wopen, cmax, ymax);
  } else {
  // chains along a strided axis: thread (c, p) owns segment p of chain c
  const int C = it.C;        // chains per workgroup
  const int S = it.S;        // cells per segment, <= SMAX
  const int P = kBlock / C;  // segments per chain window
  const int c = t % C;
  const int p = t / C;
  const bool active = c < it.count;
  const int n = d.n_a;
  const int window = P * S;
  Rt u = 0;
  if (active) u = theta * (Rt)fb_new[it.fb + c] + omt * (Rt)fb_old[it.fb + c];
  const int tau = it.tau0 + c;
  const int64_t chain = it.base + (int64_t)(tau % d.nx) + (int64_t)(tau / d.nx) * d.hi_stride + d.cell0 + d.plane0;
  int wpar = 0;
  for (int w0 = 0; w0 < n; w0 += window, wpar ^= 1) {
    const int lb = w0 + p * S;
    const int cnt = active ? max(0, min(S, n - lb)) : 0;
    Rt y[SMAX][NP];
    Rt fo[SMAX];
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
      Rt fv[NP];
      if (s < cnt) {
#pragma unroll
        for (int q = 0; q < NP; ++q) fv[q] = (Rt)ld_state(f + chain + (int64_t)(lb + s) * d.cell_step + q * d.plane_step);
      } else {
#pragma unroll
        for (int q = 0; q < NP; ++q) fv[q] = 0;
      }
      fo[s] = fv[NP - 1];
      op.solve(fv, y[s], cmax, ymax);
    }
    // affine map of this segment: u_out = alpha u_in + beta
    Rt alpha = 1, beta = 0;
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
      if (s < cnt) {
        beta = fma(op.a, beta, theta * y[s][NP - 1] + omt * fo[s]);
        alpha *= op.a;
      }
    }
    xa[wpar][t] = alpha;
    xb[wpar][t] = beta;
    __syncthreads();
    Rt uin = u;
    for (int q = 0; q < p; ++q) uin = fma(xa[wpar][c + C * q], uin, xb[wpar][c + C * q]);
    Rt unext = uin;
    for (int q = p; q < P; ++q) unext = fma(xa[wpar][c + C * q], unext, xb[wpar][c + C * q]);
    // finish the segment with its exact inflow
    Rt uu = uin;
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
      if (s < cnt) {
        Rt xo = 0;
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          const Rt xv = fma(op.g[q], uu, y[s][q]);
          if (q == NP - 1) xo = xv;
          st_state(f + chain + (int64_t)(lb + s) * d.cell_step + q * d.plane_step, (St)xv);
        }
        uu = theta * xo + omt * fo[s];
      }
    }
    u = unext;
  }

  }

  if (PREC == kRefine) {
    // block maxima of |correction| and |solution|, one pair per workgroup
    __syncthreads();
    double *red = reinterpret_cast<double *>(&xa[0][0]);
    red[t] = cmax;
    red[kBlock + t] = ymax;
    __syncthreads();
    for (int off = kBlock / 2; off > 0; off >>= 1) {
      if (t < off) {
        red[t] = fmax(red[t], red[t + off]);
        red[kBlock + t] = fmax(red[kBlock + t], red[kBlock + t + off]);
      }
      __syncthreads();
    }
    if (t == 0) {
      stats[2 * (int64_t)blockIdx.x] = red[0];
      stats[2 * (int64_t)blockIdx.x + 1] = red[kBlock];
    }
  }
}

// ---------------------------------------------------------------------------
// inversion of the cell blocks (binary64 Gauss-Jordan, partial pivoting)
// ---------------------------------------------------------------------------
__global__ void invert_kernel(OpEntry *ops, int n_ops) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n_ops) return;
  OpEntry &op = ops[e];
  const int np = op.np;
  double a[kMaxNP][kMaxNP], inv[kMaxNP][kMaxNP];
  double norm = 0.0;
  for (int i = 0; i < kMaxNP; ++i)
    for (int j = 0; j < kMaxNP; ++j) {
      a[i][j] = (i < np && j < np) ? op.A[i * np + j] : 0.0;
      inv[i][j] = (i == j) ? 1.0 : 0.0;
      norm = fmax(norm, fabs(a[i][j]));
    }
  int singular = 0;
  for (int col = 0; col < np; ++col) {
    int piv = col;
    for (int r = col + 1; r < np; ++r)
      if (fabs(a[r][col]) > fabs(a[piv][col])) piv = r;
    if (!(fabs(a[piv][col]) > 1e-300 * norm)) {
      singular = 1;
      break;
    }
    if (piv != col) {
      for (int j = 0; j < np; ++j) {
        double tmp = a[col][j];
        a[col][j] = a[piv][j];
        a[piv][j] = tmp;
        tmp = inv[col][j];
        inv[col][j] = inv[piv][j];
        inv[piv][j] = tmp;
      }
    }
    const double rp = 1.0 / a[col][col];
    for (int j = 0; j < np; ++j) {
      a[col][j] *= rp;
      inv[col][j] *= rp;
    }
    for (int r = 0; r < np; ++r) {
      if (r == col) continue;
      const double fct = a[r][col];
      if (fct == 0.0) continue;
      for (int j = 0; j < np; ++j) {
        a[r][j] = fma(-fct, a[col][j], a[r][j]);
        inv[r][j] = fma(-fct, inv[col][j], inv[r][j]);
      }
    }
  }
  op.singular = singular;
  if (singular) return;
  for (int i = 0; i < np; ++i) {
    for (int j = 0; j < np; ++j) {
      double acc = 0.0;
      for (int k = 0; k < np; ++k) acc = fma(inv[i][k], op.B[k * np + j], acc);
      op.M[i * np + j] = acc;
      op.M32[i * np + j] = (float)acc;
      op.Ainv[i * np + j] = inv[i][j];
      op.Ainv32[i * np + j] = (float)inv[i][j];
    }
    op.g[i] = op.c0 * inv[i][0];
    op.g32[i] = (float)op.g[i];
  }
  op.a = op.theta * op.g[np - 1];
  op.a32 = (float)op.theta * op.g32[np - 1];
}

// ---------------------------------------------------------------------------
// equilibrium and relaxation
// ---------------------------------------------------------------------------
// f^eq_{i,k}(w) = w_k / nv + s_i q^{a_i}_k(w) / (2 lambda) for v_i = s_i lambda e_{a_i}.
template <int M>
__device__ inline void flux_dir(const RelaxDesc &d, const double (&w)[M], int axis, double (&q)[M]) {
  if (d.feq == 0) {
#pragma unroll
    for (int k = 0; k < M; ++k) q[k] = d.param[axis] * w[k];
  } else {
    // compressible Euler, w = (rho, rho u_1..D, E), M = D + 2
    const double gam = d.param[0];
    const int dim = M - 2;
    const double rho = w[0];
    const double rinv = 1.0 / rho;
    double ke = 0.0;
#pragma unroll
    for (int l = 0; l < M - 2; ++l) ke = fma(w[1 + l], w[1 + l] * rinv, ke);
    const double pr = (gam - 1.0) * (w[M - 1] - 0.5 * ke);
    const double ua = w[1 + axis] * rinv;
    q[0] = w[1 + axis];
#pragma unroll
    for (int l = 0; l < M - 2; ++l) q[1 + l] = w[1 + axis] * (w[1 + l] * rinv) + (l == axis ? pr : 0.0);
    q[M - 1] = (w[M - 1] + pr) * ua;
    (void)dim;
  }
}

template <int NV, int M>
__device__ inline void equilibrium(const RelaxDesc &d, const double (&w)[M], double (&fe)[NV][M]) {
  double qd[3][M];
  const int dim = d.dim;
#pragma unroll
  for (int a = 0; a < 3; ++a)
    if (a < dim) flux_dir<M>(d, w, a, qd[a]);
  const double inv_nv = 1.0 / NV;
  const double h2l = 0.5 / d.lambda;
#pragma unroll
  for (int i = 0; i < NV; ++i) {
    const int ax = d.axis[i];
    const double sg = d.sign[i] * h2l;
#pragma unroll
    for (int k = 0; k < M; ++k) {
      double qv = 0.0;
#pragma unroll
      for (int a = 0; a < 3; ++a)
        if (a == ax) qv = qd[a][k];
      fe[i][k] = fma(sg, qv, w[k] * inv_nv);
    }
  }
}

// mode 0: relax (w from f);  mode 1: f = f^eq(w_in).  The flux of one axis
// at a time is formed and the velocities along that axis are updated at once,
// so the n_v x m equilibrium values never live in registers together.
template <int PREC, int NV, int M>
__global__ __launch_bounds__(kBlock) void relax_kernel(const RelaxItem *__restrict__ items,
                                                      const RelaxDesc *__restrict__ descs,
                                                      typename Pol<PREC>::St *__restrict__ f,
                                                      double *__restrict__ w_out,
                                                      const double *__restrict__ w_in, double omega, int mode) {
  using St = typename Pol<PREC>::St;
  const RelaxItem it = items[blockIdx.x];
  const RelaxDesc d = descs[it.desc];
  const int64_t nodes = d.nodes;
  St *fi = f + d.f_base;
  const double inv_nv = 1.0 / NV;
  const double h2l = 0.5 / d.lambda;
  for (int64_t node = it.node0 + threadIdx.x; node < it.node0 + it.count; node += kBlock) {
    double w[M];
    double fv[NV][M];
    if (mode == 0) {
#pragma unroll
      for (int i = 0; i < NV; ++i)
#pragma unroll
        for (int k = 0; k < M; ++k) fv[i][k] = (double)ld_state(fi + (int64_t)(i * M + k) * nodes + node);
#pragma unroll
      for (int k = 0; k < M; ++k) {
        // Neumaier compensated sum over velocities, fixed order
        double s = fv[0][k], comp = 0.0;
#pragma unroll
        for (int i = 1; i < NV; ++i) {
          const double x = fv[i][k];
          const double tt = s + x;
          comp += (fabs(s) >= fabs(x)) ? ((s - tt) + x) : ((x - tt) + s);
          s = tt;
        }
        w[k] = s + comp;
      }
    } else {
#pragma unroll
      for (int k = 0; k < M; ++k) w[k] = w_in[d.w_base + (int64_t)k * nodes + node];
#pragma unroll
      for (int i = 0; i < NV; ++i)
#pragma unroll
        for (int k = 0; k < M; ++k) fv[i][k] = 0.0;
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (a >= d.dim) break;
      double q[M];
      flux_dir<M>(d, w, a, q);
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        if (d.axis[i] != a) continue;
        const double sg = d.sign[i] * h2l;
#pragma unroll
        for (int k = 0; k < M; ++k) {
          const double fe = fma(sg, q[k], w[k] * inv_nv);
          const double nv = (mode == 0) ? fma(omega, fe - fv[i][k], fv[i][k]) : fe;
          st_state(fi + (int64_t)(i * M + k) * nodes + node, (St)nv);
        }
      }
    }
    if (w_out != nullptr) {
#pragma unroll
      for (int k = 0; k < M; ++k) w_out[d.w_base + (int64_t)k * nodes + node] = w[k];
    }
  }
}

template <int NV, int M>
__global__ __launch_bounds__(kBlock) void inflow_eq_kernel(const InflowDesc *__restrict__ items,
                                                          const RelaxDesc *__restrict__ descs,
                                                          const double *__restrict__ w_inflow,
                                                          double *__restrict__ fb) {
  const InflowDesc it = items[blockIdx.y];
  const RelaxDesc d = descs[it.relax_desc];
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < it.per_comp; e += (int64_t)gridDim.x * kBlock) {
    double w[M];
#pragma unroll
    for (int k = 0; k < M; ++k) w[k] = w_inflow[it.w_base + k * it.per_comp + e];
    double fe[NV][M];
    equilibrium<NV, M>(d, w, fe);
#pragma unroll
    for (int i = 0; i < NV; ++i)
      if (i == it.vel) {
#pragma unroll
        for (int k = 0; k < M; ++k) fb[it.fb_base + k * it.per_comp + e] = fe[i][k];
      }
  }
}

// ---------------------------------------------------------------------------
// D2Q9 lattice model of the isothermal Euler equations with gravity (Sec. 5.1)
// ---------------------------------------------------------------------------
// w = P f = (rho, rho u_x, rho u_y); with c^2 = lambda^2 / 3 and
// s_i = (c_i . u) / lambda for v_i = lambda c_i:
//   f_i^eq = wt_i rho (1 + 3 s_i + 9/2 s_i^2 - 3/2 |u|^2 / lambda^2),
// wt = 4/9 (c_i = 0), 1/9 (|c_i| = 1), 1/36 (|c_i|^2 = 2).
__device__ inline double lattice_weight(int cx, int cy) {
  const int r = cx * cx + cy * cy;
  return r == 0 ? 4.0 / 9.0 : (r == 1 ? 1.0 / 9.0 : 1.0 / 36.0);
}

__device__ inline double lattice_feq(double wt, int cx, int cy, double rho, double jx, double jy, double inv_l) {
  const double ux = jx / rho, uy = jy / rho;
  const double s = (cx * ux + cy * uy) * inv_l;
  const double uu = (ux * ux + uy * uy) * inv_l * inv_l;
  return wt * rho * (1.0 + 3.0 * s + 4.5 * s * s - 1.5 * uu);
}

// Source step S_2(h) on the equilibrium part (Sec. 3.2): the moments move by
// h S(w), S = (0, 0, -g rho), which keeps rho, so the Crank-Nicolson update
// is exact; f moves by f^eq(w') - f^eq(w).
__device__ inline void lattice_source(const RelaxDesc &d, double (&fv)[9], const double (&wt)[9], double rho,
                                      double jx, double &jy, double h, double inv_l) {
  const double jy2 = jy - h * d.param[0] * rho;
#pragma unroll
  for (int i = 0; i < 9; ++i)
    fv[i] += lattice_feq(wt[i], d.cx[i], d.cy[i], rho, jx, jy2, inv_l) -
             lattice_feq(wt[i], d.cx[i], d.cy[i], rho, jx, jy, inv_l);
  jy = jy2;
}

template <int PREC>
__global__ __launch_bounds__(kBlock) void lattice_kernel(const RelaxItem *__restrict__ items,
                                                        const RelaxDesc *__restrict__ descs,
                                                        typename Pol<PREC>::St *__restrict__ f,
                                                        double *__restrict__ w_out, const double *__restrict__ w_in,
                                                        double omega, double h_pre, double h_post, int mode) {
  using St = typename Pol<PREC>::St;
  const RelaxItem it = items[blockIdx.x];
  const RelaxDesc d = descs[it.desc];
  const int64_t nodes = d.nodes;
  St *fi = f + d.f_base;
  const double lam = d.lambda;
  const double inv_l = 1.0 / lam;
  const bool source = d.param[0] != 0.0;
  double wt[9];
#pragma unroll
  for (int i = 0; i < 9; ++i) wt[i] = lattice_weight(d.cx[i], d.cy[i]);
  for (int64_t node = it.node0 + threadIdx.x; node < it.node0 + it.count; node += kBlock) {
    double fv[9];
    double rho, jx, jy;
    if (mode == 0) {
#pragma unroll
      for (int i = 0; i < 9; ++i) fv[i] = (double)ld_state(fi + (int64_t)i * nodes + node);
      // moments: Neumaier compensated sums in a fixed order
      double acc[3] = {fv[0], fv[0] * d.cx[0], fv[0] * d.cy[0]};
      double comp[3] = {0.0, 0.0, 0.0};
#pragma unroll
      for (int i = 1; i < 9; ++i) {
        const double x[3] = {fv[i], fv[i] * d.cx[i], fv[i] * d.cy[i]};
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const double tt = acc[k] + x[k];
          comp[k] += (fabs(acc[k]) >= fabs(x[k])) ? ((acc[k] - tt) + x[k]) : ((x[k] - tt) + acc[k]);
          acc[k] = tt;
        }
      }
      rho = acc[0] + comp[0];
      jx = lam * (acc[1] + comp[1]);
      jy = lam * (acc[2] + comp[2]);
    } else {
      rho = w_in[d.w_base + node];
      jx = w_in[d.w_base + nodes + node];
      jy = w_in[d.w_base + 2 * nodes + node];
#pragma unroll
      for (int i = 0; i < 9; ++i) fv[i] = 0.0;
    }
    if (mode == 1) {
#pragma unroll
      for (int i = 0; i < 9; ++i)
        st_state(fi + (int64_t)i * nodes + node, (St)lattice_feq(wt[i], d.cx[i], d.cy[i], rho, jx, jy, inv_l));
      continue;
    }
    if (source && h_pre != 0.0) lattice_source(d, fv, wt, rho, jx, jy, h_pre, inv_l);
#pragma unroll
    for (int i = 0; i < 9; ++i)
      fv[i] = fma(omega, lattice_feq(wt[i], d.cx[i], d.cy[i], rho, jx, jy, inv_l) - fv[i], fv[i]);
    if (source && h_post != 0.0) lattice_source(d, fv, wt, rho, jx, jy, h_post, inv_l);
#pragma unroll
    for (int i = 0; i < 9; ++i) st_state(fi + (int64_t)i * nodes + node, (St)fv[i]);
    if (w_out != nullptr) {
      w_out[d.w_base + node] = rho;
      w_out[d.w_base + nodes + node] = jx;
      w_out[d.w_base + 2 * nodes + node] = jy;
    }
  }
}

__global__ __launch_bounds__(kBlock) void lattice_inflow_kernel(const InflowDesc *__restrict__ items,
                                                               const RelaxDesc *__restrict__ descs,
                                                               const double *__restrict__ w_inflow,
                                                               double *__restrict__ fb) {
  const InflowDesc it = items[blockIdx.y];
  const RelaxDesc d = descs[it.relax_desc];
  const int cx = d.cx[it.vel], cy = d.cy[it.vel];
  const double wt = lattice_weight(cx, cy);
  const double inv_l = 1.0 / d.lambda;
  for (int64_t e = (int64_t)blockIdx.x * kBlock + threadIdx.x; e < it.per_comp; e += (int64_t)gridDim.x * kBlock) {
    const double rho = w_inflow[it.w_base + e];
    const double jx = w_inflow[it.w_base + it.per_comp + e];
    const double jy = w_inflow[it.w_base + 2 * it.per_comp + e];
    fb[it.fb_base + e] = lattice_feq(wt, cx, cy, rho, jx, jy, inv_l);
  }
}

__global__ void fill_kernel(double *p, int64_t n, double value) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

// ---------------------------------------------------------------------------
// dense path: velocities with two or three non-zero components
// ---------------------------------------------------------------------------
// Operator row layout (doubles): M (N x N) | G_0 G_1 G_2 (N x F each) | A | B | Ainv
struct DenseRowLayout {
  int64_t n, f;
  __host__ __device__ int64_t g(int a) const { return n * n + a * n * f; }
  __host__ __device__ int64_t a_off() const { return n * n + 3 * n * f; }
  __host__ __device__ int64_t b_off() const { return 2 * n * n + 3 * n * f; }
  __host__ __device__ int64_t ai_off() const { return 3 * n * n + 3 * n * f; }
};

__global__ __launch_bounds__(kDenseThreads) void dense_invert_kernel(double *table, const int64_t *row_off,
                                                                    const DenseDesc *descs,
                                                                    const int32_t *row_desc, const double *c0,
                                                                    int32_t *flags, int n, int F) {
  __shared__ double a[kDenseMaxN][kDenseMaxN + 1];
  __shared__ double inv[kDenseMaxN][kDenseMaxN + 1];
  __shared__ double fct[kDenseMaxN];
  __shared__ double norm;
  __shared__ int piv, sing;
  const int r = blockIdx.x;
  const int t = threadIdx.x;
  double *row = table + row_off[r];
  const DenseRowLayout L{n, F};
  for (int e = t; e < n * n; e += kDenseThreads) {
    const int i = e / n, j = e - (e / n) * n;
    a[i][j] = row[L.a_off() + e];
    inv[i][j] = (i == j) ? 1.0 : 0.0;
  }
  __syncthreads();
  if (t == 0) {
    double m = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) m = fmax(m, fabs(a[i][j]));
    norm = m;
    sing = 0;
  }
  __syncthreads();
  for (int col = 0; col < n; ++col) {
    if (t == 0) {
      int pv = col;
      for (int i = col + 1; i < n; ++i)
        if (fabs(a[i][col]) > fabs(a[pv][col])) pv = i;
      piv = pv;
      if (!(fabs(a[pv][col]) > 1e-300 * norm)) sing = 1;
    }
    __syncthreads();
    if (sing) break;
    if (piv != col) {
      for (int j = t; j < n; j += kDenseThreads) {
        double tmp = a[col][j];
        a[col][j] = a[piv][j];
        a[piv][j] = tmp;
        tmp = inv[col][j];
        inv[col][j] = inv[piv][j];
        inv[piv][j] = tmp;
      }
    }
    __syncthreads();
    const double rp = 1.0 / a[col][col];
    __syncthreads();
    for (int j = t; j < n; j += kDenseThreads) {
      a[col][j] *= rp;
      inv[col][j] *= rp;
    }
    __syncthreads();
    for (int i = t; i < n; i += kDenseThreads) fct[i] = (i == col) ? 0.0 : a[i][col];
    __syncthreads();
    for (int e = t; e < n * n; e += kDenseThreads) {
      const int i = e / n, j = e - (e / n) * n;
      if (i == col) continue;
      a[i][j] = fma(-fct[i], a[col][j], a[i][j]);
      inv[i][j] = fma(-fct[i], inv[col][j], inv[i][j]);
    }
    __syncthreads();
  }
  if (t == 0) flags[r] = sing;
  if (sing) return;
  const DenseDesc &d = descs[row_desc[r]];
  for (int e = t; e < n * n; e += kDenseThreads) {
    const int i = e / n, j = e - (e / n) * n;
    double acc = 0.0;
    for (int k = 0; k < n; ++k) acc = fma(inv[i][k], row[L.b_off() + (int64_t)k * n + j], acc);
    row[e] = acc;                       // M = Ainv B
    row[L.ai_off() + e] = inv[i][j];    // Ainv
  }
  for (int e = t; e < 3 * n * F; e += kDenseThreads) {
    const int ax = e / (n * F);
    const int rem = e - ax * n * F;
    const int i = rem / F, tt = rem - (rem / F) * F;
    const double c = c0[3 * r + ax];
    row[L.g(ax) + (int64_t)i * F + tt] = (c == 0.0) ? 0.0 : c * inv[i][d.face_q[ax][tt]];
  }
}

// downwind-local node index of face node t on the face q_a = qa of axis a
template <int NP, int DIM>
__device__ constexpr int face_node(int a, int t, int qa) {
  int q = 0, stride = 1, rem = t;
  for (int b = 0; b < DIM; ++b) {
    int qb = 0;
    if (b == a) {
      qb = qa;
    } else {
      qb = rem % NP;
      rem /= NP;
    }
    q += qb * stride;
    stride *= NP;
  }
  return q;
}

// Cross-tile hand-off.  A tile's inflow traces are written by its upwind
// tiles, which may run on another XCD (each XCD has its own L2).  Every trace
// value is written once per sweep, into a slot that was filled with a
// signalling-NaN sentinel before the launch; arithmetic never produces a
// signalling NaN, so a slot that no longer holds the sentinel holds its final
// value.  Both sides use device-scope atomic read-modify-writes, which are
// performed at the device's point of coherence, so no cache-wide write-back or
// invalidation is needed and each cell waits only for its own upwind cell.
// Current content of a trace slot, read with a compare-and-swap that writes
// the sentinel back only where it already is (an idempotent or-with-zero
// would be turned into a plain load by the compiler).
__device__ inline uint64_t dense_peek_trace(uint64_t *p) {
  uint64_t cur = kDenseTraceEmpty;
  __hip_atomic_compare_exchange_strong(p, &cur, kDenseTraceEmpty, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                       __HIP_MEMORY_SCOPE_AGENT);
  return cur;
}

// The inflow traces a cell needs from upwind tiles (up to one face per axis).
// Every slot is requested at once, so a ready face costs one round trip; the
// slots still empty are polled again after a short sleep.  The producer was
// claimed earlier and is resident, so the wait ends; the wall-clock bound
// (1 s at the 100 MHz constant clock) and the shared error flag turn a logic
// error into one reported failure instead of a hang.
template <int DIM, int F>
__device__ inline void dense_take_faces(uint64_t *const (&src)[DIM], uint64_t (&b)[DIM][F], int32_t *err_flag) {
  bool ready = true;
#pragma unroll
  for (int a = 0; a < DIM; ++a)
    if (src[a])
#pragma unroll
      for (int tt = 0; tt < F; ++tt) b[a][tt] = dense_peek_trace(src[a] + tt);
#pragma unroll
  for (int a = 0; a < DIM; ++a)
    if (src[a])
#pragma unroll
      for (int tt = 0; tt < F; ++tt) ready = ready && b[a][tt] != kDenseTraceEmpty;
  if (ready) return;
  const uint64_t t_start = wall_clock64();
  for (;;) {
    __builtin_amdgcn_s_sleep(2);
    ready = true;
#pragma unroll
    for (int a = 0; a < DIM; ++a)
      if (src[a])
#pragma unroll
        for (int tt = 0; tt < F; ++tt)
          if (b[a][tt] == kDenseTraceEmpty) b[a][tt] = dense_peek_trace(src[a] + tt);
#pragma unroll
    for (int a = 0; a < DIM; ++a)
      if (src[a])
#pragma unroll
        for (int tt = 0; tt < F; ++tt) ready = ready && b[a][tt] != kDenseTraceEmpty;
    if (ready) return;
    if (wall_clock64() - t_start > 100000000ull ||
        __hip_atomic_load(err_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
      __hip_atomic_fetch_or(err_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
#pragma unroll
      for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int tt = 0; tt < F; ++tt)
          if (b[a][tt] == kDenseTraceEmpty) b[a][tt] = 0;
      return;
    }
  }
}

__device__ inline void dense_put_trace(uint64_t *p, double v) {
  __hip_atomic_exchange(p, (uint64_t)__double_as_longlong(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// One wave per tile, in one of two schedules:
// * claimed (LEVEL = false): one launch for all tiles.  The tile index is
//   claimed by lane 0 from a counter that hands out tiles in dependency order
//   (upwind tiles first) and broadcast with readfirstlane, so it is
//   wave-uniform; inflow traces arrive through the atomic slots above, cell by
//   cell, so a tile starts as soon as its first upwind cells are done.
// * levelled (LEVEL = true): one launch per tile diagonal; the launch's tiles
//   are order[0 .. n_tiles).  Upwind tiles belong to earlier launches, whose
//   writes the kernel boundary makes visible: plain loads and stores, no
//   waiting.
// Either way descriptors and operator rows are read through scalar loads and
// all control flow that depends on the tile is uniform.  Inside the tile the
// cells are solved diagonal by diagonal; the inflow traces of a cell come from
// the previous diagonal through LDS, from an upwind tile through the trace
// slots, or from the domain inflow data.
template <int PREC, int NP, int DIM, bool LEVEL>
__global__ __launch_bounds__(kDenseThreads) void dense_sweep_kernel(
    const DenseTile *__restrict__ tiles, const int32_t *__restrict__ order, const DenseFam *__restrict__ fams,
    const DenseDesc *__restrict__ descs, const double *__restrict__ table, int dt_idx,
    typename Pol<PREC>::St *__restrict__ f, const double *__restrict__ fb_old, const double *__restrict__ fb_new,
    uint64_t *traces, int32_t *counter, int32_t *err_flag, int n_tiles) {
  static_assert(kDenseThreads == 64, "one workgroup is one wave");
  using St = typename Pol<PREC>::St;
  using Rt = typename Pol<PREC>::Rt;
  constexpr int N = DIM == 2 ? NP * NP : NP * NP * NP;
  constexpr int F = DIM == 2 ? NP : NP * NP;
  __shared__ Rt otr[3][kDenseThreads][F];  // outflow traces per axis of every cell of the tile
  const int t = threadIdx.x;
  int claim = blockIdx.x;
  if (!LEVEL) {
    if (t == 0) claim = atomicAdd(counter, 1);
    claim = __builtin_amdgcn_readfirstlane(claim);
    if (claim >= n_tiles) {  // the counter was not reset: report, do nothing
      if (t == 0) __hip_atomic_fetch_or(err_flag, 2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return;
    }
  }
  const int tile = order[claim];
  const DenseTile tl = tiles[tile];
  const DenseFam fm = fams[tl.fam];
  const DenseDesc &d = descs[fm.desc];

  // this thread's cell: local coordinates over the non-zero components
  int cl[3] = {0, 0, 0}, tstride[3] = {0, 0, 0};
  int rem = t, st_acc = 1;
  bool active = true;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    if (d.sgn[a] == 0) continue;
    cl[a] = rem % d.T[a];
    rem /= d.T[a];
    tstride[a] = st_acc;
    st_acc *= d.T[a];
  }
  if (rem != 0) active = false;
  int x[3] = {0, 0, 0};
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    if (d.sgn[a] == 0) {
      x[a] = (a == d.trans_axis) ? fm.slice : 0;
    } else {
      const int p = tl.tc[a] * d.T[a] + cl[a];
      if (p >= d.n[a]) active = false;
      x[a] = d.sgn[a] > 0 ? p : d.n[a] - 1 - p;
    }
  }
  const int64_t cell = x[0] + (int64_t)d.n[0] * (x[1] + (int64_t)d.n[1] * x[2]);
  const double *row = table + d.op_off + (int64_t)dt_idx * d.op_stride;
  const DenseRowLayout L{N, F};

  // load the cell and apply the local block
  Rt fv[N], y[N];
#pragma unroll
  for (int q = 0; q < N; ++q) fv[q] = active ? (Rt)ld_state(f + fm.f_base + d.plane_off[q] + cell) : (Rt)0;
  if (PREC == kRefine) {
    double r[N];
    float r32[N], y1[N];
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double acc = 0.0;
#pragma unroll
      for (int j = 0; j < N; ++j) acc = fma(row[L.b_off() + i * N + j], (double)fv[j], acc);
      r[i] = acc;
      r32[i] = (float)acc;
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      float acc = 0.f;
#pragma unroll
      for (int j = 0; j < N; ++j) acc = fmaf((float)row[L.ai_off() + i * N + j], r32[j], acc);
      y1[i] = acc;
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      double acc = r[i];
#pragma unroll
      for (int j = 0; j < N; ++j) acc = fma(-row[L.a_off() + i * N + j], (double)y1[j], acc);
      r32[i] = (float)acc;
    }
#pragma unroll
    for (int i = 0; i < N; ++i) {
      float acc = 0.f;
#pragma unroll
      for (int j = 0; j < N; ++j) acc = fmaf((float)row[L.ai_off() + i * N + j], r32[j], acc);
      y[i] = (Rt)((double)y1[i] + (double)acc);
    }
  } else {
#pragma unroll
    for (int i = 0; i < N; ++i) {
      Rt acc = 0;
#pragma unroll
      for (int j = 0; j < N; ++j) acc = fma((Rt)row[i * N + j], fv[j], acc);
      y[i] = acc;
    }
  }
  const Rt th = (Rt)d.theta;
  const Rt omt = (Rt)1 - th;

  int diag = 0, ndiag = 1;
#pragma unroll
  for (int a = 0; a < DIM; ++a)
    if (d.sgn[a] != 0) {
      diag += cl[a];
      ndiag += d.T[a] - 1;
    }
  // Inflow data of the faces that are not fed from inside the tile: domain
  // inflow (always ready), or, in the levelled schedule, the traces of an
  // upwind tile of an earlier launch.  Both are fetched before the diagonal
  // loop, so that the loop issues no global load it would have to wait for.
  Rt uin[DIM][F];
  uint64_t *rsrc[DIM];
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    rsrc[a] = nullptr;
#pragma unroll
    for (int tt = 0; tt < F; ++tt) uin[a][tt] = (Rt)0;
    if (!active || d.sgn[a] == 0 || cl[a] > 0) continue;
    if (tl.up[a] >= 0) {
      // face cell index of this cell on faces normal to a (tile-local)
      int fc = 0, fs = 1;
#pragma unroll
      for (int b = 0; b < DIM; ++b)
        if (b != a && d.sgn[b] != 0) {
          fc += cl[b] * fs;
          fs *= d.T[b];
        }
      rsrc[a] = traces + tl.trace_off + (int64_t)a * tl.slot + fc * F;
      if (LEVEL)
#pragma unroll
        for (int tt = 0; tt < F; ++tt) uin[a][tt] = (Rt)__longlong_as_double((long long)rsrc[a][tt]);
    } else {
      // domain inflow face: transverse cell index over the other axes
      int64_t tau = 0, ts = 1;
#pragma unroll
      for (int b = 0; b < DIM; ++b)
        if (b != a) {
          tau += x[b] * ts;
          ts *= d.n[b];
        }
      const int64_t base = fm.fb_base + d.fb_axis_off[a] + tau;
#pragma unroll
      for (int tt = 0; tt < F; ++tt) {
        const int64_t k = base + (int64_t)d.fb_t[a][tt] * d.fb_ntc[a];
        uin[a][tt] = th * (Rt)fb_new[k] + omt * (Rt)fb_old[k];
      }
    }
  }

  for (int s = 0; s < ndiag; ++s) {
    if (active && diag == s) {
      if (!LEVEL) {
        uint64_t rb[DIM][F];
        dense_take_faces<DIM, F>(rsrc, rb, err_flag);
#pragma unroll
        for (int a = 0; a < DIM; ++a)
          if (rsrc[a])
#pragma unroll
            for (int tt = 0; tt < F; ++tt) uin[a][tt] = (Rt)__longlong_as_double((long long)rb[a][tt]);
      }
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        if (d.sgn[a] == 0) continue;
        Rt u[F];
        if (cl[a] > 0) {
#pragma unroll
          for (int tt = 0; tt < F; ++tt) u[tt] = otr[a][t - tstride[a]][tt];
        } else {
#pragma unroll
          for (int tt = 0; tt < F; ++tt) u[tt] = uin[a][tt];
        }
#pragma unroll
        for (int i = 0; i < N; ++i) {
          Rt acc = y[i];
#pragma unroll
          for (int tt = 0; tt < F; ++tt) acc = fma((Rt)row[L.g(a) + i * F + tt], u[tt], acc);
          y[i] = acc;
        }
      }
#pragma unroll
      for (int q = 0; q < N; ++q) st_state(f + fm.f_base + d.plane_off[q] + cell, (St)y[q]);
      // outflow traces: theta x + (1 - theta) f^n on each downwind face
#pragma unroll
      for (int b = 0; b < DIM; ++b) {
        if (d.sgn[b] == 0) continue;
        int fc = 0, fs = 1;
#pragma unroll
        for (int a2 = 0; a2 < DIM; ++a2)
          if (a2 != b && d.sgn[a2] != 0) {
            fc += cl[a2] * fs;
            fs *= d.T[a2];
          }
        const bool to_next = cl[b] == d.T[b] - 1 && tl.down[b] >= 0;
        uint64_t *dst = nullptr;
        if (to_next) {
          const DenseTile &dn = tiles[tl.down[b]];
          dst = traces + dn.trace_off + (int64_t)b * dn.slot + fc * F;
        }
#pragma unroll
        for (int tt = 0; tt < F; ++tt) {
          const int q = face_node<NP, DIM>(b, tt, NP - 1);
          const Rt o = th * y[q] + omt * fv[q];
          otr[b][t][tt] = o;
          if (to_next) {
            if (LEVEL)
              dst[tt] = (uint64_t)__double_as_longlong((double)o);
            else
              dense_put_trace(dst + tt, (double)o);
          }
        }
      }
    }
    // The next diagonal reads this one's outflow traces from LDS.  The
    // workgroup is a single wave, whose LDS accesses execute in order, so
    // only the compiler has to be kept from moving them across the step;
    // global stores stay in flight (a workgroup barrier would wait for them).
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
  }
}

__global__ void fill_int_kernel(int32_t *p, int64_t n, int32_t value) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

__global__ void fill_u64_kernel(uint64_t *p, int64_t n, uint64_t value) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

// ---------------------------------------------------------------------------
// dispatch
// ---------------------------------------------------------------------------
template <int PREC, int NP>
hipError_t go_sweep(const SweepItem *items, int n_items, const SweepDesc *descs, const OpEntry *ops,
                    int dt_idx, void *f, const double *fb_old, const double *fb_new, double *stats,
                    hipStream_t st) {
  using St = typename Pol<PREC>::St;
  constexpr int SMAX = sweep_smax(NP);
  hipLaunchKernelGGL((sweep_kernel<PREC, NP, SMAX>), dim3(n_items), dim3(kBlock), 0, st, items, descs, ops,
                     dt_idx, static_cast<St *>(f), fb_old, fb_new, stats);
  return hipGetLastError();
}

template <int PREC>
hipError_t go_sweep_np(int np, const SweepItem *items, int n_items, const SweepDesc *descs,
                       const OpEntry *ops, int dt_idx, void *f, const double *fb_old, const double *fb_new,
                       double *stats, hipStream_t st) {
  switch (np) {
    case 2: return go_sweep<PREC, 2>(items, n_items, descs, ops, dt_idx, f, fb_old, fb_new, stats, st);
    case 3: return go_sweep<PREC, 3>(items, n_items, descs, ops, dt_idx, f, fb_old, fb_new, stats, st);
    case 4: return go_sweep<PREC, 4>(items, n_items, descs, ops, dt_idx, f, fb_old, fb_new, stats, st);
    case 5: return go_sweep<PREC, 5>(items, n_items, descs, ops, dt_idx, f, fb_old, fb_new, stats, st);
    default: return hipErrorInvalidValue;
  }
}

template <int PREC, int NV>
hipError_t go_relax_m(int m, const RelaxItem *items, int n_items, const RelaxDesc *descs, void *f, double *w_out,
                      const double *w_in, double omega, int mode, hipStream_t st) {
  using St = typename Pol<PREC>::St;
  St *fp = static_cast<St *>(f);
  switch (m) {
#define PDG_RELAX_CASE(MM)                                                                                   \
  case MM:                                                                                                   \
    hipLaunchKernelGGL((relax_kernel<PREC, NV, MM>), dim3(n_items), dim3(kBlock), 0, st, items, descs, fp, \
                       w_out, w_in, omega, mode);                                                            \
    return hipGetLastError();
    PDG_RELAX_CASE(1)
    PDG_RELAX_CASE(2)
    PDG_RELAX_CASE(3)
    PDG_RELAX_CASE(4)
    PDG_RELAX_CASE(5)
    PDG_RELAX_CASE(6)
    PDG_RELAX_CASE(7)
    PDG_RELAX_CASE(8)
#undef PDG_RELAX_CASE
    default: return hipErrorInvalidValue;
  }
}

template <int NV>
hipError_t go_inflow_m(int m, const InflowDesc *items, int n_items, const RelaxDesc *descs, const double *w_in,
                       double *fb, hipStream_t st) {
  const dim3 grid(64, n_items);
  switch (m) {
#define PDG_INFLOW_CASE(MM)                                                                                      \
  case MM:                                                                                                       \
    hipLaunchKernelGGL((inflow_eq_kernel<NV, MM>), grid, dim3(kBlock), 0, st, items, descs, w_in, fb);        \
    return hipGetLastError();
    PDG_INFLOW_CASE(1)
    PDG_INFLOW_CASE(2)
    PDG_INFLOW_CASE(3)
    PDG_INFLOW_CASE(4)
    PDG_INFLOW_CASE(5)
    PDG_INFLOW_CASE(6)
    PDG_INFLOW_CASE(7)
    PDG_INFLOW_CASE(8)
#undef PDG_INFLOW_CASE
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_invert(OpEntry *ops, int n_ops, hipStream_t st) {
  if (n_ops <= 0) return hipSuccess;
  hipLaunchKernelGGL(invert_kernel, dim3((n_ops + 63) / 64), dim3(64), 0, st, ops, n_ops);
  return hipGetLastError();
}

hipError_t launch_sweep(int prec, int np, const SweepItem *items, int n_items,
                        const SweepDesc *descs, const OpEntry *ops, int dt_idx, void *f, const double *fb_old,
                        const double *fb_new, double *stats, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  switch (prec) {
    case kF64: return go_sweep_np<kF64>(np, items, n_items, descs, ops, dt_idx, f, fb_old, fb_new, stats, st);
    case kF32: return go_sweep_np<kF32>(np, items, n_items, descs, ops, dt_idx, f, fb_old, fb_new, stats, st);
    case kRefine: return go_sweep_np<kRefine>(np, items, n_items, descs, ops, dt_idx, f, fb_old, fb_new, stats, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_relax(int prec, int nv, int m, const RelaxItem *items, int n_items, const RelaxDesc *descs,
                        void *f, double *w_out, const double *w_in, double omega, int mode, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
#define PDG_RELAX_NV(PR)                                                                            \
  switch (nv) {                                                                                     \
    case 4: return go_relax_m<PR, 4>(m, items, n_items, descs, f, w_out, w_in, omega, mode, st);    \
    case 6: return go_relax_m<PR, 6>(m, items, n_items, descs, f, w_out, w_in, omega, mode, st);    \
    default: return hipErrorInvalidValue;                                                           \
  }
  switch (prec) {
    case kF64: PDG_RELAX_NV(kF64)
    case kF32: PDG_RELAX_NV(kF32)
    case kRefine: PDG_RELAX_NV(kRefine)
    default: return hipErrorInvalidValue;
  }
#undef PDG_RELAX_NV
}

hipError_t launch_inflow_eq(int nv, int m, const InflowDesc *items, int n_items, const RelaxDesc *descs,
                            const double *w_inflow, double *fb, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  switch (nv) {
    case 4: return go_inflow_m<4>(m, items, n_items, descs, w_inflow, fb, st);
    case 6: return go_inflow_m<6>(m, items, n_items, descs, w_inflow, fb, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_fill_int(int32_t *p, int64_t n, int32_t value, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>(1024, (n + 255) / 256);
  hipLaunchKernelGGL(fill_int_kernel, dim3(grid), dim3(256), 0, st, p, n, value);
  return hipGetLastError();
}

hipError_t launch_fill_u64(uint64_t *p, int64_t n, uint64_t value, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  const int grid = (int)std::min<int64_t>(1024, (n + 255) / 256);
  hipLaunchKernelGGL(fill_u64_kernel, dim3(grid), dim3(256), 0, st, p, n, value);
  return hipGetLastError();
}

hipError_t launch_dense_invert(double *table, const int64_t *row_off, const DenseDesc *descs,
                               const int32_t *row_desc, const double *c0, int32_t *flags, int n_rows, int n,
                               int F, hipStream_t st) {
  if (n_rows <= 0) return hipSuccess;
  if (n > kDenseMaxN || F > kDenseMaxF) return hipErrorInvalidValue;
  hipLaunchKernelGGL(dense_invert_kernel, dim3(n_rows), dim3(kDenseThreads), 0, st, table, row_off, descs, row_desc,
                     c0, flags, n, F);
  return hipGetLastError();
}

template <int PREC, int NP, int DIM>
hipError_t go_dense(bool level, const DenseTile *tiles, const int32_t *order, int n_tiles, const DenseFam *fams,
                    const DenseDesc *descs, const double *table, int dt_idx, void *f, const double *fb_old,
                    const double *fb_new, uint64_t *traces, int32_t *counter, int32_t *err, hipStream_t st) {
  using St = typename Pol<PREC>::St;
  if (level)
    hipLaunchKernelGGL((dense_sweep_kernel<PREC, NP, DIM, true>), dim3(n_tiles), dim3(kDenseThreads), 0, st, tiles,
                       order, fams, descs, table, dt_idx, static_cast<St *>(f), fb_old, fb_new, traces, counter, err,
                       n_tiles);
  else
    hipLaunchKernelGGL((dense_sweep_kernel<PREC, NP, DIM, false>), dim3(n_tiles), dim3(kDenseThreads), 0, st, tiles,
                       order, fams, descs, table, dt_idx, static_cast<St *>(f), fb_old, fb_new, traces, counter, err,
                       n_tiles);
  return hipGetLastError();
}

template <int PREC>
hipError_t go_dense_shape(bool level, int np, int dim, const DenseTile *tiles, const int32_t *order, int n_tiles,
                          const DenseFam *fams, const DenseDesc *descs, const double *table, int dt_idx, void *f,
                          const double *fb_old, const double *fb_new, uint64_t *traces, int32_t *counter,
                          int32_t *err, hipStream_t st) {
#define PDG_DENSE_CASE(NPV, DIMV)                                                                             \
  if (np == NPV && dim == DIMV)                                                                               \
    return go_dense<PREC, NPV, DIMV>(level, tiles, order, n_tiles, fams, descs, table, dt_idx, f, fb_old, fb_new,   \
                                     traces, counter, err, st);
  PDG_DENSE_CASE(2, 2)
  PDG_DENSE_CASE(3, 2)
  PDG_DENSE_CASE(4, 2)
  PDG_DENSE_CASE(5, 2)
  PDG_DENSE_CASE(2, 3)
  PDG_DENSE_CASE(3, 3)
#undef PDG_DENSE_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_dense_sweep(int prec, bool level, int np, int dim, const DenseTile *tiles, const int32_t *order,
                              int n_tiles, const DenseFam *fams, const DenseDesc *descs, const double *table,
                              int dt_idx, void *f, const double *fb_old, const double *fb_new, uint64_t *traces,
                              int32_t *counter, int32_t *err_flag, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  switch (prec) {
    case kF64: return go_dense_shape<kF64>(level, np, dim, tiles, order, n_tiles, fams, descs, table, dt_idx, f, fb_old, fb_new, traces, counter, err_flag, st);
    case kF32: return go_dense_shape<kF32>(level, np, dim, tiles, order, n_tiles, fams, descs, table, dt_idx, f, fb_old, fb_new, traces, counter, err_flag, st);
    case kRefine: return go_dense_shape<kRefine>(level, np, dim, tiles, order, n_tiles, fams, descs, table, dt_idx, f, fb_old, fb_new, traces, counter, err_flag, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_lattice(int prec, const RelaxItem *items, int n_items, const RelaxDesc *descs, void *f,
                          double *w_out, const double *w_in, double omega, double h_pre, double h_post, int mode,
                          hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  switch (prec) {
    case kF64:
      hipLaunchKernelGGL(lattice_kernel<kF64>, dim3(n_items), dim3(kBlock), 0, st, items, descs,
                         static_cast<double *>(f), w_out, w_in, omega, h_pre, h_post, mode);
      break;
    case kF32:
      hipLaunchKernelGGL(lattice_kernel<kF32>, dim3(n_items), dim3(kBlock), 0, st, items, descs,
                         static_cast<float *>(f), w_out, w_in, omega, h_pre, h_post, mode);
      break;
    case kRefine:
      hipLaunchKernelGGL(lattice_kernel<kRefine>, dim3(n_items), dim3(kBlock), 0, st, items, descs,
                         static_cast<double *>(f), w_out, w_in, omega, h_pre, h_post, mode);
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_lattice_inflow(const InflowDesc *items, int n_items, const RelaxDesc *descs, const double *w_in,
                                 double *fb, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(lattice_inflow_kernel, dim3(64, n_items), dim3(kBlock), 0, st, items, descs, w_in, fb);
  return hipGetLastError();
}

hipError_t launch_fill(double *p, int64_t n, double value, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(256), dim3(256), 0, st, p, n, value);
  return hipGetLastError();
}

}  // namespace pdg
