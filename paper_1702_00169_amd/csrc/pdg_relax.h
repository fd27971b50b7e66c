// Node-local arithmetic of the relaxation for the {+-lambda e_k} velocity
// sets (eq. collision_cn, Sec. 4.4), shared by the relaxation kernel and the
// fused relaxation + sweep kernel.
#pragma once

#include "pdg_device.h"

namespace pdg {
namespace {

// Moments w_k = sum_i f_{i,k}: Neumaier compensated sum over the velocities
// in a fixed order.
template <int NV, int M>
__device__ inline void moments(const double (&fv)[NV][M], double (&w)[M]) {
#pragma unroll
  for (int k = 0; k < M; ++k) {
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
}

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

}  // namespace
}  // namespace pdg
