// gfx950 node-local kernels: moments, equilibria, the collision update and
// the source step, and small fill kernels.
//
// Relaxation (eq. collision_cn, Sec. 4.4): one thread per node reads the nv x m
// values of that node (node-major layout: coalesced across threads), forms
// w with a compensated (Neumaier) sum in a fixed velocity order, evaluates
// f^eq(w) and applies f += omega (f^eq - f).

#include "pdg_device.h"
#include "pdg_relax.h"

namespace pdg {
namespace {

// ---------------------------------------------------------------------------
// equilibrium and relaxation
// ---------------------------------------------------------------------------
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
                                                      const State<PREC> f,
                                                      double *__restrict__ w_out,
                                                      const double *__restrict__ w_in, double omega, int mode) {
  const RelaxItem it = items[blockIdx.x];
  const RelaxDesc d = descs[it.desc];
  const int64_t nodes = d.nodes;
  const int64_t fi = d.f_base;
  const double inv_nv = 1.0 / NV;
  const double h2l = 0.5 / d.lambda;
  for (int64_t node0 = it.node0 + threadIdx.x; node0 < it.node0 + it.count; node0 += kBlock) {
    int64_t node = node0;
    double w[M];
    double fv[NV][M];
    if (mode == 0) {
#pragma unroll
      for (int i = 0; i < NV; ++i)
#pragma unroll
        for (int k = 0; k < M; ++k) fv[i][k] = (double)f.ld(fi + (int64_t)(i * M + k) * nodes + node);
      moments<NV, M>(fv, w);
      // 48-bit state: make the stores recompute their addresses, or the
      // compiler keeps the two 64-bit plane addresses of every load live
      // until the store to the same place (measured: fewer registers for
      // n_v m <= 20, more for the larger sets, so those keep the default)
      if constexpr (PREC == kP48 && NV * M <= 20) asm volatile("" : "+v"(node));
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
          f.st(fi + (int64_t)(i * M + k) * nodes + node, nv);
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
                                                        const State<PREC> f,
                                                        double *__restrict__ w_out, const double *__restrict__ w_in,
                                                        double omega, double h_pre, double h_post, int mode) {
  const RelaxItem it = items[blockIdx.x];
  const RelaxDesc d = descs[it.desc];
  const int64_t nodes = d.nodes;
  const int64_t fi = d.f_base;
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
      for (int i = 0; i < 9; ++i) fv[i] = (double)f.ld(fi + (int64_t)i * nodes + node);
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
        f.st(fi + (int64_t)i * nodes + node, lattice_feq(wt[i], d.cx[i], d.cy[i], rho, jx, jy, inv_l));
      continue;
    }
    if (source && h_pre != 0.0) lattice_source(d, fv, wt, rho, jx, jy, h_pre, inv_l);
#pragma unroll
    for (int i = 0; i < 9; ++i)
      fv[i] = fma(omega, lattice_feq(wt[i], d.cx[i], d.cy[i], rho, jx, jy, inv_l) - fv[i], fv[i]);
    if (source && h_post != 0.0) lattice_source(d, fv, wt, rho, jx, jy, h_post, inv_l);
#pragma unroll
    for (int i = 0; i < 9; ++i) f.st(fi + (int64_t)i * nodes + node, fv[i]);
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

__global__ void fill_int_kernel(int32_t *p, int64_t n, int32_t value) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

__global__ void fill_u64_kernel(uint64_t *p, int64_t n, uint64_t value) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = value;
}

// state <-> binary64 (to_f64: x = state; else state = x), grid-stride
template <int PREC>
__global__ __launch_bounds__(kBlock) void convert_kernel(const State<PREC> f, double *__restrict__ x, int64_t n,
                                                        int to_f64) {
  for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) {
    if (to_f64)
      x[i] = (double)f.ld(i);
    else
      f.st(i, (typename Pol<PREC>::Rt)x[i]);
  }
}

template <int PREC, int NV>
hipError_t go_relax_m(int m, const RelaxItem *items, int n_items, const RelaxDesc *descs, StateBuf f, double *w_out,
                      const double *w_in, double omega, int mode, hipStream_t st) {
  const State<PREC> fp = State<PREC>::make(f);
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

hipError_t launch_relax(int prec, int nv, int m, const RelaxItem *items, int n_items, const RelaxDesc *descs,
                        StateBuf f, double *w_out, const double *w_in, double omega, int mode, hipStream_t st) {
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
    case kP48: PDG_RELAX_NV(kP48)
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

hipError_t launch_lattice(int prec, const RelaxItem *items, int n_items, const RelaxDesc *descs, StateBuf f,
                          double *w_out, const double *w_in, double omega, double h_pre, double h_post, int mode,
                          hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
#define PDG_LATTICE_CASE(PR)                                                                                 \
  case PR:                                                                                                   \
    hipLaunchKernelGGL(lattice_kernel<PR>, dim3(n_items), dim3(kBlock), 0, st, items, descs,                 \
                       State<PR>::make(f), w_out, w_in, omega, h_pre, h_post, mode);                         \
    break;
  switch (prec) {
    PDG_LATTICE_CASE(kF64)
    PDG_LATTICE_CASE(kF32)
    PDG_LATTICE_CASE(kRefine)
    PDG_LATTICE_CASE(kP48)
    default: return hipErrorInvalidValue;
  }
#undef PDG_LATTICE_CASE
  return hipGetLastError();
}

hipError_t launch_lattice_inflow(const InflowDesc *items, int n_items, const RelaxDesc *descs, const double *w_in,
                                 double *fb, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  hipLaunchKernelGGL(lattice_inflow_kernel, dim3(64, n_items), dim3(kBlock), 0, st, items, descs, w_in, fb);
  return hipGetLastError();
}

hipError_t launch_convert(int prec, StateBuf f, double *x, bool to_f64, hipStream_t st) {
  if (f.n <= 0) return hipSuccess;
  const dim3 grid((unsigned)std::min<int64_t>(4096, (f.n + kBlock - 1) / kBlock));
#define PDG_CONVERT_CASE(PR)                                                                                 \
  case PR:                                                                                                   \
    hipLaunchKernelGGL(convert_kernel<PR>, grid, dim3(kBlock), 0, st, State<PR>::make(f), x, f.n, to_f64 ? 1 : 0); \
    break;
  switch (prec) {
    PDG_CONVERT_CASE(kF64)
    PDG_CONVERT_CASE(kF32)
    PDG_CONVERT_CASE(kRefine)
    PDG_CONVERT_CASE(kP48)
    default: return hipErrorInvalidValue;
  }
#undef PDG_CONVERT_CASE
  return hipGetLastError();
}

hipError_t launch_fill(double *p, int64_t n, double value, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_kernel, dim3(256), dim3(256), 0, st, p, n, value);
  return hipGetLastError();
}

}  // namespace pdg
