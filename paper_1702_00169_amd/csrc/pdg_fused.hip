// gfx950 kernel of the fused collision + x transport: one pass over the
// state that relaxes every node (eq. collision_cn, Sec. 4.4) and solves the
// chains of the two velocities along the contiguous axis (Sec. 4.1-4.2) on
// the relaxed values while they are still in registers.
//
// In the step C T(dt) C T(dt) .. every collision is followed by a transport,
// and the velocities along x are transported on rows that are contiguous in
// memory, the same rows a node-parallel collision reads.  One thread per
// (cell of a row, transverse node) loads the n_v m values of each of its d+1
// nodes along x, forms the moments and the relaxed values, writes back the
// relaxed values of the velocities along the other axes (their chains run in
// the following y / z sweep), and keeps those of +x and -x for the row's two
// chain solves: the cell block x_l = M f_l + g u_l and the inflow recurrence
// u_{l+1} = a u_l + beta_l as a segmented scan over the row, forward for +x
// and backward for -x.  Per step the state is then read and written once by
// this pass and once more only for the velocities along y and z.

#include "pdg_cellop.h"
#include "pdg_device.h"
#include "pdg_relax.h"

namespace pdg {
namespace {

// Threads of a row's workgroup at most: (d+1) blocks of the row length
// rounded up to a wave.  Two waves per SIMD leave each thread the registers
// for all n_v m values of its node.
constexpr int kFusedMaxThreads = 512;

// Component passes of one direction at most: ceil(m / (d+1)) over the
// supported (d+1, m).
constexpr int kFusedKB = 3;

// Inclusive scans of I_l = a I_{l-1} + beta_l along one row, KB of them at
// once (the component passes of one direction: their shuffles interleave and
// they share one barrier), held by the threads of a block (one cell per
// thread, NW waves, cell x at lane x of the block).  DIR = +1 scans with
// increasing x (chain position l = x), DIR = -1 with decreasing x
// (l = nx - 1 - x); padding lanes past the row's end carry l = 0 and
// beta = 0, so they never feed a cell of the row.  apow[s] = a^(2^s),
// alane = a^(k + 1) with k the thread's distance from the wave edge it scans
// from.  I receives the scans of beta; prev the I of the upwind neighbour
// (or the carry into the wave for the wave's first element).  Every thread
// of the workgroup calls it (it synchronises the workgroup once).
template <class Rt, int DIR, int KB>
__device__ __forceinline__ void row_scan(const Rt (&beta)[KB], int l, const Rt (&apow)[7], Rt alane,
                                         Rt (*wtot)[kFusedKB][kFusedMaxThreads / 64], int nwb, int par,
                                         Rt (&I)[KB], Rt (&prev)[KB]) {
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  const int b0 = (wv / nwb) * nwb;           // first wave of this thread's block
  const int k = DIR > 0 ? lane : 63 - lane;  // elements before this one in scan order within the wave
  const int kw = l < k ? l : k;              // of them, those in the row
#pragma unroll
  for (int j = 0; j < KB; ++j) I[j] = beta[j];
#pragma unroll
  for (int s = 0; s < 6; ++s) {
    const int dd = 1 << s;
#pragma unroll
    for (int j = 0; j < KB; ++j) {
      const Rt up = DIR > 0 ? __shfl_up(I[j], dd, 64) : __shfl_down(I[j], dd, 64);
      if (kw >= dd) I[j] = fma(apow[s], up, I[j]);
    }
  }
  if (k == 63) {  // the wave's totals (a full wave of the row: l >= 63 here)
#pragma unroll
    for (int j = 0; j < KB; ++j) wtot[par][j][wv] = I[j];
  }
  __syncthreads();
  // carry into this wave: the totals of the block's waves before it in scan
  // order, each a full wave of the row
  const int wi = wv - b0;
  const int nbefore = DIR > 0 ? wi : nwb - 1 - wi;
#pragma unroll
  for (int j = 0; j < KB; ++j) {
    Rt cin = 0;
    for (int i = 0; i < nbefore; ++i) {
      const int w = DIR > 0 ? b0 + i : b0 + nwb - 1 - i;
      cin = fma(apow[6], cin, wtot[par][j][w]);
    }
    if (l > k) I[j] = fma(alane, cin, I[j]);
    const Rt nb = DIR > 0 ? __shfl_up(I[j], 1, 64) : __shfl_down(I[j], 1, 64);
    prev[j] = k > 0 ? nb : cin;
  }
}

// One workgroup per row of cells (instance, transverse node jt, row tau) and
// NP blocks of nxp = nx rounded up to 64 threads: thread (block jx, lane x)
// owns node jx of cell x.  The relaxed values of +x and -x go to LDS
// (dynamic shared memory: 2 M NP nxp values); then block b solves the chains
// of components k = b, b + NP, .. for +x and then for -x.
template <int PREC, int NP, int NV, int M>
__global__ __launch_bounds__(kFusedMaxThreads) void relax_xsweep_kernel(
    const FusedItem *__restrict__ items, const FusedDesc *__restrict__ fdescs,
    const RelaxDesc *__restrict__ rdescs, const OpEntry *__restrict__ ops, int dt_idx, const State<PREC> f,
    const double *__restrict__ fb_old, const double *__restrict__ fb_new, double omega,
    double *__restrict__ stats) {
  using Rt = typename Pol<PREC>::Rt;
  extern __shared__ __align__(16) unsigned char fused_lds[];
  __shared__ Rt wtot[2][kFusedKB][kFusedMaxThreads / 64];
  __shared__ double red[2][kFusedMaxThreads / 64];
  const FusedItem it = items[blockIdx.x];
  const FusedDesc fd = fdescs[it.desc];
  const RelaxDesc rd = rdescs[fd.rdesc];
  const int t = threadIdx.x;
  const int lane = t & 63, wv = t >> 6;
  const int nx = fd.nx;
  const int nxp = (nx + 63) & ~63;
  const int nwb = nxp >> 6;     // waves per block
  const int b = wv / nwb;       // block: node jx in the relaxation, component class in the transport
  const int x = t - b * nxp;    // cell of the row
  const bool cell_ok = x < nx;
  const int row = it.row0;
  const int jt = row / fd.ntau, tau = row - jt * fd.ntau;
  const int64_t cell = (int64_t)(cell_ok ? x : 0) + (int64_t)nx * tau;
  const int64_t nodes = rd.nodes;
  const int64_t fi = rd.f_base;
  const double inv_nv = 1.0 / NV;
  const double h2l = 0.5 / rd.lambda;
  Rt *fxl = reinterpret_cast<Rt *>(fused_lds);  // [h][k][jx][nxp]
  auto fx_at = [&](int h, int k, int jx) -> Rt & { return fxl[((h * M + k) * NP + jx) * nxp + x]; };

  // ---- collision at node (jx = b, jt) of cell x ----
  {
    // planes of the instance from scalar bases, nodes by 32-bit offsets
    uint32_t node = (uint32_t)((int64_t)(b + NP * jt) * fd.nc + cell);
    typename State<PREC>::Raw fr[NV][M];
#pragma unroll
    for (int i = 0; i < NV; ++i)
#pragma unroll
      for (int k = 0; k < M; ++k) fr[i][k] = f.at(fi + (int64_t)(i * M + k) * nodes).ldr32(node);
    double fv[NV][M];
#pragma unroll
    for (int i = 0; i < NV; ++i)
#pragma unroll
      for (int k = 0; k < M; ++k) fv[i][k] = (double)f.dec(fr[i][k]);
    double w[M];
    moments<NV, M>(fv, w);
    // The stores below recompute their addresses from here on: without this
    // the compiler keeps the 64-bit address of every load live until the
    // store to the same place, 2 n_v m registers more per thread.
    asm volatile("" : "+v"(node));
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      if (a >= rd.dim) break;
      double q[M];
      flux_dir<M>(rd, w, a, q);
#pragma unroll
      for (int i = 0; i < NV; ++i) {
        if (rd.axis[i] != a) continue;
        const double sg = rd.sign[i] * h2l;
#pragma unroll
        for (int k = 0; k < M; ++k) {
          const double fe = fma(sg, q[k], w[k] * inv_nv);
          const double nv = fma(omega, fe - fv[i][k], fv[i][k]);
          if (a == 0)
            fx_at(rd.sign[i] > 0 ? 0 : 1, k, b) = (Rt)nv;
          else if (cell_ok)
            f.at(fi + (int64_t)(i * M + k) * nodes).st32(node, nv);
        }
      }
    }
  }
  __syncthreads();

  // ---- the chains of +x and -x along the row ----
  double cmax = 0.0, ymax = 0.0;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    CellOp<PREC, NP> op;
    op.load(ops[fd.op[h] + dt_idx]);
    const Rt theta = op.theta;
    const Rt omt = (Rt)1 - theta;
    const Rt a = op.a;
    Rt apow[7];
    apow[0] = a;
#pragma unroll
    for (int s = 1; s < 7; ++s) apow[s] = apow[s - 1] * apow[s - 1];
    const int kk = h == 0 ? lane : 63 - lane;
    Rt alane = 1;
#pragma unroll
    for (int s = 0; s < 7; ++s)
      if ((kk + 1) & (1 << s)) alane *= apow[s];
    const int l = cell_ok ? (h == 0 ? x : nx - 1 - x) : 0;  // chain position; padding lanes start nothing
    const int v = fd.vx[h];
    constexpr int KB = (M + NP - 1) / NP;
    static_assert(KB <= kFusedKB, "component passes per direction");
    Rt y[KB][NP], beta[KB], ub[KB];
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      const int k = kb * NP + b;
      const bool on = cell_ok && k < M;
      Rt fl[NP];  // downwind-local order: node 0 receives the inflow
#pragma unroll
      for (int q = 0; q < NP; ++q) fl[q] = on ? fx_at(h, k, h == 0 ? q : NP - 1 - q) : (Rt)0;
      op.solve(fl, y[kb], cmax, ymax);
      beta[kb] = on ? theta * y[kb][NP - 1] + omt * fl[NP - 1] : (Rt)0;
      ub[kb] = 0;
      if (on && l == 0) {
        const int64_t bo = fd.fb[h] + ((int64_t)k * fd.tnodes + jt) * fd.ntau + tau;
        ub[kb] = theta * (Rt)fb_new[bo] + omt * (Rt)fb_old[bo];
        beta[kb] = fma(a, ub[kb], beta[kb]);
      }
    }
    Rt I[KB], prev[KB];
    if (h == 0)
      row_scan<Rt, 1, KB>(beta, l, apow, alane, wtot, nwb, h, I, prev);
    else
      row_scan<Rt, -1, KB>(beta, l, apow, alane, wtot, nwb, h, I, prev);
#pragma unroll
    for (int kb = 0; kb < KB; ++kb) {
      const int k = kb * NP + b;
      if (cell_ok && k < M) {
        const Rt u = l == 0 ? ub[kb] : prev[kb];
        const State<PREC> pv = f.at(fi + (int64_t)(v * M + k) * nodes);
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          const int jx = h == 0 ? q : NP - 1 - q;
          pv.st32((uint32_t)((int64_t)(jx + NP * jt) * fd.nc + cell), fma(op.g[q], u, y[kb][q]));
        }
      }
    }
  }

  // refinement statistics of the workgroup (largest correction, largest value)
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    cmax = fmax(cmax, __shfl_xor(cmax, off, 64));
    ymax = fmax(ymax, __shfl_xor(ymax, off, 64));
  }
  if (lane == 0) {
    red[0][wv] = cmax;
    red[1][wv] = ymax;
  }
  __syncthreads();
  if (t == 0) {
    double c = 0.0, y = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) {
      c = fmax(c, red[0][i]);
      y = fmax(y, red[1][i]);
    }
    stats[2 * (int64_t)blockIdx.x] = c;
    stats[2 * (int64_t)blockIdx.x + 1] = y;
  }
}

template <int PREC, int NP, int NV>
hipError_t go_fused_m(int m, int nx, const FusedItem *items, int n_items, const FusedDesc *fdescs,
                      const RelaxDesc *rdescs, const OpEntry *ops, int dt_idx, StateBuf f, const double *fb_old,
                      const double *fb_new, double omega, double *stats, hipStream_t st) {
  const State<PREC> fp = State<PREC>::make(f);
  const int nxp = (nx + 63) & ~63;
  using Rt = typename Pol<PREC>::Rt;
  switch (m) {
#define PDG_FUSED_CASE(MM)                                                                                     \
  case MM:                                                                                                     \
    hipLaunchKernelGGL((relax_xsweep_kernel<PREC, NP, NV, (MM)>), dim3(n_items), dim3(NP * nxp),              \
                       (size_t)2 * (MM) * NP * nxp * sizeof(Rt), st, items, fdescs, rdescs, ops, dt_idx, fp,    \
                       fb_old, fb_new, omega, stats);                                                          \
    return hipGetLastError();
    PDG_FUSED_CASE(1)
    PDG_FUSED_CASE(NV == 4 ? 4 : 5)  // the Euler model: m = D + 2
#undef PDG_FUSED_CASE
    default: return hipErrorInvalidValue;
  }
}

template <int PREC, int NP>
hipError_t go_fused_nv(int nv, int m, int nx, const FusedItem *items, int n_items, const FusedDesc *fdescs,
                       const RelaxDesc *rdescs, const OpEntry *ops, int dt_idx, StateBuf f, const double *fb_old,
                       const double *fb_new, double omega, double *stats, hipStream_t st) {
  switch (nv) {
    case 4: return go_fused_m<PREC, NP, 4>(m, nx, items, n_items, fdescs, rdescs, ops, dt_idx, f, fb_old, fb_new, omega, stats, st);
    case 6: return go_fused_m<PREC, NP, 6>(m, nx, items, n_items, fdescs, rdescs, ops, dt_idx, f, fb_old, fb_new, omega, stats, st);
    default: return hipErrorInvalidValue;
  }
}

template <int PREC>
hipError_t go_fused_np(int np, int nv, int m, int nx, const FusedItem *items, int n_items, const FusedDesc *fdescs,
                       const RelaxDesc *rdescs, const OpEntry *ops, int dt_idx, StateBuf f, const double *fb_old,
                       const double *fb_new, double omega, double *stats, hipStream_t st) {
  switch (np) {
    case 2: return go_fused_nv<PREC, 2>(nv, m, nx, items, n_items, fdescs, rdescs, ops, dt_idx, f, fb_old, fb_new, omega, stats, st);
    case 3: return go_fused_nv<PREC, 3>(nv, m, nx, items, n_items, fdescs, rdescs, ops, dt_idx, f, fb_old, fb_new, omega, stats, st);
    case 4: return go_fused_nv<PREC, 4>(nv, m, nx, items, n_items, fdescs, rdescs, ops, dt_idx, f, fb_old, fb_new, omega, stats, st);
    case 5: return go_fused_nv<PREC, 5>(nv, m, nx, items, n_items, fdescs, rdescs, ops, dt_idx, f, fb_old, fb_new, omega, stats, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

bool fused_supported(int np, int nv, int m, int nx) {
  return np >= 2 && np <= 5 && ((nv == 4 && (m == 1 || m == 4)) || (nv == 6 && (m == 1 || m == 5))) && nx >= 1 &&
         np * ((nx + 63) & ~63) <= kFusedMaxThreads;
}

hipError_t launch_relax_xsweep(int prec, int np, int nv, int m, int nx, const FusedItem *items, int n_items,
                               const FusedDesc *fdescs, const RelaxDesc *rdescs, const OpEntry *ops, int dt_idx,
                               StateBuf f, const double *fb_old, const double *fb_new, double omega, double *stats,
                               hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  if (!fused_supported(np, nv, m, nx)) return hipErrorInvalidValue;
  switch (prec) {
    case kF64: return go_fused_np<kF64>(np, nv, m, nx, items, n_items, fdescs, rdescs, ops, dt_idx, f, fb_old, fb_new, omega, stats, st);
    case kF32: return go_fused_np<kF32>(np, nv, m, nx, items, n_items, fdescs, rdescs, ops, dt_idx, f, fb_old, fb_new, omega, stats, st);
    case kRefine: return go_fused_np<kRefine>(np, nv, m, nx, items, n_items, fdescs, rdescs, ops, dt_idx, f, fb_old, fb_new, omega, stats, st);
    case kP48: return go_fused_np<kP48>(np, nv, m, nx, items, n_items, fdescs, rdescs, ops, dt_idx, f, fb_old, fb_new, omega, stats, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pdg
