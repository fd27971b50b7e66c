// gfx950 kernels of the transport sweep for axis-aligned velocities.
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

#include "pdg_device.h"
#include "pdg_cellop.h"

namespace pdg {
namespace {

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
                                           const State<PREC> f,
                                           const double *__restrict__ fb_old, const double *__restrict__ fb_new,
                                           typename Pol<PREC>::Rt (*wtot)[4], int (*wopen)[4], double &cmax,
                                           double &ymax) {
  using Rt = typename Pol<PREC>::Rt;
  // 256-cell chunks whose loads are issued together: eight for cells of up
  // to three nodes (the registers allow it at the same occupancy), four above
#ifdef PDG_KCH
  constexpr int KCH = PDG_KCH;
#else
  constexpr int KCH = NP <= 3 ? 8 : 4;
#endif
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
    // issue the loads of KCH chunks before any of them is used (and before
    // any is converted to the arithmetic type)
    typename State<PREC>::Raw fr[KCH][NP];
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
      // lanes past the end load the item's first cell (always in bounds):
      // the loads stay unconditional, so they are all issued before any wait
      const int pis = valid ? pi : 0;
#pragma unroll
      for (int q = 0; q < NP; ++q) fr[k][q] = f.ldr(rowbase + q * d.plane_step + pis);
    }
#pragma unroll
    for (int k = 0; k < KCH; ++k, par ^= 1) {
      if (c0 + k * kBlock >= total) break;  // uniform across the block
      const bool valid = pidx[k] >= 0;
      const int l = pos[k];
      const int r = row[k];
      Rt fv[NP];
#pragma unroll
      for (int q = 0; q < NP; ++q) fv[q] = valid ? f.dec(fr[k][q]) : (Rt)0;
      Rt y[NP];
      op.solve(fv, y, cmax, ymax);
      const Rt fo = fv[NP - 1];
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
        for (int q = 0; q < NP; ++q) f.st(rowbase + q * d.plane_step + pidx[k], fma(op.g[q], u, y[q]));
      }
      carry = cw;
    }
  }
}

// One work item of the uniform-mesh sweep (chains of one family); the LDS
// buffers belong to the calling kernel, stats to this workgroup (2 doubles).
template <int PREC, int NP, int SMAX>
__device__ __forceinline__ void sweep_item(const SweepItem &it, const SweepDesc *__restrict__ descs,
                                           const OpEntry *__restrict__ ops, int dt_idx, const State<PREC> f,
                                           const double *__restrict__ fb_old, const double *__restrict__ fb_new,
                                           double *__restrict__ stats, typename Pol<PREC>::Rt (*xa)[kBlock],
                                           typename Pol<PREC>::Rt (*xb)[kBlock], typename Pol<PREC>::Rt (*wtot)[4],
                                           int (*wopen)[4]) {
  using Rt = typename Pol<PREC>::Rt;
  const SweepDesc d = descs[it.desc];
  CellOp<PREC, NP> op;
  op.load(ops[d.op + dt_idx]);
  const Rt theta = op.theta;
  const Rt omt = (Rt)1 - theta;

  const int t = threadIdx.x;
  double cmax = 0.0, ymax = 0.0;

  if (it.xk) {
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
  // inactive lanes address chain tau0 (in bounds) and cells past the chain
  // end address its last cell: every load is unconditional and in bounds,
  // and the values of those lanes and cells are never used
  const int tau = it.tau0 + (active ? c : 0);
  const int64_t chain = it.base + (int64_t)(tau % d.nx) + (int64_t)(tau / d.nx) * d.hi_stride + d.cell0 + d.plane0;
  int wpar = 0;
  for (int w0 = 0; w0 < n; w0 += window, wpar ^= 1) {
    const int lb = w0 + p * S;
    const int cnt = active ? max(0, min(S, n - lb)) : 0;
    Rt y[SMAX][NP];
    Rt fo[SMAX];
    typename State<PREC>::Raw fr[SMAX][NP];
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
      const int64_t cl = min(lb + s, n - 1);
#pragma unroll
      for (int q = 0; q < NP; ++q) fr[s][q] = f.ldr(chain + cl * d.cell_step + q * d.plane_step);
    }
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
      Rt fv[NP];
#pragma unroll
      for (int q = 0; q < NP; ++q) fv[q] = s < cnt ? f.dec(fr[s][q]) : (Rt)0;
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
          f.st(chain + (int64_t)(lb + s) * d.cell_step + q * d.plane_step, xv);
        }
        uu = theta * xo + omt * fo[s];
      }
    }
    u = unext;
  }

  }

  if (refine_prec(PREC)) {
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
      stats[0] = red[0];
      stats[1] = red[kBlock];
    }
  }
}

template <int PREC, int NP, int SMAX>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void sweep_kernel(
    const SweepItem *__restrict__ items, const SweepDesc *__restrict__ descs, const OpEntry *__restrict__ ops,
    int dt_idx, const State<PREC> f, const double *__restrict__ fb_old, const double *__restrict__ fb_new,
    double *__restrict__ stats) {
  using Rt = typename Pol<PREC>::Rt;
  __shared__ Rt xa[2][kBlock];
  __shared__ Rt xb[2][kBlock];
  __shared__ Rt wtot[2][4];
  __shared__ int wopen[2][4];
  sweep_item<PREC, NP, SMAX>(items[blockIdx.x], descs, ops, dt_idx, f, fb_old, fb_new, stats + 2 * (int64_t)blockIdx.x,
                             xa, xb, wtot, wopen);
}

// The items of every node count in one launch (batches of instances of
// different degrees): each workgroup dispatches on its item's node count, so
// the launch has one tail instead of one per node count.
template <int PREC>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3))) void sweep_mixed_kernel(
    const SweepItem *__restrict__ items, const SweepDesc *__restrict__ descs, const OpEntry *__restrict__ ops,
    int dt_idx, const State<PREC> f, const double *__restrict__ fb_old, const double *__restrict__ fb_new,
    double *__restrict__ stats) {
  using Rt = typename Pol<PREC>::Rt;
  __shared__ Rt xa[2][kBlock];
  __shared__ Rt xb[2][kBlock];
  __shared__ Rt wtot[2][4];
  __shared__ int wopen[2][4];
  const SweepItem it = items[blockIdx.x];
  double *st = stats + 2 * (int64_t)blockIdx.x;
  switch (ops[descs[it.desc].op].np) {
    case 2: sweep_item<PREC, 2, sweep_smax(2)>(it, descs, ops, dt_idx, f, fb_old, fb_new, st, xa, xb, wtot, wopen); break;
    case 3: sweep_item<PREC, 3, sweep_smax(3)>(it, descs, ops, dt_idx, f, fb_old, fb_new, st, xa, xb, wtot, wopen); break;
    case 4: sweep_item<PREC, 4, sweep_smax(4)>(it, descs, ops, dt_idx, f, fb_old, fb_new, st, xa, xb, wtot, wopen); break;
    default: sweep_item<PREC, 5, sweep_smax(5)>(it, descs, ops, dt_idx, f, fb_old, fb_new, st, xa, xb, wtot, wopen); break;
  }
}

// Chains on a graded axis: the cell size, and with it the cell operator,
// changes along the chain (operator row op + dt_idx * n_a + l for downwind
// position l).  Same thread mapping as the strided chains above -- thread
// (c, p) owns segment p of chain c, the segment maps are composed through
// LDS -- with each cell's own M, g and a: the segment map is
// u_out = (prod a_l) u_in + beta with beta_{l+1} = a_l beta_l + theta (M_l
// f_l)_out + (1 - theta) f_l,out.  Used for chains along any axis.  WPOS:
// C is a multiple of 64, so every wave sits at one chain position and reads
// the cell operators through scalar loads (they then take no vector
// registers, and more waves fit on a SIMD).
template <int PREC, int NP, int SMAX, bool WPOS>
__global__ __launch_bounds__(kBlock) void sweep_graded_kernel(const SweepItem *__restrict__ items,
                                                             const SweepDesc *__restrict__ descs,
                                                             const OpEntry *__restrict__ ops, int dt_idx,
                                                             const State<PREC> f,
                                                             const double *__restrict__ fb_old,
                                                             const double *__restrict__ fb_new,
                                                             double *__restrict__ stats) {
  using Rt = typename Pol<PREC>::Rt;
  __shared__ Rt xa[2][kBlock];
  __shared__ Rt xb[2][kBlock];
  const SweepItem it = items[blockIdx.x];
  const SweepDesc d = descs[it.desc];
  const OpEntry *row = ops + d.op + (int64_t)dt_idx * d.n_a;
  const Rt theta = (Rt)row[0].theta;
  const Rt omt = (Rt)1 - theta;
  const int t = threadIdx.x;
  double cmax = 0.0, ymax = 0.0;
  const int C = it.C;
  const int S = it.S;
  const int P = kBlock / C;
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
    // operator rows of the window's cells (the same for every lane of a wave
    // when WPOS)
    const int lbo = WPOS ? __builtin_amdgcn_readfirstlane(lb) : lb;
    const int cnto = max(0, min(S, n - lbo));
    Rt y[SMAX][NP], gs[SMAX][NP];
    Rt fo[SMAX], as[SMAX];
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
      Rt fv[NP];
      if (s < cnt) {
#pragma unroll
        for (int q = 0; q < NP; ++q) fv[q] = f.ld(chain + (int64_t)(lb + s) * d.cell_step + q * d.plane_step);
      } else {
#pragma unroll
        for (int q = 0; q < NP; ++q) fv[q] = 0;
      }
      fo[s] = fv[NP - 1];
      CellOp<PREC, NP> op;
      op.load(row[s < cnto ? lbo + s : 0]);
      op.solve(fv, y[s], cmax, ymax);
#pragma unroll
      for (int q = 0; q < NP; ++q) gs[s][q] = op.g[q];
      as[s] = op.a;
    }
    Rt alpha = 1, beta = 0;
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
      if (s < cnt) {
        beta = fma(as[s], beta, theta * y[s][NP - 1] + omt * fo[s]);
        alpha *= as[s];
      }
    }
    xa[wpar][t] = alpha;
    xb[wpar][t] = beta;
    __syncthreads();
    Rt uin = u;
    for (int q = 0; q < p; ++q) uin = fma(xa[wpar][c + C * q], uin, xb[wpar][c + C * q]);
    Rt unext = uin;
    for (int q = p; q < P; ++q) unext = fma(xa[wpar][c + C * q], unext, xb[wpar][c + C * q]);
    Rt uu = uin;
#pragma unroll
    for (int s = 0; s < SMAX; ++s) {
      if (s < cnt) {
        Rt xo = 0;
#pragma unroll
        for (int q = 0; q < NP; ++q) {
          const Rt xv = fma(gs[s][q], uu, y[s][q]);
          if (q == NP - 1) xo = xv;
          f.st(chain + (int64_t)(lb + s) * d.cell_step + q * d.plane_step, xv);
        }
        uu = theta * xo + omt * fo[s];
      }
    }
    u = unext;
  }
  if (refine_prec(PREC)) {
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
    if (!(fabs(a[piv][col]) > kSingularPivot * norm)) {
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
// dispatch
// ---------------------------------------------------------------------------
template <int PREC, int NP>
hipError_t go_sweep(bool graded, bool wpos, const SweepItem *items, int n_items, const SweepDesc *descs,
                    const OpEntry *ops, int dt_idx, StateBuf f, const double *fb_old, const double *fb_new,
                    double *stats, hipStream_t st) {
  constexpr int SMAX = sweep_smax(NP);
  constexpr int SMAXG = sweep_smax_graded(NP);
  if (graded && wpos)
    hipLaunchKernelGGL((sweep_graded_kernel<PREC, NP, SMAXG, true>), dim3(n_items), dim3(kBlock), 0, st, items, descs,
                       ops, dt_idx, State<PREC>::make(f), fb_old, fb_new, stats);
  else if (graded)
    hipLaunchKernelGGL((sweep_graded_kernel<PREC, NP, SMAXG, false>), dim3(n_items), dim3(kBlock), 0, st, items,
                       descs, ops, dt_idx, State<PREC>::make(f), fb_old, fb_new, stats);
  else
    hipLaunchKernelGGL((sweep_kernel<PREC, NP, SMAX>), dim3(n_items), dim3(kBlock), 0, st, items, descs, ops,
                       dt_idx, State<PREC>::make(f), fb_old, fb_new, stats);
  return hipGetLastError();
}

template <int PREC>
hipError_t go_sweep_np(bool graded, bool wpos, int np, const SweepItem *items, int n_items, const SweepDesc *descs,
                       const OpEntry *ops, int dt_idx, StateBuf f, const double *fb_old, const double *fb_new,
                       double *stats, hipStream_t st) {
  switch (np) {
    case 2: return go_sweep<PREC, 2>(graded, wpos, items, n_items, descs, ops, dt_idx, f, fb_old, fb_new, stats, st);
    case 3: return go_sweep<PREC, 3>(graded, wpos, items, n_items, descs, ops, dt_idx, f, fb_old, fb_new, stats, st);
    case 4: return go_sweep<PREC, 4>(graded, wpos, items, n_items, descs, ops, dt_idx, f, fb_old, fb_new, stats, st);
    case 5: return go_sweep<PREC, 5>(graded, wpos, items, n_items, descs, ops, dt_idx, f, fb_old, fb_new, stats, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_invert(OpEntry *ops, int n_ops, hipStream_t st) {
  if (n_ops <= 0) return hipSuccess;
  hipLaunchKernelGGL(invert_kernel, dim3((n_ops + 63) / 64), dim3(64), 0, st, ops, n_ops);
  return hipGetLastError();
}

hipError_t launch_sweep_mixed(int prec, const SweepItem *items, int n_items, const SweepDesc *descs,
                              const OpEntry *ops, int dt_idx, StateBuf f, const double *fb_old,
                              const double *fb_new, double *stats, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
#define PDG_MIXED_CASE(PR)                                                                                   \
  case PR:                                                                                                   \
    hipLaunchKernelGGL(sweep_mixed_kernel<PR>, dim3(n_items), dim3(kBlock), 0, st, items, descs, ops, dt_idx, \
                       State<PR>::make(f), fb_old, fb_new, stats);                                           \
    break;
  switch (prec) {
    PDG_MIXED_CASE(kF64)
    PDG_MIXED_CASE(kF32)
    PDG_MIXED_CASE(kRefine)
    PDG_MIXED_CASE(kP48)
    default: return hipErrorInvalidValue;
  }
#undef PDG_MIXED_CASE
  return hipGetLastError();
}

hipError_t launch_sweep(int prec, int np, bool graded, bool wpos, const SweepItem *items, int n_items,
                        const SweepDesc *descs, const OpEntry *ops, int dt_idx, StateBuf f, const double *fb_old,
                        const double *fb_new, double *stats, hipStream_t st) {
  if (n_items <= 0) return hipSuccess;
  switch (prec) {
    case kF64: return go_sweep_np<kF64>(graded, wpos, np, items, n_items, descs, ops, dt_idx, f, fb_old, fb_new, stats, st);
    case kF32: return go_sweep_np<kF32>(graded, wpos, np, items, n_items, descs, ops, dt_idx, f, fb_old, fb_new, stats, st);
    case kRefine: return go_sweep_np<kRefine>(graded, wpos, np, items, n_items, descs, ops, dt_idx, f, fb_old, fb_new, stats, st);
    case kP48: return go_sweep_np<kP48>(graded, wpos, np, items, n_items, descs, ops, dt_idx, f, fb_old, fb_new, stats, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pdg
