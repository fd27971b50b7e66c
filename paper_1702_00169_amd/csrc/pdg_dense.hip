// gfx950 kernels of the transport sweep for velocities with two or three
// non-zero components: dense cell blocks in a tiled wavefront.

#include <type_traits>
#include <utility>

#include "pdg_device.h"

namespace pdg {
namespace {

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
  // A^{-1} rounded to binary32 (n^2 floats in (n^2 + 1) / 2 doubles): the
  // refined solve reads its binary32 operands as they are
  __host__ __device__ int64_t ai32_off() const { return 4 * n * n + 3 * n * f; }
  // transfer operator of a full tile (two-dimensional velocities only)
  __host__ __device__ int64_t r_off() const { return 4 * n * n + 3 * n * f + (n * n + 1) / 2; }
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
      if (!(fabs(a[pv][col]) > kSingularPivot * norm)) sing = 1;
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
    reinterpret_cast<float *>(row + L.ai32_off())[e] = (float)inv[i][j];
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

// number of nodes on the downwind faces: NP^DIM - (NP-1)^DIM
template <int NP, int DIM>
__device__ constexpr int dense_out_nodes() {
  int all = 1, inner = 1;
  for (int b = 0; b < DIM; ++b) {
    all *= NP;
    inner *= NP - 1;
  }
  return all - inner;
}

// true when node q lies on a downwind face (some coordinate equals NP - 1)
template <int NP, int DIM>
__device__ constexpr bool on_out_face(int q) {
  for (int b = 0; b < DIM; ++b) {
    if (q % NP == NP - 1) return true;
    q /= NP;
  }
  return false;
}

// y = A^{-1} B f of one cell in the precision of the policy.  Binary32 +
// refinement: binary32 solve, binary64 residual B f - A y, one binary32
// correction.
template <int PREC, int N, int F>
__device__ __forceinline__ void dense_local_solve(const double *row, const typename Pol<PREC>::Rt (&fv)[N],
                                                  typename Pol<PREC>::Rt (&y)[N]) {
  using Rt = typename Pol<PREC>::Rt;
  const DenseRowLayout L{N, F};
  if (refine_prec(PREC)) {
    const float *ai32 = reinterpret_cast<const float *>(row + L.ai32_off());
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
      for (int j = 0; j < N; ++j) acc = fmaf(ai32[i * N + j], r32[j], acc);
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
      for (int j = 0; j < N; ++j) acc = fmaf(ai32[i * N + j], r32[j], acc);
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
}

// ---------------------------------------------------------------------------
// transfer schedule (two-dimensional velocities with two non-zero components)
// ---------------------------------------------------------------------------
// A full tile of T x T cells is linear in its data: its outflow traces are
// Z(f, domain inflow) + R u, u its inflow traces from upwind tiles.  Traces
// of a tile edge are indexed edge cell by edge cell, face node fastest: the
// west (inflow) and east (outflow) edges by cell row j as j F + tt, the south
// and north edges by cell column i as T F + i F + tt, so the east/north part
// of a tile's output is the west/south part of its neighbours' input.  R
// (2TF x 2TF) is the same for every full tile of a (velocity, sub-step).  It
// is stored in the order of the A operand of the binary64 16x16x4 MFMA:
// element (row o, column c) at ((o / 16) (2TF / 4) + c / 4) 64 + o % 16 +
// 16 (c % 4), so that lane l of a wave reads entry l of each 16 x 4 block.
constexpr int kTransferT = 8;        // tile edge (cells)
constexpr int kTransferMaxDiag = 64; // tiles per diagonal held in LDS (edge <= 512 cells)

__host__ __device__ constexpr int64_t transfer_index(int o, int c, int nr) {
  return ((int64_t)(o / 16) * (nr / 4) + c / 4) * 64 + o % 16 + 16 * (c % 4);
}

// One thread per column c of R: the tile is solved from f = 0 with the unit
// inflow e_c, cell by cell in row order (a cell's west and south neighbours
// come first), keeping only the traces that cross cell faces: with f = 0 the
// local solve gives y = 0, so x = G_0 u_west + G_1 u_south and an outflow
// trace is theta x at the outflow face node.
template <int NP>
__global__ __launch_bounds__(128) void dense_transfer_operator_kernel(double *table, const int64_t *row_off,
                                                                      const DenseDesc *descs,
                                                                      const int32_t *row_desc) {
  constexpr int N = NP * NP, F = NP, T = kTransferT, TF = T * F, NR = 2 * TF;
  const int c = threadIdx.x;
  if (c >= NR) return;
  double *row = table + row_off[blockIdx.x];
  const DenseDesc &d = descs[row_desc[blockIdx.x]];
  if (d.nshape > 1) return;  // graded cells: rows without a transfer operator
  const DenseRowLayout L{N, F};
  const double th = d.theta;
  const double *g0 = row + L.g(0);
  const double *g1 = row + L.g(1);
  double us[T][F];  // inflow from the south of each cell column: the north traces of the row below
#pragma unroll
  for (int i = 0; i < T; ++i)
#pragma unroll
    for (int tt = 0; tt < F; ++tt) us[i][tt] = (c == TF + i * F + tt) ? 1.0 : 0.0;
  for (int j = 0; j < T; ++j) {
    double uw[F];
#pragma unroll
    for (int tt = 0; tt < F; ++tt) uw[tt] = (c == j * F + tt) ? 1.0 : 0.0;
#pragma unroll
    for (int i = 0; i < T; ++i) {
      double ue[F], un[F];
#pragma unroll
      for (int tt = 0; tt < F; ++tt) {
        const int qe = face_node<NP, 2>(0, tt, NP - 1);
        const int qn = face_node<NP, 2>(1, tt, NP - 1);
        double xe = 0.0, xn = 0.0;
#pragma unroll
        for (int s2 = 0; s2 < F; ++s2) {
          xe = fma(g0[qe * F + s2], uw[s2], fma(g1[qe * F + s2], us[i][s2], xe));
          xn = fma(g0[qn * F + s2], uw[s2], fma(g1[qn * F + s2], us[i][s2], xn));
        }
        ue[tt] = th * xe;
        un[tt] = th * xn;
      }
#pragma unroll
      for (int tt = 0; tt < F; ++tt) {
        uw[tt] = ue[tt];
        us[i][tt] = un[tt];
      }
    }
#pragma unroll
    for (int tt = 0; tt < F; ++tt) row[L.r_off() + transfer_index(j * F + tt, c, NR)] = uw[tt];
  }
#pragma unroll
  for (int i = 0; i < T; ++i)
#pragma unroll
    for (int tt = 0; tt < F; ++tt) row[L.r_off() + transfer_index(TF + i * F + tt, c, NR)] = us[i][tt];
}

// The trace wavefront of one family (velocity, component) over its tile
// diagonals, after the zero-inflow tile pass has left each tile's Z in the
// slots of its downwind tiles.  Tile (I, J) of diagonal s = I + J takes its
// inflow from the outputs of (I - 1, J) and (I, J - 1) on diagonal s - 1;
// the outputs of a diagonal are one matrix product OUT = Z + R IN over its
// tiles (columns), computed as 16 x 16 blocks of binary64 MFMA: product wave
// w < 4 owns the row blocks w, w + 4, .. of R, whose A operands stay in
// registers for the whole sweep.  The outputs replace Z in the slots, where
// the final tile pass reads them as exact inflow traces.
//
// Diagonals live in three LDS buffers: diagonal s in buffer s % 3 holds Z(s)
// before its product and OUT(s) after.  The product waves touch no global
// memory in the loop.  Three loader waves take turns (diagonal t by loader
// t % 3): they issue the loads of Z(t) three diagonals ahead and write them
// to LDS one diagonal ahead, into the buffer that diagonal t - 3 left (with
// diagonals of up to 64 tiles, two loaders per residue split the rows); the
// store wave writes OUT(s - 1) to the slots while diagonal s is computed.  On
// this architecture loads and stores share one wait counter, so keeping each
// wave to one kind keeps every wait to the wave's own oldest requests.
typedef double transfer_d4 __attribute__((ext_vector_type(4)));
// four product waves, the store wave and 3 MD / 32 loader waves
__host__ __device__ constexpr int transfer_threads(int md) { return (5 + 3 * (md / 32)) * 64; }
// The values loaded for Z where a tile column has no downwind slot.
__device__ uint64_t kTransferZero[128] = {};  // never written; more than any NR

// Workgroup barrier that orders LDS only: global stores in flight are not
// drained (nothing in the wavefront reads a slot that is written in the same
// launch).  The empty asm keeps the compiler from moving loads across it.
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __asm__ __volatile__("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

template <int F, int MD>
__global__ __launch_bounds__(transfer_threads(MD)) void dense_transfer_kernel(const DenseTile *__restrict__ tiles,
                                                                          const DenseFam *__restrict__ fams,
                                                                          const int32_t *__restrict__ fam_list,
                                                                          const DenseDesc *__restrict__ descs,
                                                                          const double *__restrict__ table,
                                                                          int dt_idx, uint64_t *__restrict__ traces) {
  constexpr int N = F * F, T = kTransferT, TF = T * F, NR = 2 * TF, KS = NR / 4, NRB = NR / 16;
  constexpr int NPW = (NRB + 3) / 4;               // row blocks per product wave
  constexpr int NCB = MD / 16;                     // column blocks of the longest diagonal
  constexpr int LS = MD + 16;                      // LDS row stride (doubles): 16 mod 32 keeps reads conflict-free
  constexpr int NLP = MD / 32;                     // loaders per diagonal residue mod 3
  constexpr int OQL = NR / 4 / NLP;                // row quads per loader
  __shared__ double ob[3][NR][LS];                 // [diagonal % 3][row][tile column]
  const DenseFam fm = fams[fam_list[blockIdx.x]];
  const DenseDesc &d = descs[fm.desc];
  const DenseRowLayout L{N, F};
  const double *R = table + d.op_off + (int64_t)dt_idx * d.op_stride + L.r_off();
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  const int nt0 = fm.nt[0], nt1 = fm.nt[1];
  const int ndiag = nt0 + nt1 - 1;
  // A family's tiles were given their trace slots in order (t0 fastest), 3
  // axis slots each: tile (I, J)'s slots start at tbase + (I + nt0 J) 3 slot.
  const int slot = tiles[fm.tile0].slot;
  const int64_t tbase = tiles[fm.tile0].trace_off;
  auto diag_len = [&](int s) { return min(s, nt0 - 1) - max(0, s - nt1 + 1) + 1; };
  // slot rows fed by the tile in column j of diagonal s: the axis-0 slot of
  // (I + 1, J) takes its east outputs (rows o < TF), the axis-1 slot of
  // (I, J + 1) its north outputs (rows TF + ..); null where the tile has no
  // such downwind neighbour or j is past the diagonal's end.  Computed once
  // per tile column, so each row is one fixed offset from its base.
  auto out_rows = [&](int s, int j, uint64_t *&east, uint64_t *&north) {
    const int ilo = max(0, s - nt1 + 1), ihi = min(s, nt0 - 1);
    const int I = ilo + j, J = s - I;
    const bool in = I <= ihi;
    east = in && I + 1 < nt0 ? traces + tbase + (int64_t)((I + 1) + nt0 * J) * (3 * slot) : nullptr;
    north = in && J + 1 < nt1 ? traces + tbase + (int64_t)(I + nt0 * (J + 1)) * (3 * slot) + slot : nullptr;
  };
  if (w >= 4) {
    // memory waves: lane l covers rows 4 oq + l / 16 and tile columns
    // 16 jq + l % 16 of a diagonal (conflict-free in LDS, 32-byte runs in the slots)
    const int jl = l & 15, ol = l >> 4;
    if (w == 4) {
      auto store_diag = [&](int s) {
        const int n = diag_len(s), buf = s % 3;
#pragma unroll
        for (int jq = 0; jq < NCB; ++jq) {
          if (jq * 16 >= n) break;  // wave-uniform
          const int j = 16 * jq + jl;
          uint64_t *east, *north;
          out_rows(s, j, east, north);
#pragma unroll
          for (int oq = 0; oq < NR / 4; ++oq) {
            const int o = 4 * oq + ol;
            uint64_t *row = oq < TF / 4 ? east : north;
            if (row) row[oq < TF / 4 ? o : o - TF] = (uint64_t)__double_as_longlong(ob[buf][o][j]);
          }
        }
      };
      for (int p = -1; p < ndiag; ++p) {
        if (p >= 1) store_diag(p - 1);
        lds_barrier();
      }
      store_diag(ndiag - 1);
      return;
    }
    const int k = (w - 5) % 3;             // this loader's diagonals: t % 3 == k
    const int oq0 = ((w - 5) / 3) * OQL;   // and its row quads
    double zr[OQL][NCB];
    auto issue = [&](int t) {
      const int n = diag_len(t);
#pragma unroll
      for (int jq = 0; jq < NCB; ++jq) {
        if (jq * 16 >= n) break;  // wave-uniform
        uint64_t *east, *north;
        out_rows(t, 16 * jq + jl, east, north);
        // rows without a slot read zeros (row index 4 oq < NR)
        const uint64_t *eb = east ? east + ol : kTransferZero;
        const uint64_t *nb = north ? north + ol - TF : kTransferZero;
#pragma unroll
        for (int q = 0; q < OQL; ++q) {
          const int oq = oq0 + q;
          const uint64_t *row = oq < TF / 4 ? eb : nb;
          zr[q][jq] = __longlong_as_double((long long)row[4 * oq]);
        }
      }
    };
    auto write = [&](int t) {
      const int n = diag_len(t), buf = t % 3;
#pragma unroll
      for (int jq = 0; jq < NCB; ++jq) {
        if (jq * 16 >= n) break;  // wave-uniform
#pragma unroll
        for (int q = 0; q < OQL; ++q) ob[buf][4 * (oq0 + q) + ol][16 * jq + jl] = zr[q][jq];
      }
    };
    // Z(t) is loaded during phases t - 3 .. t - 1 (from the prologue for
    // t < 3) and written to LDS in phase t - 1
    for (int p = -1; p < ndiag; ++p) {
      const int tw = p + 1, tl = p + 3;
      if (tw < ndiag && tw % 3 == k) {
        if (tw == 0) issue(0);
        write(tw);
      }
      if (p == -1 && k == 1 && 1 < ndiag) issue(1);
      if (tl < ndiag && tl % 3 == k) issue(tl);
      lds_barrier();
    }
    return;
  }
  double A[NPW][KS];
#pragma unroll
  for (int r = 0; r < NPW; ++r)
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) A[r][ks] = (w + 4 * r < NRB) ? R[((w + 4 * r) * KS + ks) * 64 + l] : 0.0;
  // B operand: lane l holds row kq = l / 16, column jj = l % 16 of a 4 x 16
  // block; C and D: register i of lane l holds row 4 i + kq, column jj
  const int jj = l & 15, kq = l >> 4;
  lds_barrier();  // Z(0) in LDS
  for (int s = 0; s < ndiag; ++s) {
    const int cur = s % 3, prv = (s + 2) % 3;
    const int ilo = max(0, s - nt1 + 1), ihi = min(s, nt0 - 1);
    const int plo = max(0, s - nt1);  // first tile column I of diagonal s - 1
    const int ncb = (ihi - ilo) / 16 + 1;
    // column blocks in pairs: every B operand of a pair is read (from an
    // in-range column, then masked) before the two MFMA chains are issued
    // interleaved; the second chain is skipped past the diagonal's end
#pragma unroll
    for (int cp = 0; cp < NCB; cp += 2) {
      if (cp >= ncb) break;  // wave-uniform
      const bool two = cp + 1 < ncb;
      double b[2][KS];
      int jcol[2];
      bool valid[2];
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int j = (cp + h) * 16 + jj;
        jcol[h] = j;
        valid[h] = cp + h < ncb && ilo + j <= ihi;
        const int I = ilo + j, J = s - I;
        // west neighbour (I - 1, J) and south neighbour (I, J - 1) on diagonal s - 1
        const bool west = valid[h] && I > 0, south = valid[h] && J > 0;
        const int cw = west ? I - 1 - plo : 0, cs = south ? I - plo : 0;
#pragma unroll
        for (int ks = 0; ks < KS; ++ks) {
          const int kk = 4 * ks + kq;  // input index
          const bool use = kk < TF ? west : south;
          const double x = ob[prv][kk][kk < TF ? cw : cs];
          b[h][ks] = use ? x : 0.0;
        }
      }
#pragma unroll
      for (int r = 0; r < NPW; ++r) {
        const int rb = w + 4 * r;
        if (rb >= NRB) break;  // wave-uniform
        transfer_d4 acc0, acc1;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          acc0[i] = ob[cur][rb * 16 + 4 * i + kq][jcol[0]];
          acc1[i] = ob[cur][rb * 16 + 4 * i + kq][jcol[1]];
        }
        if (two) {
#pragma unroll
          for (int ks = 0; ks < KS; ++ks) {
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(A[r][ks], b[0][ks], acc0, 0, 0, 0);
            acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(A[r][ks], b[1][ks], acc1, 0, 0, 0);
          }
        } else {
#pragma unroll
          for (int ks = 0; ks < KS; ++ks)
            acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(A[r][ks], b[0][ks], acc0, 0, 0, 0);
        }
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          if (!valid[h]) continue;
#pragma unroll
          for (int i = 0; i < 4; ++i) ob[cur][rb * 16 + 4 * i + kq][jcol[h]] = h == 0 ? acc0[i] : acc1[i];
        }
      }
    }
    lds_barrier();
  }
}

// Register slots of the claimed schedule's trace requests: up to 4 (three
// diagonals ahead), as many as fit in 64 VGPRs.
template <int DIM, int F>
__device__ constexpr int dense_peek_ring() {
  const int r = 64 / (2 * DIM * F);
  return r < 1 ? 1 : (r > 4 ? 4 : r);
}

// One turn of the request ring: step(s0 + k, k) for k = 0 .. RING - 1 while
// s0 + k < n, with k a constant.
template <class Step, int... K>
__device__ __forceinline__ void dense_ring_turn(int s0, int n, Step &step, std::integer_sequence<int, K...>) {
  ((s0 + K < n ? step(s0 + K, std::integral_constant<int, K>{}) : void()), ...);
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

// Report a failure of the dense sweep (code 1: a wait gave up, 2: a claim
// past the last tile) on the device flag and, if there is one, on the
// host-visible flag.
__device__ inline void dense_fail(const DenseErr &err, int code) {
  __hip_atomic_fetch_or(err.dev, code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (err.host) __hip_atomic_fetch_or(err.host, code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// The inflow traces a cell needs from upwind tiles (up to one face per axis,
// at traces + src[a]; src[a] < 0 where the face is not fed by a tile).
// Every slot is requested at once, so a ready face costs one round trip; the
// slots still empty are polled again after a short sleep.  The producer was
// claimed earlier and is resident, so the wait ends; the wall-clock bound
// (err.wait_ticks of the 100 MHz constant clock, 1 s by default) and the
// shared error flag turn a logic error into one reported failure instead of
// a hang.
template <int DIM, int F>
__device__ inline void dense_take_faces(uint64_t *traces, const int64_t (&src)[DIM], uint64_t (&b)[DIM][F],
                                        const DenseErr &err) {
  bool ready = true;
#pragma unroll
  for (int a = 0; a < DIM; ++a)
    if (src[a] >= 0)
#pragma unroll
      for (int tt = 0; tt < F; ++tt) b[a][tt] = dense_peek_trace(traces + src[a] + tt);
#pragma unroll
  for (int a = 0; a < DIM; ++a)
    if (src[a] >= 0)
#pragma unroll
      for (int tt = 0; tt < F; ++tt) ready = ready && b[a][tt] != kDenseTraceEmpty;
  if (ready) return;
  const uint64_t t_start = wall_clock64();
  for (int naps = 1;; naps = naps < 8 ? 2 * naps : 8) {
    // back off (up to ~0.4 us between polls): the waiting waves would
    // otherwise keep the atomic units busy for the waves that produce
    for (int k = 0; k < naps; ++k) __builtin_amdgcn_s_sleep(2);
    ready = true;
#pragma unroll
    for (int a = 0; a < DIM; ++a)
      if (src[a] >= 0)
#pragma unroll
        for (int tt = 0; tt < F; ++tt)
          if (b[a][tt] == kDenseTraceEmpty) b[a][tt] = dense_peek_trace(traces + src[a] + tt);
#pragma unroll
    for (int a = 0; a < DIM; ++a)
      if (src[a] >= 0)
#pragma unroll
        for (int tt = 0; tt < F; ++tt) ready = ready && b[a][tt] != kDenseTraceEmpty;
    if (ready) return;
    if (wall_clock64() - t_start > err.wait_ticks ||
        __hip_atomic_load(err.dev, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
      dense_fail(err, 1);
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

// One wave per tile, in one of these modes (DenseMode):
// * claimed (kDenseClaim): one launch for all tiles.  The tile index is
//   claimed by lane 0 from a counter that hands out tiles in dependency order
//   (upwind tiles first) and broadcast with readfirstlane, so it is
//   wave-uniform; inflow traces arrive through the atomic slots above, cell by
//   cell, so a tile starts as soon as its first upwind cells are done.
// * levelled (kDenseLevel): one launch per tile diagonal; the launch's tiles
//   are order[0 .. n_tiles).  Upwind tiles belong to earlier launches, whose
//   writes the kernel boundary makes visible: plain loads and stores, no
//   waiting.
// * the two tile passes of the transfer schedule (all tiles in one launch,
//   no waiting): kDenseZero solves each tile with the traces of its upwind
//   tiles taken as zero (domain inflow as given) and stores only its outflow
//   traces, into the downwind tiles' slots; after the trace wavefront has
//   replaced them by the exact traces (dense_transfer_kernel), kDenseFinal
//   solves each tile with them and stores the cells (and no traces).
// Either way descriptors and operator rows are read through scalar loads and
// all control flow that depends on the tile is uniform.  Inside the tile the
// cells are solved diagonal by diagonal; the inflow traces of a cell come from
// the previous diagonal through LDS, from an upwind tile through the trace
// slots, or from the domain inflow data.
template <int PREC, int NP, int DIM, int MODE, bool GRADED>
__global__ __launch_bounds__(kDenseThreads) void dense_sweep_kernel(
    const DenseTile *__restrict__ tiles, const int32_t *__restrict__ order, const DenseFam *__restrict__ fams,
    const DenseDesc *__restrict__ descs, const double *__restrict__ table, int dt_idx,
    const State<PREC> f, const double *__restrict__ fb_old, const double *__restrict__ fb_new,
    uint64_t *traces, int32_t *counter, const DenseErr err, int n_tiles) {
  static_assert(kDenseThreads == 64, "one workgroup is one wave");
  using Rt = typename Pol<PREC>::Rt;
  constexpr int N = DIM == 2 ? NP * NP : NP * NP * NP;
  constexpr int F = DIM == 2 ? NP : NP * NP;
  __shared__ Rt otr[3][kDenseThreads][F];  // outflow traces per axis of every cell of the tile
  __shared__ Rt gl[DIM][N][F];             // G_a of the tile's operator row
  const int t = threadIdx.x;
  int claim = blockIdx.x;
  if (MODE == kDenseClaim) {
    if (t == 0) claim = atomicAdd(counter, 1);
    claim = __builtin_amdgcn_readfirstlane(claim);
    if (claim >= n_tiles) {  // the counter was not reset: report, do nothing
      if (t == 0) dense_fail(err, 2);
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
  // the operator row of this cell's size class (one class on uniform cells)
  const bool graded = GRADED && d.nshape > 1;  // wave-uniform
  int64_t shape = 0;
  if (graded) {
#pragma unroll
    for (int a = 0; a < DIM; ++a)
      if (d.rank_off[a] >= 0) {
        const int xa = min(max(x[a], 0), d.n[a] - 1);  // lanes past the mesh read a valid class
        shape += (int64_t)table[d.rank_off[a] + xa] * d.rank_stride[a];
      }
  }
  const double *row = table + d.op_off + ((int64_t)dt_idx * d.nshape + shape) * d.op_stride;
  const DenseRowLayout L{N, F};

  // Stage the coupling blocks G_a in LDS (vector loads, all lanes; graded
  // meshes read each cell's own from its row), load the cell and apply the
  // local block.
  if (!graded) {
#pragma unroll
    for (int a = 0; a < DIM; ++a)
      for (int e = t; e < N * F; e += kDenseThreads) gl[a][e / F][e % F] = (Rt)row[L.g(a) + e];
  }
  auto G = [&](int a, int q, int tt) -> Rt { return graded ? (Rt)row[L.g(a) + q * F + tt] : gl[a][q][tt]; };
  Rt fv[N], y[N];
#pragma unroll
  for (int q = 0; q < N; ++q) fv[q] = active ? f.ld(fm.f_base + d.plane_off[q] + cell) : (Rt)0;
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
  int64_t rsrc[DIM];  // offset of the upwind tile's trace slots, -1 if none
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    rsrc[a] = -1;
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
      if (MODE == kDenseZero) continue;  // upwind tile's traces taken as zero
      rsrc[a] = tl.trace_off + (int64_t)a * tl.slot + fc * F;
      if (MODE == kDenseLevel || MODE == kDenseFinal)
#pragma unroll
        for (int tt = 0; tt < F; ++tt) uin[a][tt] = (Rt)__longlong_as_double((long long)traces[rsrc[a] + tt]);
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

  // The local block, once the loads above are all in flight.
  dense_local_solve<PREC, N, F>(row, fv, y);
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

  // Loop-invariant data of the diagonal loop, read once: the axis signs, the
  // downwind trace slots and, when they fit in registers, the rows of G_a
  // that the outflow nodes need.
  bool on[DIM];
  int64_t dst[DIM];  // offset of the downwind tile's trace slots, -1 if none
#pragma unroll
  for (int b = 0; b < DIM; ++b) {
    on[b] = d.sgn[b] != 0;
    dst[b] = -1;
    if (!on[b] || !active || cl[b] != d.T[b] - 1 || tl.down[b] < 0) continue;
    int fc = 0, fs = 1;
#pragma unroll
    for (int a2 = 0; a2 < DIM; ++a2)
      if (a2 != b && d.sgn[a2] != 0) {
        fc += cl[a2] * fs;
        fs *= d.T[a2];
      }
    const DenseTile &dn = tiles[tl.down[b]];
    dst[b] = dn.trace_off + (int64_t)b * dn.slot + fc * F;
  }
  int up_lds[DIM];
#pragma unroll
  for (int a = 0; a < DIM; ++a) up_lds[a] = t - tstride[a];
  // G rows in registers (<= 128 VGPRs) shorten each diagonal step, which is on
  // the critical path of the claimed and levelled schedules; the two passes
  // of the transfer schedule have no critical path inside a tile and keep
  // them in LDS, for the occupancy
  constexpr bool kRegG = (MODE == kDenseClaim || MODE == kDenseLevel) &&
                         dense_out_nodes<NP, DIM>() * DIM * F * (int)sizeof(Rt) <= 512;
  Rt gr[DIM][N][F];
  if constexpr (kRegG) {
#pragma unroll
    for (int a = 0; a < DIM; ++a)
#pragma unroll
      for (int q = 0; q < N; ++q)
        if (on_out_face<NP, DIM>(q))
#pragma unroll
          for (int tt = 0; tt < F; ++tt) gr[a][q][tt] = G(a, q, tt);
  }

  // Claimed schedule: a cell's traces from upwind tiles are requested AHEAD
  // diagonals before the cell's own (compare-and-swap reads that do not
  // wait), so the round trip overlaps the diagonals in between; only a value
  // still empty when it is needed is polled again, waiting.  The requests
  // land in a ring of AHEAD + 1 register slots (lanes of different
  // diagonals write different registers: a register with a request in
  // flight cannot be read by any lane); the diagonal loop is unrolled by the
  // ring length, so the slot indices are constants.  The ring is kept within
  // 64 VGPRs; without one (large faces) a cell requests and waits at its own
  // diagonal.
  constexpr int RING = dense_peek_ring<DIM, F>();
  constexpr int AHEAD = RING - 1;
  // (no ring: a one-slot placeholder, unused)
  uint64_t pk[AHEAD > 0 ? RING : 1][AHEAD > 0 ? DIM : 1][AHEAD > 0 ? F : 1];
  if constexpr (AHEAD > 0) {
#pragma unroll
    for (int k = 0; k < RING; ++k)
#pragma unroll
      for (int a = 0; a < DIM; ++a)
#pragma unroll
        for (int tt = 0; tt < F; ++tt) pk[k][a][tt] = kDenseTraceEmpty;
  }
  auto peek = [&](auto &slot) {
#pragma unroll
    for (int a = 0; a < DIM; ++a)
      if (rsrc[a] >= 0)
#pragma unroll
        for (int tt = 0; tt < F; ++tt) slot[a][tt] = dense_peek_trace(traces + rsrc[a] + tt);
  };
  if constexpr (MODE == kDenseClaim && AHEAD > 0) {
    if (active && diag < AHEAD) {
#pragma unroll
      for (int k = 0; k < AHEAD; ++k)
        if (diag == k) peek(pk[k]);
    }
  }

  // Diagonal by diagonal, a cell needs only its outflow traces on the
  // critical path: the nodes on its downwind faces.  The inflow traces it
  // used are kept (uin) for the update of the other nodes after the loop.
  // diagonal s; k = s mod RING, a constant (the slot of diagonal s)
  auto step = [&](int s, auto kc) {
    constexpr int k = decltype(kc)::value;
    if constexpr (MODE == kDenseClaim && AHEAD > 0) {
      if (active && diag == s + AHEAD) peek(pk[(k + AHEAD) % RING]);
    }
    if (active && diag == s) {
      if constexpr (MODE == kDenseClaim && AHEAD > 0) {
        // the request made AHEAD diagonals ago; poll again only if empty
        uint64_t(&cur)[DIM][F] = pk[k];
        bool ready = true;
#pragma unroll
        for (int a = 0; a < DIM; ++a)
          if (rsrc[a] >= 0)
#pragma unroll
            for (int tt = 0; tt < F; ++tt) ready = ready && cur[a][tt] != kDenseTraceEmpty;
        if (!ready) dense_take_faces<DIM, F>(traces, rsrc, cur, err);
#pragma unroll
        for (int a = 0; a < DIM; ++a)
          if (rsrc[a] >= 0)
#pragma unroll
            for (int tt = 0; tt < F; ++tt) uin[a][tt] = (Rt)__longlong_as_double((long long)cur[a][tt]);
      } else if constexpr (MODE == kDenseClaim) {
        // no ring: request and wait now
        uint64_t rb[DIM][F];
        dense_take_faces<DIM, F>(traces, rsrc, rb, err);
#pragma unroll
        for (int a = 0; a < DIM; ++a)
          if (rsrc[a] >= 0)
#pragma unroll
            for (int tt = 0; tt < F; ++tt) uin[a][tt] = (Rt)__longlong_as_double((long long)rb[a][tt]);
      }
#pragma unroll
      for (int a = 0; a < DIM; ++a)
        if (on[a] && cl[a] > 0)
#pragma unroll
          for (int tt = 0; tt < F; ++tt) uin[a][tt] = otr[a][up_lds[a]][tt];
      Rt yo[N];
#pragma unroll
      for (int q = 0; q < N; ++q) yo[q] = y[q];
#pragma unroll
      for (int a = 0; a < DIM; ++a) {
        if (!on[a]) continue;
#pragma unroll
        for (int q = 0; q < N; ++q) {
          if (!on_out_face<NP, DIM>(q)) continue;
#pragma unroll
          for (int tt = 0; tt < F; ++tt) yo[q] = fma(kRegG ? gr[a][q][tt] : G(a, q, tt), uin[a][tt], yo[q]);
        }
      }
      // outflow traces: theta x + (1 - theta) f^n on each downwind face
#pragma unroll
      for (int b = 0; b < DIM; ++b) {
        if (!on[b]) continue;
#pragma unroll
        for (int tt = 0; tt < F; ++tt) {
          const int q = face_node<NP, DIM>(b, tt, NP - 1);
          const Rt o = th * yo[q] + omt * fv[q];
          otr[b][t][tt] = o;
          if (dst[b] >= 0) {
            if constexpr (MODE == kDenseLevel || MODE == kDenseZero)
              traces[dst[b] + tt] = (uint64_t)__double_as_longlong((double)o);
            else if constexpr (MODE == kDenseClaim)
              dense_put_trace(traces + dst[b] + tt, (double)o);
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
  };
  if constexpr (MODE != kDenseClaim) {
    for (int s = 0; s < ndiag; ++s) step(s, std::integral_constant<int, 0>{});
  } else {
    for (int s0 = 0; s0 < ndiag; s0 += RING) dense_ring_turn(s0, ndiag, step, std::make_integer_sequence<int, RING>{});
  }
  if (MODE == kDenseZero || !active) return;
  // every node: x = y + sum_a G_a u_a (the face nodes again, in the same
  // order, so they equal the values the traces were taken from)
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    if (!on[a]) continue;
#pragma unroll
    for (int q = 0; q < N; ++q)
#pragma unroll
      for (int tt = 0; tt < F; ++tt) y[q] = fma(G(a, q, tt), uin[a][tt], y[q]);
  }
#pragma unroll
  for (int q = 0; q < N; ++q) f.st(fm.f_base + d.plane_off[q] + cell, y[q]);
}

}  // namespace

hipError_t launch_dense_invert(double *table, const int64_t *row_off, const DenseDesc *descs,
                               const int32_t *row_desc, const double *c0, int32_t *flags, int n_rows, int n,
                               int F, hipStream_t st) {
  if (n_rows <= 0) return hipSuccess;
  if (n > kDenseMaxN || F > kDenseMaxF) return hipErrorInvalidValue;
  hipLaunchKernelGGL(dense_invert_kernel, dim3(n_rows), dim3(kDenseThreads), 0, st, table, row_off, descs, row_desc,
                     c0, flags, n, F);
  return hipGetLastError();
}

hipError_t launch_dense_transfer_operator(int np, double *table, const int64_t *row_off, const DenseDesc *descs,
                                          const int32_t *row_desc, int n_rows, hipStream_t st) {
  if (n_rows <= 0) return hipSuccess;
  switch (np) {
#define PDG_TOP_CASE(NPV)                                                                                    \
  case NPV:                                                                                                  \
    hipLaunchKernelGGL(dense_transfer_operator_kernel<NPV>, dim3(n_rows), dim3(128), 0, st, table, row_off, \
                       descs, row_desc);                                                                     \
    break;
    PDG_TOP_CASE(2)
    PDG_TOP_CASE(3)
    PDG_TOP_CASE(4)
    PDG_TOP_CASE(5)
#undef PDG_TOP_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_dense_transfer(int np, int max_diag, const DenseTile *tiles, const DenseFam *fams,
                                 const int32_t *fam_list, int n_fams, const DenseDesc *descs, const double *table,
                                 int dt_idx, uint64_t *traces, hipStream_t st) {
  if (n_fams <= 0) return hipSuccess;
  if (max_diag < 1 || max_diag > kTransferMaxDiag) return hipErrorInvalidValue;
  const bool wide = max_diag > 32;
  switch (np) {
#define PDG_TR_CASE(NPV)                                                                                        \
  case NPV:                                                                                                     \
    if (wide)                                                                                                   \
      hipLaunchKernelGGL((dense_transfer_kernel<NPV, 64>), dim3(n_fams), dim3(transfer_threads(64)), 0, st,    \
                         tiles, fams, fam_list, descs, table, dt_idx, traces);                                  \
    else                                                                                                        \
      hipLaunchKernelGGL((dense_transfer_kernel<NPV, 32>), dim3(n_fams), dim3(transfer_threads(32)), 0, st,    \
                         tiles, fams, fam_list, descs, table, dt_idx, traces);                                  \
    break;
    PDG_TR_CASE(2)
    PDG_TR_CASE(3)
    PDG_TR_CASE(4)
    PDG_TR_CASE(5)
#undef PDG_TR_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <int PREC, int NP, int DIM>
hipError_t go_dense(int mode, const DenseTile *tiles, const int32_t *order, int n_tiles, const DenseFam *fams,
                    const DenseDesc *descs, const double *table, int dt_idx, StateBuf f, const double *fb_old,
                    const double *fb_new, uint64_t *traces, int32_t *counter, DenseErr err, hipStream_t st) {
#define PDG_DENSE_MODE(M, G)                                                                                    \
  hipLaunchKernelGGL((dense_sweep_kernel<PREC, NP, DIM, M, G>), dim3(n_tiles), dim3(kDenseThreads), 0, st, tiles, \
                     order, fams, descs, table, dt_idx, State<PREC>::make(f), fb_old, fb_new, traces, counter, err,  \
                     n_tiles)
  switch (mode) {
    case kDenseClaim: PDG_DENSE_MODE(kDenseClaim, false); break;
    case kDenseLevel: PDG_DENSE_MODE(kDenseLevel, false); break;
    case kDenseClaim | kDenseGraded: PDG_DENSE_MODE(kDenseClaim, true); break;
    case kDenseLevel | kDenseGraded: PDG_DENSE_MODE(kDenseLevel, true); break;
    case kDenseZero:
      if constexpr (DIM != 2) return hipErrorInvalidValue;  // the transfer schedule is two-dimensional
      else PDG_DENSE_MODE(kDenseZero, false);
      break;
    case kDenseFinal:
      if constexpr (DIM != 2) return hipErrorInvalidValue;
      else PDG_DENSE_MODE(kDenseFinal, false);
      break;
    default: return hipErrorInvalidValue;
  }
#undef PDG_DENSE_MODE
  return hipGetLastError();
}

template <int PREC>
hipError_t go_dense_shape(int mode, int np, int dim, const DenseTile *tiles, const int32_t *order, int n_tiles,
                          const DenseFam *fams, const DenseDesc *descs, const double *table, int dt_idx, StateBuf f,
                          const double *fb_old, const double *fb_new, uint64_t *traces, int32_t *counter,
                          DenseErr err, hipStream_t st) {
#define PDG_DENSE_CASE(NPV, DIMV)                                                                             \
  if (np == NPV && dim == DIMV)                                                                               \
    return go_dense<PREC, NPV, DIMV>(mode, tiles, order, n_tiles, fams, descs, table, dt_idx, f, fb_old, fb_new,    \
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

hipError_t launch_dense_sweep(int prec, int mode, int np, int dim, const DenseTile *tiles, const int32_t *order,
                              int n_tiles, const DenseFam *fams, const DenseDesc *descs, const double *table,
                              int dt_idx, StateBuf f, const double *fb_old, const double *fb_new, uint64_t *traces,
                              int32_t *counter, DenseErr err, hipStream_t st) {
  if (n_tiles <= 0) return hipSuccess;
  switch (prec) {
    case kF64: return go_dense_shape<kF64>(mode, np, dim, tiles, order, n_tiles, fams, descs, table, dt_idx, f, fb_old, fb_new, traces, counter, err, st);
    case kF32: return go_dense_shape<kF32>(mode, np, dim, tiles, order, n_tiles, fams, descs, table, dt_idx, f, fb_old, fb_new, traces, counter, err, st);
    case kRefine: return go_dense_shape<kRefine>(mode, np, dim, tiles, order, n_tiles, fams, descs, table, dt_idx, f, fb_old, fb_new, traces, counter, err, st);
    case kP48: return go_dense_shape<kP48>(mode, np, dim, tiles, order, n_tiles, fams, descs, table, dt_idx, f, fb_old, fb_new, traces, counter, err, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace pdg
