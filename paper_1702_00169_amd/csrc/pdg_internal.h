// Internal data structures shared by the host runtime (pdg_host.cpp) and the
// gfx950 kernels (pdg_sweep.hip: axis-aligned transport; pdg_local.hip:
// node-local steps; pdg_dense.hip: dense transport).  Not part of the public
// ABI.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

namespace pdg {

constexpr int kMaxNP = 5;       // d + 1 for degree <= 4
constexpr int kBlock = 256;     // threads per workgroup of every kernel
constexpr int kMaxNV = 27;
constexpr int kMaxM = 8;
// A cell block is taken as singular when a Gauss-Jordan pivot (partial
// pivoting) is at most this fraction of its largest entry: an exactly singular
// block leaves a pivot of rounding size, and the blocks I + theta dt Gamma
// of a forward step keep every pivot above 0.2 of the largest entry (d <= 4).
constexpr double kSingularPivot = 1e-12;

// One (instance, velocity) line family: how a chain (a line of cells along
// the velocity axis, ordered downwind) is addressed in the state array.
struct SweepDesc {
  int64_t cell_step;   // signed element step between consecutive downwind cells
  int64_t cell0;       // element offset of the upwind-most cell of a chain
  int64_t plane_step;  // signed element step between downwind-local nodes q, q+1
  int64_t plane0;      // element offset of local node q = 0 (the inflow node)
  int32_t n_a;         // cells per chain
  int32_t nx;          // transverse decode: tau -> (tau % nx) + (tau / nx) * hi_stride
  int64_t hi_stride;
  int32_t op;          // operator-table row of dt_sub = dt; op + 1 is dt/2
  int32_t x_kind;      // 1: chains along the contiguous axis; 2: chains on a graded axis
                       // (operator rows op + dt_idx * n_a + l; launched on their own)
};

// One workgroup's share of a sweep: `count` consecutive chains (tau0 ..) of
// one (instance, velocity, component, transverse node) family.
struct SweepItem {
  int64_t base;   // element offset of (instance, v, k, transverse node plane)
  int64_t fb;     // fb offset of chain tau0
  int32_t desc;   // SweepDesc index
  int32_t tau0;
  int32_t count;  // chains of this item (<= C)
  int16_t C;      // strided chains: chains per workgroup (kBlock / C segments per window)
  int8_t S;       // strided chains: cells per segment (<= sweep_smax(np))
  int8_t xk;      // 1: chains along the contiguous axis (one cell per thread, wave scan)
};

// Largest segment length compiled for a node count (register budget).
#ifndef PDG_SMAX_LOW
#define PDG_SMAX_LOW 8   // d + 1 <= 3
#endif
constexpr int sweep_smax(int np) { return np <= 3 ? PDG_SMAX_LOW : 4; }
// Same for chains on graded axes, which also hold each cell's g and a.
constexpr int sweep_smax_graded(int np) { return np <= 3 ? 4 : 2; }
// Largest segment length of a launch class (chain kind 2: graded axis).
constexpr int class_smax(int np, int x_kind) { return x_kind == 2 ? sweep_smax_graded(np) : sweep_smax(np); }

// Operator table row: one (instance, velocity, dt_sub).  Downwind-local node
// order (q = 0 inflow node, q = NP-1 outflow node).  Filled partly on the host
// (A, B, c0, theta) and partly by the inversion kernel.
struct OpEntry {
  double A[kMaxNP * kMaxNP];     // I + theta dt Gamma
  double B[kMaxNP * kMaxNP];     // I - (1 - theta) dt Gamma
  double Ainv[kMaxNP * kMaxNP];  // A^{-1}
  double M[kMaxNP * kMaxNP];     // A^{-1} B
  double g[kMaxNP];              // c0 A^{-1} e_0
  double c0;                     // dt * (2 |v| / h) / w_0 (inflow coefficient)
  double theta;
  double a;                      // theta * g[NP-1]: chain recurrence factor
  float M32[kMaxNP * kMaxNP];
  float Ainv32[kMaxNP * kMaxNP];
  float g32[kMaxNP];
  float a32;
  int32_t np;
  int32_t singular;              // set by the inversion kernel
  int32_t pad[2];
};

// Per-instance data of the node-local kernels.
struct RelaxDesc {
  int64_t f_base;      // element offset of the instance in f
  int64_t w_base;      // element offset of the instance in w
  int64_t nodes;       // Nd * Nc
  double param[4];     // advection: a_k; Euler: gamma; D2Q9: gravity g
  double lambda;
  int32_t nv, m, dim, feq;
  int8_t axis[kMaxNV]; // {+-lambda e_k} sets: velocity i = sign[i] * lambda * e_axis[i]
  int8_t sign[kMaxNV];
  int8_t cx[kMaxNV];   // D2Q9: velocity i = lambda (cx[i], cy[i])
  int8_t cy[kMaxNV];
  int16_t pad;
};

struct RelaxItem {
  int64_t node0;
  int32_t desc;
  int32_t count;
};

// Inflow-equilibrium items: one per (instance, velocity).
struct InflowDesc {
  int64_t fb_base;     // fb offset of (instance, v, k=0)
  int64_t w_base;      // w_inflow offset of (instance, v, moment 0)
  int64_t per_comp;    // inflow points of the velocity (values per component)
  int32_t relax_desc;
  int32_t vel;
};

// Fused collision + x transport (pdg_fused.hip; instances whose velocities
// are the set {+-lambda e_k} on a uniform box mesh).
struct FusedDesc {
  int64_t nc;        // cells
  int64_t fb[2];     // fb offset of (+x / -x velocity, k = 0, t = 0, tau = 0)
  int32_t rdesc;     // RelaxDesc of the instance
  int32_t vx[2];     // indices of the +x and -x velocities
  int32_t op[2];     // operator-table rows (dt_sub = dt) of the +x and -x velocities
  int32_t nx;        // cells per row
  int32_t ntau;      // rows of cells (nc / nx)
  int32_t tnodes;    // transverse nodes (d+1)^(D-1)
};

// One workgroup's row: row0 = jt ntau + tau (transverse node jt, row of
// cells tau).
struct FusedItem {
  int32_t desc;
  int32_t row0;
};

// ---- velocities with two or three non-zero components ---------------------
// The cell block is dense and the dependency graph is a k-dimensional
// wavefront over the axes with non-zero components.  Cells are grouped in
// tiles (8 x 8 for k = 2, 4 x 4 x 4 for k = 3); a tile waits for its upwind
// tiles and sweeps its own diagonals.
constexpr int kDenseMaxN = 27;      // (d+1)^D cell nodes handled by the dense path
constexpr int kDenseMaxF = 9;       // (d+1)^(D-1) face nodes
constexpr int kDenseThreads = 64;   // one thread per cell of a tile; one wave per tile
// content of an inflow-trace slot that has not been written yet in this sweep
// (a signalling NaN: arithmetic only ever produces quiet NaNs)
constexpr uint64_t kDenseTraceEmpty = 0x7ff4c0ffee5a1e57ull;

// One (instance, velocity) of the dense path.
struct DenseDesc {
  int64_t nc;                        // cells
  int64_t plane_off[kDenseMaxN];     // element offset of downwind-local node q's plane
  int64_t fb_axis_off[3];            // offset of axis a's face block inside a (v, k) fb block
  int64_t fb_ntc[3];                 // cells on the inflow face of axis a (Nc / n_a)
  int64_t op_off;                    // dense operator table offset of dt index 0 (doubles)
  int64_t op_stride;                 // doubles per dt index
  int32_t n[3];                      // cells per axis
  int32_t sgn[3];                    // sign of the velocity component per axis (0: zero)
  int32_t T[3];                      // tile extent per axis (1 on zero components)
  int32_t face_q[3][kDenseMaxF];     // local node of inflow-face node t of axis a (q_a = 0)
  int32_t out_q[3][kDenseMaxF];      // local node of outflow-face node t of axis a (q_a = NP-1)
  int32_t fb_t[3][kDenseMaxF];       // physical face-node index (fb layout) of face node t
  int32_t trans_axis;                // zero-component axis whose cells are independent, or -1
  // Graded meshes: the block depends on the cell sizes along the non-zero
  // components, so there is one operator row per size class (shape) and
  // sub-step: row (dt_idx nshape + shape), shape = sum_a class_a rank_stride[a],
  // class_a = table[rank_off[a] + x_a] (a small integer stored as a double)
  // for the cell coordinate x_a; rank_off[a] = -1 where axis a has one class.
  int64_t rank_off[3];
  int32_t rank_stride[3];
  int32_t nshape;                    // operator rows per sub-step (1: uniform cells)
  double theta;
};

// One (instance, velocity, component, transverse slice) sweep.
struct DenseFam {
  int64_t f_base;   // element offset of (instance, v, k, plane 0, cell 0)
  int64_t fb_base;  // fb offset of (instance, v, k)
  int32_t desc;
  int32_t slice;    // cell index along trans_axis (0 if none)
  int32_t tile0;    // launch-group index of the family's first tile (tiles follow with t0 fastest)
  int32_t nt[2];    // tiles along the first two axes
  int32_t pad;
};

// One tile of a dense sweep.
struct DenseTile {
  int64_t trace_off;  // offset of this tile's inflow-trace slots (one per axis)
  int32_t fam;
  int32_t tc[3];      // tile coordinates (downwind order), 0 on zero components
  int32_t up[3];      // upwind tile per axis, -1 on the domain boundary or zero component
  int32_t down[3];    // downwind tile per axis, -1 if none
  int32_t slot;       // doubles per axis slot of trace_off
  int32_t pad;
};

// ---- kernel launchers ------------------------------------------------------
// The state buffer of a launch: its base address and its element count n (the
// packed kP48 state holds n binary32 values followed by n int16 values).
struct StateBuf {
  void *p;
  int64_t n;
};
// kP48: the arithmetic of kRefine with the state stored in 48 bits per value
// (a binary32 plane, then an int16 plane with the next 16 bits; see State<kP48>).
enum Prec { kF64 = 0, kF32 = 1, kRefine = 2, kP48 = 3 };
constexpr bool refine_prec(int p) { return p == kRefine || p == kP48; }

hipError_t launch_invert(OpEntry *ops, int n_ops, hipStream_t st);

// Launch one sweep over items that share the node count np (any chain kind,
// tile shape or instance).  graded: chains on graded axes; wpos: their tile
// width C is a multiple of 64 (each wave at one chain position).
hipError_t launch_sweep(int prec, int np, bool graded, bool wpos, const SweepItem *items, int n_items,
                        const SweepDesc *descs, const OpEntry *ops, int dt_idx, StateBuf f, const double *fb_old,
                        const double *fb_new, double *stats, hipStream_t st);

// One launch over uniform-mesh items of any node count (each workgroup
// dispatches on its item's node count).
hipError_t launch_sweep_mixed(int prec, const SweepItem *items, int n_items, const SweepDesc *descs,
                              const OpEntry *ops, int dt_idx, StateBuf f, const double *fb_old,
                              const double *fb_new, double *stats, hipStream_t st);

// Relax / equilibrium launch for items whose instances share (nv, m).
hipError_t launch_relax(int prec, int nv, int m, const RelaxItem *items, int n_items, const RelaxDesc *descs,
                        StateBuf f, double *w_out, const double *w_in, double omega, int mode, hipStream_t st);

// Node counts, (nv, m) and row lengths the fused kernel handles
// ((d+1) ceil(nx / 64) 64 <= 512 threads per row).
bool fused_supported(int np, int nv, int m, int nx);
// Fused collision (factor omega) + transport of the +x and -x chains for
// the items (one row each) of one (d+1, nv, m, nx) group; stats: 2 doubles
// per item.
hipError_t launch_relax_xsweep(int prec, int np, int nv, int m, int nx, const FusedItem *items, int n_items,
                               const FusedDesc *fdescs, const RelaxDesc *rdescs, const OpEntry *ops, int dt_idx,
                               StateBuf f, const double *fb_old, const double *fb_new, double omega, double *stats,
                               hipStream_t st);

hipError_t launch_inflow_eq(int nv, int m, const InflowDesc *items, int n_items, const RelaxDesc *descs,
                            const double *w_inflow, double *fb, hipStream_t st);

// D2Q9 lattice instances (Sec. 5.1): mode 0 applies S(h_pre) C(omega)
// S(h_post) at every node (the source terms only where the instance has
// gravity), mode 1 sets f = f^eq(w_in).
hipError_t launch_lattice(int prec, const RelaxItem *items, int n_items, const RelaxDesc *descs, StateBuf f,
                          double *w_out, const double *w_in, double omega, double h_pre, double h_post, int mode,
                          hipStream_t st);
hipError_t launch_lattice_inflow(const InflowDesc *items, int n_items, const RelaxDesc *descs, const double *w_in,
                                 double *fb, hipStream_t st);
hipError_t launch_fill(double *p, int64_t n, double value, hipStream_t st);
// Conversion between the state of precision prec and binary64 values:
// to_f64 = true reads the state into x, false writes x into the state.
hipError_t launch_convert(int prec, StateBuf f, double *x, bool to_f64, hipStream_t st);
hipError_t launch_fill_int(int32_t *p, int64_t n, int32_t value, hipStream_t st);
hipError_t launch_fill_u64(uint64_t *p, int64_t n, uint64_t value, hipStream_t st);

// Dense cell blocks: per operator row, A and B (n x n) and the inflow
// coefficients c0[3] are set; computes Ainv, M = Ainv B and the face columns
// G_a = c0_a Ainv[:, face_q[a][t]].  Row layout (doubles): M, G[3] (n x F each),
// A, B, Ainv; flags[row] = 1 if A is singular.
hipError_t launch_dense_invert(double *table, const int64_t *row_off, const DenseDesc *descs,
                               const int32_t *row_desc, const double *c0, int32_t *flags, int n_rows, int n,
                               int F, hipStream_t st);

// Failure reporting of the dense sweep: a wait for an upwind trace that has
// lasted wait_ticks of the 100 MHz constant clock gives up; it (or a claim
// past the last tile) sets *dev (1: wait, 2: claim) and, if host is not
// NULL, *host (host-visible memory, read by the entry points without a
// synchronisation).
struct DenseErr {
  int32_t *dev;
  int32_t *host;
  uint64_t wait_ticks;
};

// Transfer operators R of full tiles (two-dimensional dense velocities), one
// per operator row listed (row_off, row_desc), after launch_dense_invert.
hipError_t launch_dense_transfer_operator(int np, double *table, const int64_t *row_off, const DenseDesc *descs,
                                          const int32_t *row_desc, int n_rows, hipStream_t st);
// Trace wavefront of the transfer schedule for the families fam_list[0..n)
// of one launch group (tiles: the group's tile array); max_diag (1..64) is the
// longest tile diagonal among them.
hipError_t launch_dense_transfer(int np, int max_diag, const DenseTile *tiles, const DenseFam *fams,
                                 const int32_t *fam_list, int n_fams, const DenseDesc *descs, const double *table,
                                 int dt_idx, uint64_t *traces, hipStream_t st);

// Modes of the dense tile kernel (see pdg_dense.hip): claimed tiles in one
// launch, one launch per tile diagonal, and the two tile passes of the
// transfer schedule (tiles with zero upwind-tile inflow storing only their
// outflow traces; tiles with their exact inflow storing only their cells).
enum DenseMode { kDenseClaim = 0, kDenseLevel = 1, kDenseZero = 2, kDenseFinal = 3 };
// Launch-mode flag: some family of the group has graded cells (an operator
// row per cell-size class); claimed and levelled modes only.
constexpr int kDenseGraded = 8;

// Dense sweep of n_tiles tiles (claim order `order`) in the given mode; for
// kDenseClaim the counter and the trace slots must be reset on entry.
hipError_t launch_dense_sweep(int prec, int mode, int np, int dim, const DenseTile *tiles, const int32_t *order,
                              int n_tiles, const DenseFam *fams, const DenseDesc *descs, const double *table,
                              int dt_idx, StateBuf f, const double *fb_old, const double *fb_new, uint64_t *traces,
                              int32_t *counter, DenseErr err, hipStream_t st);


}  // namespace pdg
