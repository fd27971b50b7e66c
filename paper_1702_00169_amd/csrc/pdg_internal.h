// Internal data structures shared by the host runtime (pdg_host.cpp) and the
// gfx950 kernels (pdg_kernels.hip).  Not part of the public ABI.
#pragma once

#include <stdint.h>

#include <hip/hip_runtime.h>

namespace pdg {

constexpr int kMaxNP = 5;       // d + 1 for degree <= 4
constexpr int kBlock = 256;     // threads per workgroup of every kernel
constexpr int kMaxNV = 27;
constexpr int kMaxM = 8;

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
  int32_t x_kind;      // 1: chains along the contiguous axis
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
constexpr int sweep_smax(int np) { return np <= 3 ? 8 : 4; }

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
  double param[4];     // advection: a_k; Euler: gamma
  double lambda;
  int32_t nv, m, dim, feq;
  int8_t axis[kMaxNV]; // velocity i = sign[i] * lambda * e_axis[i]
  int8_t sign[kMaxNV];
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
  int64_t per_comp;    // values per component
  int32_t relax_desc;
  int32_t vel;
};

// ---- kernel launchers (pdg_kernels.hip) ----------------------------------
enum Prec { kF64 = 0, kF32 = 1, kRefine = 2 };

hipError_t launch_invert(OpEntry *ops, int n_ops, hipStream_t st);

// Launch one sweep over items that share the node count np (any chain kind,
// tile shape or instance).
hipError_t launch_sweep(int prec, int np, const SweepItem *items, int n_items,
                        const SweepDesc *descs, const OpEntry *ops, int dt_idx, void *f, const double *fb_old,
                        const double *fb_new, double *stats, hipStream_t st);

// Relax / equilibrium launch for items whose instances share (nv, m).
hipError_t launch_relax(int prec, int nv, int m, const RelaxItem *items, int n_items, const RelaxDesc *descs,
                        void *f, double *w_out, const double *w_in, double omega, int mode, hipStream_t st);

hipError_t launch_inflow_eq(int nv, int m, const InflowDesc *items, int n_items, const RelaxDesc *descs,
                            const double *w_inflow, double *fb, hipStream_t st);

hipError_t launch_fill(double *p, int64_t n, double value, hipStream_t st);


}  // namespace pdg
