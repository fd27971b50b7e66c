// Host runtime of the PDG transport sweep + relaxation library (C ABI in
// include/pdg.h).
//
//  * setup (Sec. 4.1): per instance and velocity, the upwind dependency graph
//    of the Cartesian mesh (edge L -> R when the face normal n_LR has
//    n_LR . v > 0), its Kahn layering into levels, rejection of cycles, and the
//    grouping of cells into chains (lines along the velocity axis);
//  * prepare (Sec. 3.1-3.2): the one-dimensional cell blocks of eq. DG_reduit
//    built in binary64 from the Gauss-Lobatto rule, the device inversion, the
//    work items and launch groups of the sweep and relax kernels;
//  * run: sweeps, relaxations and step compositions, with the interior step
//    recorded once as a HIP graph and replayed.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/pdg.h"
#include "pdg_internal.h"

using namespace pdg;

// Scratch of pdg_transport_sweep_static, for callers that cannot allocate
// device memory: one copy per GPU, held until the process ends.  Host code
// never passes the array's name to a kernel (on the host it only stands for
// the symbol): its device address is taken per device with
// hipGetSymbolAddress and kept in g_scratch_ptr.
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};



struct Instance {
  pdg_instance_desc d;
  std::vector<double> v;     // nv * dim, physical velocities (equilibria, relaxation)
  // Transport works in the frame of the cell index axes: on box meshes that
  // is physical space (vt = v, ht = cell sizes); on an affine lattice of cell
  // edge vectors a_k it is the unit box mesh with velocity A^{-1} v and unit
  // cells (the cofactor of the affine cell map turns v into A^{-1} v in every
  // volume and face term of eq. DG_reduit).
  bool affine = false;
  double A[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // A[i][k]: component i of a_k
  std::vector<double> vt;    // nv * dim, transport-frame velocities
  double ht[3] = {1, 1, 1};  // transport-frame cell sizes (box meshes: h)
  std::vector<int> paxis, psign;  // per velocity: physical axis and sign ({+-lambda e_k} sets), -1/0 otherwise
  int64_t nc, nd, np;
  int64_t f_off, w_off, fb_off;
  std::vector<int64_t> fb_vel_off;  // per velocity, offset within the instance's fb block
  std::vector<int> axis;            // per velocity: axis of the velocity, -1 if not axis-aligned
  std::vector<int> sign;
  std::vector<int> ndep;            // per velocity: number of non-zero components
  std::vector<std::array<int, 3>> sgn;  // per velocity and axis: sign of the component (0 if zero)
  int nw = 0;                       // moments per node: m, or 3 for the D2Q9 model
  double lat_lambda = 0.0;          // D2Q9: lambda, velocity i = lambda (lat[i][0], lat[i][1])
  std::vector<std::array<int, 2>> lat;
  double h[3];
  int64_t n[3];
  bool graded[3] = {false, false, false};  // cell edges given along this axis
  std::vector<double> edge[3];             // graded axes: n[k] + 1 cell edges
};

struct Group {
  int np;                // node count of every item in the launch
  int64_t first, count;  // range in the item array
  bool graded;           // chains on graded axes (their own kernel)
  bool wpos = false;     // graded, and every tile width C a multiple of 64
};

// Fused collision + x transport launch group: items of one (d+1, nv, m, nx).
struct FusedGroup {
  int np, nv, m, nx;
  int64_t first, count;
};

struct RelaxGroup {
  int nv, m;
  int64_t first, count;
  int lattice;  // 1: D2Q9 lattice kernel, 0: {+-lambda e_k} kernel
};

// Dense launch group: tiles of one (d+1, D) kernel instantiation.
struct DenseGroup {
  int np, dim;
  int64_t first, count;  // tile range (tiles and claim order)
  int64_t sync_off;      // index of the group's tile-claim counter
  std::vector<int64_t> level;  // claim-order offsets where each tile diagonal starts (+ count)
  bool claim = false;          // one launch of claimed tiles (else one launch per tile diagonal)
  bool transfer_ok = false;    // two-dimensional, full tiles only, diagonals within the LDS limit
  bool transfer = false;       // transfer schedule: zero-inflow tiles, trace wavefront, final tiles
  int64_t tfam_first = 0, tfam_count = 0;  // its families in the transfer family list
  int tmax_diag = 0;                       // longest tile diagonal of those families
  bool graded = false;                     // some family has one operator row per cell-size class
};

// One (instance, velocity) family of chains and its launch class.
struct Family {
  int desc;                          // SweepDesc index
  int cls;                           // launch class index
  int np, x_kind, n_a, m;
  int64_t ntc;                       // chains per (component, transverse node)
  int64_t tnodes;                    // transverse node combinations
  std::vector<int64_t> plane_off;    // per transverse node: element offset of its plane
  int64_t f_vel;                     // element offset of (instance, v, k = 0, plane 0)
  int64_t comp_stride;               // Nd * Nc
  int64_t fb_vel;                    // fb offset of (instance, v, k = 0)
};

// Launch class: families sharing the node count (one kernel instantiation)
// and the chain kind (contiguous or strided axis) share one tile choice.
struct LaunchClass {
  int np, x_kind;
  int64_t chains;  // total chains of the class (all components, transverse nodes)
  int n_max;
  int C, S;        // x: C = rows per workgroup; strided: C chains, S = segment cap
  int group;       // launch group (np)
  int64_t first, count;  // item range
};

template <class T>
struct DevBuf {
  T *p = nullptr;
  size_t n = 0;
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    n = 0;
  }
  hipError_t upload(const std::vector<T> &h) {
    release();
    if (h.empty()) return hipSuccess;
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&p), h.size() * sizeof(T));
    if (e != hipSuccess) {
      p = nullptr;
      return e;
    }
    n = h.size();
    return hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice);
  }
};

}  // namespace

struct pdg_ctx {
  std::vector<Instance> inst;
  int64_t f_elems = 0, w_elems = 0, fb_elems = 0;
  // prepared state
  bool prepared = false;
  double dt = 0, theta = 0, omega = 0;
  int scheme = 0, prec = 0;
  std::vector<double> dts;  // prepared transport sub-steps; index = operator-table offset
  double tau = 0.0;         // relaxation time implied by (dt, omega)
  std::vector<OpEntry> ops_h;
  DevBuf<OpEntry> ops;
  DevBuf<SweepDesc> sdesc;
  DevBuf<SweepItem> sitems;
  std::vector<Group> groups;
  std::vector<Family> fams;
  std::vector<LaunchClass> classes;
  // dense path (velocities with two or three non-zero components)
  std::vector<DenseGroup> dgroups;
  DevBuf<DenseDesc> ddesc;
  DevBuf<DenseFam> dfams;
  DevBuf<DenseTile> dtiles;
  DevBuf<int32_t> dorder;
  DevBuf<double> dtable;
  DevBuf<uint64_t> dtraces;  // inflow-trace slots of the dense tiles (binary64 bits)
  DevBuf<int32_t> dsync;     // per group: tile-claim counter
  DevBuf<int32_t> dtfams;    // families of the transfer-schedule groups, group by group
  bool dense_claim = false;   // some dense group uses claimed tiles (their slots are reset per sweep)
  DevBuf<int32_t> derr;      // 1: a trace wait timed out, 2: claim counter overrun
  int32_t *herr = nullptr;   // host-visible copy of derr's codes (pinned, mapped)
  int32_t *herr_dev = nullptr;
  uint64_t wait_ticks = 100000000ull;  // dense trace wait bound (100 MHz ticks)
  DevBuf<RelaxDesc> rdesc;
  DevBuf<RelaxItem> ritems;
  std::vector<RelaxGroup> rgroups;
  DevBuf<InflowDesc> idesc;
  std::vector<RelaxGroup> igroups;  // (nv, m, first, count) over idesc
  DevBuf<double> stats;             // 2 doubles per sweep workgroup (and per mixed-launch workgroup after them)
  std::vector<int> item_cost;       // per item: its relative running time (longest first within a launch)
  bool mixed = false;               // one launch for the items of every node count (uniform meshes)
  DevBuf<SweepItem> smixed;         // those items, longest first
  // fused collision + x transport (the collapsed Strang step's C T pairs)
  bool fused = false;
  std::vector<FusedGroup> fgroups;  // (d+1, nv, m, nx, first, count) over fitems
  DevBuf<FusedDesc> fdesc;
  DevBuf<FusedItem> fitems;
  std::vector<int8_t> desc_x;       // per SweepDesc: chains along x (run in the fused pass)
  DevBuf<SweepItem> syz;            // sweep items of the other families, longest first
  const double *last_stats = nullptr;  // statistics written by the most recent sweep
  hipStream_t cap_stream = nullptr;
  // graph cache of the interior step
  hipGraphExec_t gexec = nullptr;
  void *g_f = nullptr;
  const double *g_fb = nullptr;
  bool stats_valid = false;
  hipStream_t last_stream = nullptr;

  void release_device() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
    g_f = nullptr;
    g_fb = nullptr;
    ops.release();
    sdesc.release();
    sitems.release();
    rdesc.release();
    ritems.release();
    idesc.release();
    ddesc.release();
    dfams.release();
    dtiles.release();
    dorder.release();
    dtable.release();
    dtraces.release();
    dsync.release();
    dtfams.release();
    derr.release();
    if (herr) (void)hipHostFree(herr);
    herr = nullptr;
    herr_dev = nullptr;
    dgroups.clear();
    stats.release();
    smixed.release();
    item_cost.clear();
    mixed = false;
    fused = false;
    fgroups.clear();
    fdesc.release();
    fitems.release();
    desc_x.clear();
    syz.release();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    cap_stream = nullptr;
    groups.clear();
    fams.clear();
    classes.clear();
    rgroups.clear();
    igroups.clear();
    prepared = false;
    stats_valid = false;
  }
};

namespace {

// ---------------------------------------------------------------------------
// one-dimensional Gauss-Lobatto rule (Sec. 3.1, eq. map_GL)
// ---------------------------------------------------------------------------
// Legendre P_k(x) by the three-term recurrence.
double legendre(int k, double x) {
  if (k == 0) return 1.0;
  double p0 = 1.0, p1 = x;
  for (int j = 2; j <= k; ++j) {
    const double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
    p0 = p1;
    p1 = p2;
  }
  return p1;
}

// Nodes: zeros of (1 - x^2) P_d'(x), found as the zeros of P_{d+1} - P_{d-1}
// (whose derivative is (2d+1) P_d) by Newton iteration from the
// Chebyshev-Lobatto points.  Weights 2 / (d (d+1) P_d(x)^2).
void gauss_lobatto(int d, std::vector<double> &x, std::vector<double> &w) {
  x.assign(d + 1, 0.0);
  w.assign(d + 1, 0.0);
  for (int j = 0; j <= d; ++j) {
    double t = -std::cos(M_PI * j / d);
    if (j > 0 && j < d) {
      for (int it = 0; it < 100; ++it) {
        const double fval = legendre(d + 1, t) - legendre(d - 1, t);
        const double dval = (2.0 * d + 1.0) * legendre(d, t);
        const double step = fval / dval;
        t -= step;
        if (std::fabs(step) < 1e-17) break;
      }
    }
    x[j] = t;
  }
  x[0] = -1.0;
  x[d] = 1.0;
  if (d % 2 == 0) x[d / 2] = 0.0;
  for (int j = 0; j <= d; ++j) {
    const double p = legendre(d, x[j]);
    w[j] = 2.0 / (d * (d + 1.0) * p * p);
  }
}

// Dm[a][b] = l_b'(x_a) by the barycentric formula:
// lam_b = 1 / prod_{k != b} (x_b - x_k); Dm[a][b] = (lam_b / lam_a) / (x_a - x_b) (a != b),
// Dm[a][a] = -sum_{b != a} Dm[a][b].
std::vector<double> derivative_matrix(const std::vector<double> &x) {
  const int n = (int)x.size();
  std::vector<double> lam(n, 1.0), dm(n * n, 0.0);
  for (int b = 0; b < n; ++b) {
    double prod = 1.0;
    for (int k = 0; k < n; ++k)
      if (k != b) prod *= x[b] - x[k];
    lam[b] = 1.0 / prod;
  }
  for (int a = 0; a < n; ++a) {
    double diag = 0.0;
    for (int b = 0; b < n; ++b) {
      if (a == b) continue;
      dm[a * n + b] = (lam[b] / lam[a]) / (x[a] - x[b]);
      diag -= dm[a * n + b];
    }
    dm[a * n + a] = diag;
  }
  return dm;
}

// One-dimensional block Gamma of eq. DG_reduit for speed V > 0 along the line
// and cell length h, in downwind-local node order (node 0 on the inflow face):
//   Gamma_ij = -(1/w_i) (2V/h) Dm[j][i] w_j              (volume term)
//            + delta_{i,NP-1} (1/w_{NP-1}) (2V/h)          (outflow face, (v.n)^+)
// and the inflow face coupling (1/w_0) (2V/h) (v.n)^- / V = -(2V/h)/w_0 at node 0.
void line_block(int d, double V, double h, std::vector<double> &gam, double &inflow_coef) {
  std::vector<double> x, w;
  gauss_lobatto(d, x, w);
  const std::vector<double> dm = derivative_matrix(x);
  const int np = d + 1;
  const double s = 2.0 * V / h;
  gam.assign(np * np, 0.0);
  for (int i = 0; i < np; ++i)
    for (int j = 0; j < np; ++j) gam[i * np + j] = -(s * dm[j * np + i] * w[j]) / w[i];
  gam[(np - 1) * np + (np - 1)] += s / w[np - 1];
  inflow_coef = s / w[0];  // magnitude of -(Gamma_{L<-R}) at node 0
}

// Cell block Gamma_{L<-L} of eq. DG_reduit for any constant velocity on a
// uniform Cartesian cell, in downwind-local tensor order (node index
// q = q_0 + NP q_1 + NP^2 q_2 with q_a = j_a if v_a >= 0 else NP-1-j_a, so
// q_a = 0 lies on the inflow face of every axis with v_a != 0).  On these
// cells the block is the Kronecker sum of the one-dimensional blocks of the
// non-zero components; kappa[a] is the inflow coupling magnitude of axis a
// (Gamma_{L<-R} = -kappa[a] at the inflow face nodes), 0 for v_a = 0.
void dense_block(int dim, int d, const double *v, const double *h, std::vector<double> &gam, double kappa[3]) {
  const int np = d + 1;
  int nd = 1;
  for (int k = 0; k < dim; ++k) nd *= np;
  gam.assign((size_t)nd * nd, 0.0);
  for (int a = 0; a < 3; ++a) kappa[a] = 0.0;
  int stride[3] = {1, np, np * np};
  for (int a = 0; a < dim; ++a) {
    if (v[a] == 0.0) continue;
    std::vector<double> g1;
    line_block(d, std::fabs(v[a]), h[a], g1, kappa[a]);
    for (int q = 0; q < nd; ++q) {
      const int qa = (q / stride[a]) % np;
      for (int qa2 = 0; qa2 < np; ++qa2) {
        const int q2 = q + (qa2 - qa) * stride[a];
        gam[(size_t)q * nd + q2] += g1[qa * np + qa2];
      }
    }
  }
}

bool is_finite(double x) { return std::isfinite(x); }

// Triple-jump coefficients of a fourth-order palindromic composition of a
// time-symmetric second-order step: g1 = 1/(2 - 2^(1/3)), g2 = 1 - 2 g1.
const double kTripleJump1 = 1.0 / (2.0 - std::cbrt(2.0));
const double kTripleJump2 = 1.0 - 2.0 / (2.0 - std::cbrt(2.0));

thread_local char g_detail[512] = "";

pdg_status from_hip_at(hipError_t e, const char *where) {
  if (e == hipSuccess) return PDG_OK;
  std::snprintf(g_detail, sizeof(g_detail), "%s: %s (%d)", where, hipGetErrorString(e), (int)e);
  if (e == hipErrorOutOfMemory) return PDG_ENOMEM;
  return PDG_EDEVICE;
}
#define from_hip(e) from_hip_at((e), __func__)
#define HIP_TRY(call)                                        \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) return from_hip_at(e_, #call);     \
  } while (0)

// ---------------------------------------------------------------------------
// dependency graph of a velocity on a Cartesian mesh and its Kahn layering
// ---------------------------------------------------------------------------
// Faces are axis-aligned, the scaled normal from L to its +e_k neighbour is
// a positive multiple of e_k, so the edge L -> L+e_k exists iff v_k > 0 and
// L+e_k -> L iff v_k < 0 (the same sign at every GL point of the face).
pdg_status mesh_levels(const Instance &in, int vel, std::vector<int32_t> &level) {
  const int dim = in.d.dim;
  const int64_t nc = in.nc;
  const double *v = &in.vt[(size_t)vel * dim];
  std::vector<int32_t> indeg(nc, 0);
  int64_t stride[3] = {1, in.n[0], in.n[0] * in.n[1]};
  auto coord = [&](int64_t c, int k) { return (c / stride[k]) % in.n[k]; };
  for (int64_t c = 0; c < nc; ++c)
    for (int k = 0; k < dim; ++k) {
      if (v[k] > 0 && coord(c, k) > 0) indeg[c]++;
      if (v[k] < 0 && coord(c, k) < in.n[k] - 1) indeg[c]++;
    }
  level.assign(nc, -1);
  std::vector<int64_t> frontier, next;
  for (int64_t c = 0; c < nc; ++c)
    if (indeg[c] == 0) frontier.push_back(c);
  int32_t lev = 0;
  int64_t done = 0;
  while (!frontier.empty()) {
    next.clear();
    for (int64_t c : frontier) {
      level[c] = lev;
      ++done;
      for (int k = 0; k < dim; ++k) {
        int64_t r = -1;
        if (v[k] > 0 && coord(c, k) < in.n[k] - 1) r = c + stride[k];
        if (v[k] < 0 && coord(c, k) > 0) r = c - stride[k];
        if (r >= 0 && --indeg[r] == 0) next.push_back(r);
      }
    }
    frontier.swap(next);
    ++lev;
  }
  return done == nc ? PDG_OK : PDG_ENOTDAG;
}

// ---------------------------------------------------------------------------
// tile choice of the sweep (lanes per chain group C, cells per segment S)
// ---------------------------------------------------------------------------
int pow2_ceil(int x) {
  int p = 1;
  while (p < x) p <<= 1;
  return p;
}

// Default tile of a launch class, from measured behaviour on gfx950: enough
// workgroups to fill the 256 CUs several times over, as much work per
// workgroup as that allows.  `PDG_TILE_X` / `PDG_TILE_Y` ("C,S") override it.
void default_tile(LaunchClass &k) {
  const int smax = class_smax(k.np, k.x_kind);
  if (k.x_kind == 1) {
    int C = 64;
    while (C > 1 && ((int64_t)C * k.n_max > 4096 || k.chains / C < 2048)) C >>= 1;
    while (C > 1 && (int64_t)C * k.n_max >= 65536) C >>= 1;
    k.C = C;
    k.S = 1;
  } else {
    int C = 64;
    while (C > 16 && k.chains / C < 4096) C >>= 1;
    k.C = C;
    k.S = smax;
  }
  const char *env = std::getenv(k.x_kind == 1 ? "PDG_TILE_X" : "PDG_TILE_Y");
  if (!env) env = std::getenv("PDG_TILE");
  int c2 = 0, s2 = 0;
  if (env && std::sscanf(env, "%d,%d", &c2, &s2) == 2 && c2 > 0 && c2 <= kBlock && s2 > 0 && s2 <= smax) {
    if (k.x_kind == 1) {
      k.C = c2;
      while (k.C > 1 && (int64_t)k.C * k.n_max >= 65536) k.C >>= 1;
    } else if (kBlock % c2 == 0) {
      k.C = c2;
      k.S = s2;
    }
  }
}

// Chains along the contiguous axis run in the row kernel (one cell per
// thread, tile S = 1) or, for tiles with S >= 2, in the segment mapping of the
// strided chains (thread (c, p) owns S consecutive cells of row c).
bool rows_mapping(const LaunchClass &k) { return k.x_kind == 1 && k.S == 1; }

// Segment length of a strided family under its class tile: the smallest
// power of two covering the chain in one window, capped by the class.
int family_S(const LaunchClass &k, int n_a) {
  if (rows_mapping(k)) return 1;
  const int P = kBlock / k.C;
  int S = 1;
  while (S < k.S && P * S < n_a) S <<= 1;
  return S;
}

// Work items of every class under the current tiles; longest-running
// workgroups first inside each launch, classes contiguous.
void build_items(pdg_ctx *c, std::vector<SweepItem> &items) {
  items.clear();
  c->item_cost.clear();
  std::vector<Group> groups;
  std::map<std::pair<int, bool>, int> group_of;
  for (LaunchClass &k : c->classes) {
    const std::pair<int, bool> key{k.np, k.x_kind == 2};
    if (!group_of.count(key)) {
      group_of[key] = (int)groups.size();
      groups.push_back(Group{k.np, 0, 0, key.second, key.second});
    }
    k.group = group_of[key];
    if (k.C % 64 != 0) groups[k.group].wpos = false;
  }
  for (size_t g = 0; g < groups.size(); ++g) {
    groups[g].first = (int64_t)items.size();
    for (LaunchClass &k : c->classes) {
      if (k.group != (int)g) continue;
      std::vector<std::pair<int, SweepItem>> list;
      for (const Family &fm : c->fams) {
        if (&c->classes[fm.cls] != &k) continue;
        const int C = k.C;
        const int S = family_S(k, fm.n_a);
        const bool rows = rows_mapping(k);
        const int cost = rows ? (int)((C * (int64_t)fm.n_a + kBlock - 1) / kBlock)
                              : ((fm.n_a + (kBlock / C) * S - 1) / ((kBlock / C) * S)) * S;
        for (int kk = 0; kk < fm.m; ++kk)
          for (int64_t t = 0; t < fm.tnodes; ++t) {
            const int64_t base = fm.f_vel + kk * fm.comp_stride + fm.plane_off[t];
            const int64_t fbb = fm.fb_vel + ((int64_t)kk * fm.tnodes + t) * fm.ntc;
            for (int64_t tau0 = 0; tau0 < fm.ntc; tau0 += C) {
              SweepItem item;
              item.base = base;
              item.fb = fbb + tau0;
              item.desc = fm.desc;
              item.tau0 = (int32_t)tau0;
              item.count = (int32_t)std::min<int64_t>(C, fm.ntc - tau0);
              item.C = (int16_t)(rows ? 0 : C);
              item.S = (int8_t)S;
              item.xk = (int8_t)(rows ? 1 : (fm.x_kind == 2 ? 2 : 0));
              list.push_back({cost, item});
            }
          }
      }
      std::stable_sort(list.begin(), list.end(),
                       [](const std::pair<int, SweepItem> &a, const std::pair<int, SweepItem> &b) {
                         return a.first > b.first;
                       });
      k.first = (int64_t)items.size();
      k.count = (int64_t)list.size();
      for (const auto &ci : list) {
        items.push_back(ci.second);
        c->item_cost.push_back(ci.first);
      }
    }
    groups[g].count = (int64_t)items.size() - groups[g].first;
  }
  c->groups = groups;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char *pdg_error_detail(void) { return g_detail; }

const char *pdg_status_string(pdg_status s) {
  switch (s) {
    case PDG_OK: return "PDG_OK";
    case PDG_EINVAL: return "PDG_EINVAL: invalid argument";
    case PDG_EUNSUPPORTED: return "PDG_EUNSUPPORTED: not supported by this build";
    case PDG_ENOTDAG: return "PDG_ENOTDAG: dependency graph has a cycle";
    case PDG_ESINGULAR: return "PDG_ESINGULAR: singular cell block";
    case PDG_ENOMEM: return "PDG_ENOMEM: out of memory";
    case PDG_EDEVICE: return "PDG_EDEVICE: HIP device error";
    case PDG_ESTATE: return "PDG_ESTATE: call out of order";
  }
  return "PDG_UNKNOWN";
}

static pdg_status topo_levels_impl(int32_t n_nodes, int64_t n_edges, const int32_t *src, const int32_t *dst,
                           int32_t *level) {
  if (n_nodes < 0 || n_edges < 0 || !level || (n_edges > 0 && (!src || !dst))) return PDG_EINVAL;
  std::vector<int32_t> indeg(n_nodes, 0);
  std::vector<int64_t> start(n_nodes + 1, 0);
  for (int64_t e = 0; e < n_edges; ++e) {
    if (src[e] < 0 || src[e] >= n_nodes || dst[e] < 0 || dst[e] >= n_nodes) return PDG_EINVAL;
    indeg[dst[e]]++;
    start[src[e] + 1]++;
  }
  for (int32_t i = 0; i < n_nodes; ++i) start[i + 1] += start[i];
  std::vector<int32_t> adj(n_edges);
  std::vector<int64_t> fill(start.begin(), start.end() - 1);
  for (int64_t e = 0; e < n_edges; ++e) adj[fill[src[e]]++] = dst[e];
  std::vector<int32_t> frontier, next;
  for (int32_t i = 0; i < n_nodes; ++i) {
    level[i] = -1;
    if (indeg[i] == 0) frontier.push_back(i);
  }
  int32_t lev = 0, done = 0;
  while (!frontier.empty()) {
    next.clear();
    for (int32_t i : frontier) {
      level[i] = lev;
      ++done;
      for (int64_t e = start[i]; e < start[i + 1]; ++e)
        if (--indeg[adj[e]] == 0) next.push_back(adj[e]);
    }
    frontier.swap(next);
    ++lev;
  }
  return done == n_nodes ? PDG_OK : PDG_ENOTDAG;
}

static pdg_status setup_mesh_impl(const pdg_instance_desc *descs, int32_t n_inst, pdg_ctx **out) {
  if (!descs || n_inst <= 0 || !out) return PDG_EINVAL;
  // owned here until handed to the caller (also on a std::bad_alloc)
  std::unique_ptr<pdg_ctx> c(new pdg_ctx());
  int64_t f_off = 0, w_off = 0, fb_off = 0;
  for (int32_t i = 0; i < n_inst; ++i) {
    const pdg_instance_desc &d = descs[i];
    Instance in;
    in.d = d;
    pdg_status err = PDG_OK;
    if (d.dim < 2 || d.dim > 3) err = PDG_EINVAL;
    else if (d.degree < 1 || d.nv < 1 || d.nv > kMaxNV || d.m < 1 || d.m > kMaxM || !d.v) err = PDG_EINVAL;
    if (err == PDG_OK && d.degree > 4) err = PDG_EUNSUPPORTED;
    // an affine lattice: some non-zero entry among the D x D cell edge vectors
    bool affine = false;
    for (int k = 0; k < d.dim && err == PDG_OK; ++k)
      for (int i = 0; i < d.dim; ++i) affine = affine || d.axes[3 * k + i] != 0.0;
    if (err == PDG_OK) {
      for (int k = 0; k < d.dim; ++k) {
        if (d.n[k] < 1) {
          err = PDG_EINVAL;
        } else if (affine) {
          // lattice from the corner lo; no graded edges, finite vectors
          if (d.edges[k] || !is_finite(d.lo[k])) err = PDG_EINVAL;
          for (int i = 0; i < d.dim; ++i)
            if (!is_finite(d.axes[3 * k + i])) err = PDG_EINVAL;
        } else if (d.edges[k]) {
          // graded axis: n[k] + 1 strictly increasing finite edges
          for (int i = 0; i <= d.n[k] && err == PDG_OK; ++i)
            if (!is_finite(d.edges[k][i]) || (i > 0 && !(d.edges[k][i] > d.edges[k][i - 1]))) err = PDG_EINVAL;
        } else if (!is_finite(d.lo[k]) || !is_finite(d.hi[k]) || !(d.hi[k] > d.lo[k])) {
          err = PDG_EINVAL;
        }
      }
    }
    if (err != PDG_OK) {
            return err;
    }
    in.d.v = nullptr;
    for (int k = 0; k < 3; ++k) {
      in.d.edges[k] = nullptr;
      if (k < d.dim && d.edges[k]) {
        in.graded[k] = true;
        in.edge[k].assign(d.edges[k], d.edges[k] + d.n[k] + 1);
        in.d.lo[k] = in.edge[k].front();
        in.d.hi[k] = in.edge[k].back();
      }
    }
    in.v.assign(d.v, d.v + (size_t)d.nv * d.dim);
    for (double x : in.v)
      if (!is_finite(x)) {
                return PDG_EINVAL;
      }
    // transport frame (see Instance) and physical axes of the velocities
    in.affine = affine;
    double ainv[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    if (affine) {
      for (int k = 0; k < d.dim; ++k)
        for (int i = 0; i < d.dim; ++i) in.A[i][k] = d.axes[3 * k + i];
      const double det = d.dim == 2 ? in.A[0][0] * in.A[1][1] - in.A[0][1] * in.A[1][0]
                                    : in.A[0][0] * (in.A[1][1] * in.A[2][2] - in.A[1][2] * in.A[2][1]) -
                                          in.A[0][1] * (in.A[1][0] * in.A[2][2] - in.A[1][2] * in.A[2][0]) +
                                          in.A[0][2] * (in.A[1][0] * in.A[2][1] - in.A[1][1] * in.A[2][0]);
      if (!(det > 0.0) || !is_finite(det)) return PDG_EINVAL;
      if (d.dim == 2) {
        ainv[0][0] = in.A[1][1] / det;
        ainv[0][1] = -in.A[0][1] / det;
        ainv[1][0] = -in.A[1][0] / det;
        ainv[1][1] = in.A[0][0] / det;
      } else {
        for (int i = 0; i < 3; ++i)
          for (int j = 0; j < 3; ++j) {
            // adjugate: cofactor of A[j][i]
            const int r0 = (j + 1) % 3, r1 = (j + 2) % 3, c0 = (i + 1) % 3, c1 = (i + 2) % 3;
            ainv[i][j] = (in.A[r0][c0] * in.A[r1][c1] - in.A[r0][c1] * in.A[r1][c0]) / det;
          }
      }
    }
    in.vt.assign(in.v.size(), 0.0);
    in.paxis.assign(d.nv, -1);
    in.psign.assign(d.nv, 0);
    for (int v = 0; v < d.nv; ++v) {
      int nzp = 0;
      for (int k = 0; k < d.dim; ++k) {
        double acc = 0.0;
        for (int i = 0; i < d.dim; ++i) acc += ainv[k][i] * in.v[(size_t)v * d.dim + i];
        in.vt[(size_t)v * d.dim + k] = affine ? acc : in.v[(size_t)v * d.dim + k];
        if (in.v[(size_t)v * d.dim + k] != 0.0) {
          ++nzp;
          in.paxis[v] = k;
          in.psign[v] = in.v[(size_t)v * d.dim + k] > 0 ? 1 : -1;
        }
      }
      if (nzp != 1) {
        in.paxis[v] = -1;
        in.psign[v] = 0;
      }
      if (affine) {
        // a component that is zero up to the rounding of A^{-1} v is zero: the
        // velocity then runs along index lines and keeps the line path
        double vmax = 0.0;
        for (int k = 0; k < d.dim; ++k) vmax = std::max(vmax, std::fabs(in.vt[(size_t)v * d.dim + k]));
        for (int k = 0; k < d.dim; ++k)
          if (std::fabs(in.vt[(size_t)v * d.dim + k]) <= 1e-13 * vmax) in.vt[(size_t)v * d.dim + k] = 0.0;
      }
    }
    in.nw = d.m;
    if (d.feq == PDG_FEQ_D2Q9) {
      // the D2Q9 lattice of Sec. 5.1: lambda x {0, +-e_x, +-e_y, (+-1, +-1)}, any order
      bool ok = d.dim == 2 && d.nv == 9 && d.m == 1;
      double lam = 0.0;
      for (int v = 0; v < d.nv && ok; ++v) lam = std::max(lam, std::fabs(in.v[(size_t)v * 2]));
      int seen[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};
      for (int v = 0; v < d.nv && ok && lam > 0.0; ++v) {
        std::array<int, 2> cc{0, 0};
        for (int k = 0; k < 2; ++k) {
          const double q = in.v[(size_t)v * 2 + k] / lam;
          if (q == 1.0) cc[k] = 1;
          else if (q == -1.0) cc[k] = -1;
          else if (q != 0.0) ok = false;
        }
        if (ok) seen[cc[0] + 1][cc[1] + 1]++;
        in.lat.push_back(cc);
      }
      for (int a = 0; a < 3 && ok; ++a)
        for (int b = 0; b < 3; ++b)
          if (seen[a][b] != 1) ok = false;
      if (!ok || !(lam > 0.0) || !is_finite(d.feq_param[0])) {
                return PDG_EINVAL;
      }
      in.lat_lambda = lam;
      in.nw = 3;
    }
    in.np = d.degree + 1;
    in.nd = 1;
    in.nc = 1;
    for (int k = 0; k < 3; ++k) {
      in.n[k] = k < d.dim ? d.n[k] : 1;
      in.h[k] = k < d.dim && !affine ? (d.hi[k] - d.lo[k]) / d.n[k] : 1.0;
      in.ht[k] = in.h[k];
    }
    for (int k = 0; k < d.dim; ++k) {
      in.nd *= in.np;
      in.nc *= in.n[k];
    }
    if (in.nc > (int64_t)1 << 31) {
            return PDG_EUNSUPPORTED;
    }
    in.axis.assign(d.nv, -1);
    in.sign.assign(d.nv, 0);
    in.ndep.assign(d.nv, 0);
    in.sgn.assign(d.nv, {0, 0, 0});
    in.fb_vel_off.assign(d.nv + 1, 0);
    int64_t fbo = 0;
    int64_t tnodes = 1;
    for (int k = 0; k < d.dim - 1; ++k) tnodes *= in.np;
    for (int v = 0; v < d.nv; ++v) {
      int nz = 0, ax = -1;
      for (int k = 0; k < d.dim; ++k) {
        const double comp = in.vt[(size_t)v * d.dim + k];
        if (comp != 0.0) {
          nz++;
          ax = k;
          in.sgn[v][k] = comp > 0 ? 1 : -1;
        }
      }
      in.ndep[v] = nz;
      if (nz == 1) {
        in.axis[v] = ax;
        in.sign[v] = in.sgn[v][ax];
      }
      // inflow data: one face block per non-zero component, [k][axis][t][tau]
      in.fb_vel_off[v] = fbo;
      for (int k = 0; k < d.dim; ++k)
        if (in.sgn[v][k] != 0) fbo += (int64_t)d.m * tnodes * (in.nc / in.n[k]);
      // the upwind dependency graph must be acyclic (Sec. 4.1)
      std::vector<int32_t> lev;
      pdg_status s = mesh_levels(in, v, lev);
      if (s != PDG_OK) {
                return s;
      }
      if (nz == 1) {
        // chains: the level of a cell is its downwind position along the axis
        int64_t stride = ax == 0 ? 1 : (ax == 1 ? in.n[0] : in.n[0] * in.n[1]);
        for (int64_t cc = 0; cc < in.nc; cc += std::max<int64_t>(1, in.nc / 997)) {
          int64_t pos = (cc / stride) % in.n[ax];
          int64_t want = in.sign[v] > 0 ? pos : in.n[ax] - 1 - pos;
          if (lev[cc] != want) {
                        return PDG_EDEVICE;  // internal inconsistency
          }
        }
      }
    }
    in.fb_vel_off[d.nv] = fbo;
    in.f_off = f_off;
    in.w_off = w_off;
    in.fb_off = fb_off;
    f_off += (int64_t)d.nv * d.m * in.nd * in.nc;
    w_off += (int64_t)in.nw * in.nd * in.nc;
    fb_off += fbo;
    c->inst.push_back(std::move(in));
  }
  c->f_elems = f_off;
  c->w_elems = w_off;
  c->fb_elems = fb_off;
  *out = c.release();
  return PDG_OK;
}

pdg_status pdg_layout(const pdg_ctx *c, int64_t *f_elems, int64_t *w_elems, int64_t *fb_elems,
                      int64_t *inst_f_offsets, int64_t *inst_w_offsets, int64_t *inst_fb_offsets) {
  if (!c) return PDG_EINVAL;
  if (f_elems) *f_elems = c->f_elems;
  if (w_elems) *w_elems = c->w_elems;
  if (fb_elems) *fb_elems = c->fb_elems;
  const size_t n = c->inst.size();
  for (size_t i = 0; i <= n; ++i) {
    if (inst_f_offsets) inst_f_offsets[i] = i < n ? c->inst[i].f_off : c->f_elems;
    if (inst_w_offsets) inst_w_offsets[i] = i < n ? c->inst[i].w_off : c->w_elems;
    if (inst_fb_offsets) inst_fb_offsets[i] = i < n ? c->inst[i].fb_off : c->fb_elems;
  }
  return PDG_OK;
}

static pdg_status node_coords_impl(const pdg_ctx *c, int32_t inst, double *vol_xyz, double *inflow_xyz) {
  if (!c || inst < 0 || inst >= (int32_t)c->inst.size()) return PDG_EINVAL;
  const Instance &in = c->inst[inst];
  const int dim = in.d.dim;
  const int np = (int)in.np;
  std::vector<double> x, w;
  gauss_lobatto(in.d.degree, x, w);
  // box meshes: coordinate along axis k; affine lattice: the index-frame
  // coordinate s_k (cell index plus the node's place in the cell), mapped to
  // physical space by phys() below
  auto pos = [&](int k, int64_t cell, int node) {
    if (in.affine) return (double)cell + 0.5 * (x[node] + 1.0);
    if (in.graded[k]) {
      const double a = in.edge[k][cell], b = in.edge[k][cell + 1];
      return a + 0.5 * (x[node] + 1.0) * (b - a);
    }
    return in.d.lo[k] + ((double)cell + 0.5 * (x[node] + 1.0)) * in.h[k];
  };
  auto phys = [&](int i, const double (&sk)[3]) {
    double acc = in.d.lo[i];
    for (int k = 0; k < dim; ++k) acc += in.A[i][k] * sk[k];
    return acc;
  };
  if (vol_xyz) {
    for (int k = 0; k < dim; ++k)
      for (int64_t j = 0; j < in.nd; ++j) {
        for (int64_t cc = 0; cc < in.nc; ++cc) {
          double sk[3] = {0, 0, 0};
          for (int k2 = 0; k2 < dim; ++k2) {
            const int jk = (int)((j / (int64_t)std::pow(np, k2)) % np);
            const int64_t stride = k2 == 0 ? 1 : (k2 == 1 ? in.n[0] : in.n[0] * in.n[1]);
            sk[k2] = pos(k2, (cc / stride) % in.n[k2], jk);
          }
          vol_xyz[((int64_t)k * in.nd + j) * in.nc + cc] = in.affine ? phys(k, sk) : sk[k];
        }
      }
  }
  if (inflow_xyz) {
    int64_t off = 0;
    for (int v = 0; v < in.d.nv; ++v)
    for (int ax = 0; ax < dim; ++ax) {
      if (in.sgn[v][ax] == 0) continue;
      int other[2], no = 0;
      for (int k = 0; k < dim; ++k)
        if (k != ax) other[no++] = k;
      const int64_t ntc = in.nc / in.n[ax];
      int64_t tnodes = 1;
      for (int k = 0; k < no; ++k) tnodes *= np;
      for (int k = 0; k < dim; ++k)
        for (int64_t t = 0; t < tnodes; ++t)
          for (int64_t tau = 0; tau < ntc; ++tau) {
            double sk[3] = {0, 0, 0};
            for (int k2 = 0; k2 < dim; ++k2) {
              if (k2 == ax) {
                // the domain face the velocity enters through
                sk[k2] = in.affine ? (in.sgn[v][ax] > 0 ? 0.0 : (double)in.n[ax])
                                   : (in.sgn[v][ax] > 0 ? in.d.lo[k2] : in.d.hi[k2]);
              } else {
                const int slot = (k2 == other[0]) ? 0 : 1;
                const int node = slot == 0 ? (int)(t % np) : (int)(t / np);
                const int64_t cell = slot == 0 ? tau % in.n[other[0]] : tau / in.n[other[0]];
                sk[k2] = pos(k2, cell, node);
              }
            }
            inflow_xyz[off + ((int64_t)k * tnodes + t) * ntc + tau] = in.affine ? phys(k, sk) : sk[k];
          }
      off += (int64_t)dim * tnodes * ntc;
    }
  }
  return PDG_OK;
}

static pdg_status levels_impl(const pdg_ctx *c, int32_t inst, int32_t vel, int32_t *level) {
  if (!c || !level || inst < 0 || inst >= (int32_t)c->inst.size()) return PDG_EINVAL;
  const Instance &in = c->inst[inst];
  if (vel < 0 || vel >= in.d.nv) return PDG_EINVAL;
  std::vector<int32_t> lev;
  pdg_status s = mesh_levels(in, vel, lev);
  if (s != PDG_OK) return s;
  std::memcpy(level, lev.data(), lev.size() * sizeof(int32_t));
  return PDG_OK;
}

pdg_status pdg_line_operator(const pdg_ctx *c, int32_t inst, int32_t vel, double *gamma, double *kappa) {
  if (!c || !gamma || !kappa || inst < 0 || inst >= (int32_t)c->inst.size()) return PDG_EINVAL;
  const Instance &in = c->inst[inst];
  if (vel < 0 || vel >= in.d.nv) return PDG_EINVAL;
  const int ax = in.axis[vel];
  if (ax < 0) return PDG_EUNSUPPORTED;
  std::vector<double> gam;
  // graded axis: the block of the chain's first (upwind-most) cell
  double h = in.ht[ax];
  if (in.graded[ax]) {
    const int64_t first = in.sign[vel] > 0 ? 0 : in.n[ax] - 1;
    h = in.edge[ax][first + 1] - in.edge[ax][first];
  }
  line_block(in.d.degree, std::fabs(in.vt[(size_t)vel * in.d.dim + ax]), h, gam, *kappa);
  std::memcpy(gamma, gam.data(), gam.size() * sizeof(double));
  return PDG_OK;
}

pdg_status pdg_cell_operator(const pdg_ctx *c, int32_t inst, int32_t vel, double *gamma, double *kappa) {
  if (!c || !gamma || !kappa || inst < 0 || inst >= (int32_t)c->inst.size()) return PDG_EINVAL;
  const Instance &in = c->inst[inst];
  if (vel < 0 || vel >= in.d.nv) return PDG_EINVAL;
  std::vector<double> gam;
  // graded axes: the sizes of the upwind-most cell
  double h[3] = {in.ht[0], in.ht[1], in.ht[2]};
  for (int a = 0; a < in.d.dim; ++a)
    if (in.graded[a]) {
      const int64_t first = in.sgn[vel][a] >= 0 ? 0 : in.n[a] - 1;
      h[a] = in.edge[a][(size_t)first + 1] - in.edge[a][(size_t)first];
    }
  dense_block(in.d.dim, in.d.degree, &in.vt[(size_t)vel * in.d.dim], h, gam, kappa);
  std::memcpy(gamma, gam.data(), gam.size() * sizeof(double));
  return PDG_OK;
}

}  // extern "C"

namespace {
pdg_status upload_items(pdg_ctx *c, const std::vector<SweepItem> &items);
}  // namespace

extern "C" {

static pdg_status prepare_impl(pdg_ctx *c, double dt, double theta, double omega, pdg_scheme scheme, pdg_precision prec,
                       void *stream) {
  if (!c) return PDG_EINVAL;
  if (!is_finite(dt) || dt == 0.0 || !is_finite(theta) || !(theta > 0.0) || theta > 1.0 || !is_finite(omega))
    return PDG_EINVAL;
  if (scheme < PDG_LIE || scheme > PDG_KIN4) return PDG_EINVAL;
  if (prec < PDG_FP64 || prec > PDG_FP32_REFINE_P48) return PDG_EINVAL;
  for (const Instance &in : c->inst)
    for (int v = 0; v < in.d.nv; ++v) {
      if (in.ndep[v] >= 2 && in.nd > kDenseMaxN) return PDG_EUNSUPPORTED;
    }
  hipStream_t st = static_cast<hipStream_t>(stream);
  c->release_device();

  // ---- transport sub-steps of the scheme (index 0: dt, 1: dt/2) ---------
  std::vector<double> dts = {dt, 0.5 * dt};
  if (scheme == PDG_KIN) dts.push_back(0.25 * dt);
  if (scheme == PDG_KIN4) {
    for (double g : {kTripleJump1, kTripleJump2}) {
      dts.push_back(0.25 * g * dt);
      dts.push_back(0.5 * g * dt);
    }
  }
  // collision over h: omega(h) = 2h / (2 tau + h), tau from omega over dt
  const double tau = omega == 2.0 ? 0.0 : dt * (2.0 - omega) / (2.0 * omega);
  if (!is_finite(tau)) return PDG_EINVAL;
  for (double h : dts)
    if (2.0 * tau + 0.5 * h == 0.0 || 2.0 * tau + h == 0.0) return PDG_EINVAL;

  // ---- operator table: (instance, velocity, dt_sub in dts) ---------------
  std::vector<OpEntry> ops;
  std::vector<SweepDesc> sdesc;
  std::vector<std::vector<int>> vel_desc(c->inst.size());  // (instance, velocity) -> SweepDesc, -1 if none
  std::vector<Family> fams;
  std::vector<LaunchClass> classes;
  for (size_t ii = 0; ii < c->inst.size(); ++ii) {
    const Instance &in = c->inst[ii];
    const int np = (int)in.np;
    const int dim = in.d.dim;
    for (int v = 0; v < in.d.nv; ++v) {
      if (in.ndep[v] != 1) continue;  // zero velocity: identity; two or more components: dense path
      const int ax = in.axis[v];
      const double V = std::fabs(in.vt[(size_t)v * dim + ax]);
      // one operator row per sub-step; on a graded axis one per sub-step
      // and downwind position (rows [dt_idx][l], l = 0 upwind-most)
      const bool graded = in.graded[ax];
      const int64_t npos = graded ? in.n[ax] : 1;
      const int op_index = (int)ops.size();  // + dt_idx (* n_a + l when graded)
      for (double ds : dts)
        for (int64_t l = 0; l < npos; ++l) {
          double h = in.ht[ax];
          if (graded) {
            const int64_t phys = in.sign[v] > 0 ? l : in.n[ax] - 1 - l;
            h = in.edge[ax][phys + 1] - in.edge[ax][phys];
          }
          std::vector<double> gam;
          double inflow = 0.0;
          line_block(in.d.degree, V, h, gam, inflow);
          OpEntry e;
          std::memset(&e, 0, sizeof(e));
          e.np = np;
          e.theta = theta;
          e.c0 = ds * inflow;
          for (int i = 0; i < np; ++i)
            for (int j = 0; j < np; ++j) {
              const double id = i == j ? 1.0 : 0.0;
              e.A[i * np + j] = id + theta * ds * gam[i * np + j];
              e.B[i * np + j] = id - (1.0 - theta) * ds * gam[i * np + j];
            }
          ops.push_back(e);
        }
      // chain addressing
      const int64_t nc = in.nc;
      const int64_t cstride = ax == 0 ? 1 : (ax == 1 ? in.n[0] : in.n[0] * in.n[1]);
      int64_t pstride = 1;
      for (int k = 0; k < ax; ++k) pstride *= np;
      pstride *= nc;
      SweepDesc sd;
      std::memset(&sd, 0, sizeof(sd));
      sd.n_a = (int32_t)in.n[ax];
      sd.cell_step = in.sign[v] > 0 ? cstride : -cstride;
      sd.cell0 = in.sign[v] > 0 ? 0 : (in.n[ax] - 1) * cstride;
      sd.plane_step = in.sign[v] > 0 ? pstride : -pstride;
      sd.plane0 = in.sign[v] > 0 ? 0 : (int64_t)(np - 1) * pstride;
      sd.op = op_index;
      sd.x_kind = graded ? 2 : (ax == 0 ? 1 : 0);
      if (ax == 0) {
        sd.nx = 1;
        sd.hi_stride = in.n[0];
      } else if (ax == 1) {
        sd.nx = (int32_t)in.n[0];
        sd.hi_stride = in.n[0] * in.n[1];
      } else {
        sd.nx = (int32_t)(in.n[0] * in.n[1]);
        sd.hi_stride = 0;
      }
      const int desc_index = (int)sdesc.size();
      sdesc.push_back(sd);
      if (vel_desc[ii].empty()) vel_desc[ii].assign(in.d.nv, -1);
      vel_desc[ii][v] = desc_index;
      Family fm;
      fm.desc = desc_index;
      fm.np = np;
      fm.x_kind = sd.x_kind;
      fm.n_a = sd.n_a;
      fm.m = in.d.m;
      fm.ntc = nc / in.n[ax];
      fm.tnodes = 1;
      for (int k = 0; k < dim - 1; ++k) fm.tnodes *= np;
      int other[2] = {0, 0}, no = 0;
      for (int k = 0; k < dim; ++k)
        if (k != ax) other[no++] = k;
      for (int64_t t = 0; t < fm.tnodes; ++t) {
        // transverse node t -> plane offset
        int64_t plane = 0;
        int64_t rem = t;
        for (int o = 0; o < no; ++o) {
          const int64_t jo = rem % np;
          rem /= np;
          int64_t ps = 1;
          for (int kk = 0; kk < other[o]; ++kk) ps *= np;
          plane += jo * ps;
        }
        fm.plane_off.push_back(plane * nc);
      }
      fm.comp_stride = in.nd * nc;
      fm.f_vel = in.f_off + (int64_t)v * in.d.m * in.nd * nc;
      fm.fb_vel = in.fb_off + in.fb_vel_off[v];
      fm.cls = -1;
      for (size_t k = 0; k < classes.size(); ++k)
        if (classes[k].np == np && classes[k].x_kind == sd.x_kind) fm.cls = (int)k;
      if (fm.cls < 0) {
        LaunchClass k;
        std::memset(&k, 0, sizeof(k));
        k.np = np;
        k.x_kind = sd.x_kind;
        fm.cls = (int)classes.size();
        classes.push_back(k);
      }
      classes[fm.cls].chains += (int64_t)fm.m * fm.tnodes * fm.ntc;
      classes[fm.cls].n_max = std::max(classes[fm.cls].n_max, fm.n_a);
      fams.push_back(std::move(fm));
    }
  }
  for (LaunchClass &k : classes) default_tile(k);
  c->fams = std::move(fams);
  c->classes = std::move(classes);
  std::vector<SweepItem> items;
  build_items(c, items);

  // ---- dense path tables -----------------------------------------------------
  std::vector<DenseDesc> ddesc;
  std::vector<std::pair<int, int>> ddshape;  // (np, dim) per descriptor
  std::vector<DenseFam> dfam;
  std::vector<DenseTile> dtile;
  std::vector<double> dtable;
  std::vector<int64_t> drow_off;
  std::vector<int32_t> drow_desc;
  std::vector<double> drow_c0;
  std::vector<std::pair<int, int>> dshape;  // (np, dim) per family
  int64_t trace_total = 0;
  for (size_t ii = 0; ii < c->inst.size(); ++ii) {
    const Instance &in = c->inst[ii];
    const int np = (int)in.np, dim = in.d.dim;
    const int N = (int)in.nd;
    int F = 1;
    for (int k = 0; k < dim - 1; ++k) F *= np;
    for (int v = 0; v < in.d.nv; ++v) {
      if (in.ndep[v] < 2) continue;
      DenseDesc dd;
      std::memset(&dd, 0, sizeof(dd));
      dd.nc = in.nc;
      dd.theta = theta;
      dd.trans_axis = -1;
      int64_t fboff = 0, tnodes = F;
      for (int a = 0; a < 3; ++a) {
        dd.n[a] = (int32_t)in.n[a];
        dd.sgn[a] = a < dim ? in.sgn[v][a] : 0;
        dd.T[a] = dd.sgn[a] == 0 ? 1 : (in.ndep[v] == 2 ? 8 : 4);
        if (a < dim && dd.sgn[a] == 0) dd.trans_axis = a;
        if (dd.sgn[a] != 0) {
          dd.fb_axis_off[a] = fboff;
          dd.fb_ntc[a] = in.nc / in.n[a];
          fboff += tnodes * dd.fb_ntc[a];
        }
      }
      const int64_t per_comp = fboff;
      // node planes in downwind-local order
      for (int q = 0; q < N; ++q) {
        int64_t j = 0, st2 = 1;
        int rem = q;
        for (int a = 0; a < dim; ++a) {
          const int qa = rem % np;
          rem /= np;
          const int ja = dd.sgn[a] < 0 ? np - 1 - qa : qa;
          j += ja * st2;
          st2 *= np;
        }
        dd.plane_off[q] = j * in.nc;
      }
      for (int a = 0; a < dim; ++a)
        for (int t = 0; t < F; ++t) {
          int q = 0, stride = 1, rem = t, tphys = 0, ps = 1;
          for (int b = 0; b < dim; ++b) {
            int qb;
            if (b == a) {
              qb = 0;
            } else {
              qb = rem % np;
              rem /= np;
              const int jb = dd.sgn[b] < 0 ? np - 1 - qb : qb;
              tphys += jb * ps;
              ps *= np;
            }
            q += qb * stride;
            stride *= np;
          }
          dd.face_q[a][t] = q;
          dd.fb_t[a][t] = tphys;
        }
      // operator rows: one per transport sub-step and cell-size class.  On a
      // graded axis with a non-zero component the block depends on the cell
      // size, so the distinct sizes of that axis are classes and a row is kept
      // for every combination of classes (nshape rows per sub-step).
      std::vector<double> hcls[3];
      std::vector<int32_t> cls_of[3];
      double hcell[3] = {in.ht[0], in.ht[1], in.ht[2]};
      int nshape = 1;
      for (int a = 0; a < 3; ++a) {
        dd.rank_off[a] = -1;
        dd.rank_stride[a] = 0;
        if (a >= dim || dd.sgn[a] == 0 || !in.graded[a]) continue;
        std::vector<double> hs((size_t)in.n[a]);
        for (int64_t i = 0; i < in.n[a]; ++i) hs[(size_t)i] = in.edge[a][(size_t)i + 1] - in.edge[a][(size_t)i];
        std::vector<double> u = hs;
        std::sort(u.begin(), u.end());
        u.erase(std::unique(u.begin(), u.end()), u.end());
        hcell[a] = u[0];
        if (u.size() == 1) continue;  // evenly spaced edges: one class
        cls_of[a].resize(hs.size());
        for (size_t i = 0; i < hs.size(); ++i)
          cls_of[a][i] = (int32_t)(std::lower_bound(u.begin(), u.end(), hs[i]) - u.begin());
        hcls[a] = u;
        dd.rank_stride[a] = nshape;
        nshape *= (int)u.size();
      }
      dd.nshape = nshape;
      std::vector<std::vector<double>> gams((size_t)nshape);
      std::vector<std::array<double, 3>> kaps((size_t)nshape);
      for (int sh = 0; sh < nshape; ++sh) {
        double h[3] = {hcell[0], hcell[1], hcell[2]};
        for (int a = 0; a < 3; ++a)
          if (!hcls[a].empty()) h[a] = hcls[a][(size_t)(sh / dd.rank_stride[a]) % hcls[a].size()];
        dense_block(dim, in.d.degree, &in.vt[(size_t)v * dim], h, gams[(size_t)sh], kaps[(size_t)sh].data());
      }
      // 2D velocities with two non-zero components on uniform cells also keep
      // the transfer operator of a full tile (2TF x 2TF, T = 8)
      const int64_t nr = 2LL * 8 * F;
      const int64_t stride_row =
          4LL * N * N + 3LL * N * F + (N * N + 1) / 2 + (dim == 2 && nshape == 1 ? nr * nr : 0);
      dd.op_off = (int64_t)dtable.size();
      dd.op_stride = stride_row;
      const int desc_index = (int)ddesc.size();
      for (double ds : dts)
        for (int sh = 0; sh < nshape; ++sh) {
          const std::vector<double> &gam = gams[(size_t)sh];
          const int64_t off = (int64_t)dtable.size();
          dtable.resize(dtable.size() + stride_row, 0.0);
          for (int i = 0; i < N; ++i)
            for (int j = 0; j < N; ++j) {
              const double id = i == j ? 1.0 : 0.0;
              dtable[off + (int64_t)N * N + 3LL * N * F + i * N + j] = id + theta * ds * gam[(size_t)i * N + j];
              dtable[off + 2LL * N * N + 3LL * N * F + i * N + j] = id - (1.0 - theta) * ds * gam[(size_t)i * N + j];
            }
          drow_off.push_back(off);
          drow_desc.push_back(desc_index);
          for (int a = 0; a < 3; ++a) drow_c0.push_back(ds * kaps[(size_t)sh][a]);
        }
      // size class of every cell coordinate along the graded axes
      for (int a = 0; a < 3; ++a)
        if (!cls_of[a].empty()) {
          dd.rank_off[a] = (int64_t)dtable.size();
          for (int32_t k : cls_of[a]) dtable.push_back((double)k);
        }
      ddesc.push_back(dd);
      ddshape.push_back({np, dim});
      // families (component x transverse slice) and their tiles
      const int nslice = dd.trans_axis >= 0 ? (int)in.n[dd.trans_axis] : 1;
      int ntile[3];
      for (int a = 0; a < 3; ++a) ntile[a] = dd.sgn[a] == 0 ? 1 : (int)((in.n[a] + dd.T[a] - 1) / dd.T[a]);
      int slot = 0;  // doubles per axis slot: largest tile face x F
      for (int a = 0; a < dim; ++a) {
        if (dd.sgn[a] == 0) continue;
        int cells = 1;
        for (int b = 0; b < dim; ++b)
          if (b != a && dd.sgn[b] != 0) cells *= dd.T[b];
        slot = std::max(slot, cells * F);
      }
      for (int k = 0; k < in.d.m; ++k)
        for (int sl = 0; sl < nslice; ++sl) {
          DenseFam fmd;
          fmd.f_base = in.f_off + (int64_t)(v * in.d.m + k) * in.nd * in.nc;
          fmd.fb_base = in.fb_off + in.fb_vel_off[v] + (int64_t)k * per_comp;
          fmd.desc = desc_index;
          fmd.slice = sl;
          fmd.tile0 = (int32_t)dtile.size();  // global for now; group-local after sorting
          fmd.nt[0] = ntile[0];
          fmd.nt[1] = ntile[1];
          fmd.pad = 0;
          const int fam_index = (int)dfam.size();
          dfam.push_back(fmd);
          dshape.push_back({np, dim});
          const int64_t tile0 = (int64_t)dtile.size();
          for (int t2 = 0; t2 < ntile[2]; ++t2)
            for (int t1 = 0; t1 < ntile[1]; ++t1)
              for (int t0 = 0; t0 < ntile[0]; ++t0) {
                DenseTile tl;
                std::memset(&tl, 0, sizeof(tl));
                tl.fam = fam_index;
                tl.tc[0] = t0;
                tl.tc[1] = t1;
                tl.tc[2] = t2;
                tl.slot = slot;
                tl.trace_off = trace_total;
                trace_total += 3LL * slot;
                const int tcs[3] = {t0, t1, t2};
                const int tstr[3] = {1, ntile[0], ntile[0] * ntile[1]};
                const int64_t me = tile0 + t0 + (int64_t)ntile[0] * (t1 + (int64_t)ntile[1] * t2);
                for (int a = 0; a < 3; ++a) {
                  tl.up[a] = (dd.sgn[a] != 0 && tcs[a] > 0) ? (int32_t)(me - tstr[a]) : -1;
                  tl.down[a] = (dd.sgn[a] != 0 && tcs[a] + 1 < ntile[a]) ? (int32_t)(me + tstr[a]) : -1;
                }
                dtile.push_back(tl);
              }
        }
    }
  }
  // launch groups by (d+1, D); claim order: tiles by diagonal, so every tile's
  // upwind tiles are claimed before it
  std::vector<DenseTile> dtile_sorted;
  std::vector<int32_t> dorder;
  std::vector<DenseGroup> dgroups;
  std::vector<int32_t> tfam;  // families of transfer-eligible groups
  int64_t sync_total = 0;
  {
    std::map<std::pair<int, int>, std::vector<int64_t>> by_shape;
    for (size_t i = 0; i < dtile.size(); ++i) by_shape[dshape[dtile[i].fam]].push_back((int64_t)i);
    std::vector<int64_t> new_index(dtile.size(), -1);
    for (auto &kv : by_shape) {
      DenseGroup g;
      g.np = kv.first.first;
      g.dim = kv.first.second;
      g.first = (int64_t)dtile_sorted.size();
      g.count = (int64_t)kv.second.size();
      g.sync_off = sync_total;
      sync_total += 1;
      for (int64_t i : kv.second) {
        new_index[i] = (int64_t)dtile_sorted.size() - g.first;  // index within the group
        dtile_sorted.push_back(dtile[i]);
      }
      dgroups.push_back(g);
    }
    // remap neighbour indices to group-local indices, build claim orders
    for (DenseGroup &g : dgroups) {
      std::vector<std::pair<int, int32_t>> diag;
      for (int64_t i = 0; i < g.count; ++i) {
        DenseTile &tl = dtile_sorted[g.first + i];
        for (int a = 0; a < 3; ++a) {
          if (tl.up[a] >= 0) tl.up[a] = (int32_t)new_index[tl.up[a]];
          if (tl.down[a] >= 0) tl.down[a] = (int32_t)new_index[tl.down[a]];
        }
        diag.push_back({tl.tc[0] + tl.tc[1] + tl.tc[2], (int32_t)i});
      }
      std::stable_sort(diag.begin(), diag.end(),
                       [](const std::pair<int, int32_t> &x, const std::pair<int, int32_t> &y) { return x.first < y.first; });
      for (size_t k = 0; k < diag.size(); ++k) {
        if (k == 0 || diag[k].first != diag[k - 1].first) g.level.push_back((int64_t)k);
        dorder.push_back(diag[k].second);
      }
      g.level.push_back(g.count);
    }
    // families: group-local first tile; transfer eligibility per group (every
    // family two-dimensional with full 8 x 8 tiles and diagonals of at most
    // kTransferMaxDiag tiles)
    std::vector<int> fam_group(dfam.size(), -1);
    for (size_t gi = 0; gi < dgroups.size(); ++gi) dgroups[gi].transfer_ok = dgroups[gi].dim == 2;
    for (size_t fi = 0; fi < dfam.size(); ++fi) {
      DenseFam &fmd = dfam[fi];
      const int64_t t0 = fmd.tile0;
      for (size_t gi = 0; gi < dgroups.size(); ++gi)
        if (new_index[t0] >= 0 && dshape[fi] == std::make_pair(dgroups[gi].np, dgroups[gi].dim)) {
          fam_group[fi] = (int)gi;
          break;
        }
      fmd.tile0 = (int32_t)new_index[t0];
      const DenseDesc &dd = ddesc[fmd.desc];
      const int gi = fam_group[fi];
      if (gi < 0) continue;
      const bool full = dd.n[0] % 8 == 0 && dd.n[1] % 8 == 0 && dd.sgn[0] != 0 && dd.sgn[1] != 0;
      // one transfer operator per (velocity, sub-step): uniform cells only
      if (!full || dd.nshape > 1 || std::min(fmd.nt[0], fmd.nt[1]) > 64) dgroups[gi].transfer_ok = false;
      if (dd.nshape > 1) dgroups[gi].graded = true;
      dgroups[gi].tmax_diag = std::max(dgroups[gi].tmax_diag, std::min(fmd.nt[0], fmd.nt[1]));
    }
    for (size_t gi = 0; gi < dgroups.size(); ++gi) {
      dgroups[gi].tfam_first = (int64_t)tfam.size();
      if (dgroups[gi].transfer_ok)
        for (size_t fi = 0; fi < dfam.size(); ++fi)
          if (fam_group[fi] == (int)gi) tfam.push_back((int32_t)fi);
      dgroups[gi].tfam_count = (int64_t)tfam.size() - dgroups[gi].tfam_first;
    }
  }

  // ---- relax tables --------------------------------------------------------
  std::vector<RelaxDesc> rdesc;
  // items grouped by kernel: (lattice, nv, m)
  std::map<std::array<int, 3>, std::vector<RelaxItem>> ritems_by;
  std::vector<InflowDesc> idesc_all;
  std::map<std::array<int, 3>, std::vector<InflowDesc>> iby;
  bool relax_ok = true;
  int64_t w_inflow_off = 0;
  for (size_t ii = 0; ii < c->inst.size(); ++ii) {
    const Instance &in = c->inst[ii];
    RelaxDesc rd;
    std::memset(&rd, 0, sizeof(rd));
    rd.f_base = in.f_off;
    rd.w_base = in.w_off;
    rd.nodes = in.nd * in.nc;
    for (int k = 0; k < 4; ++k) rd.param[k] = in.d.feq_param[k];
    rd.nv = in.d.nv;
    rd.m = in.d.m;
    rd.dim = in.d.dim;
    rd.feq = in.d.feq;
    const int lattice = in.d.feq == PDG_FEQ_D2Q9 ? 1 : 0;
    bool ok = true;
    if (lattice) {
      // validated at setup
      rd.lambda = in.lat_lambda;
      for (int v = 0; v < 9; ++v) {
        rd.cx[v] = (int8_t)in.lat[v][0];
        rd.cy[v] = (int8_t)in.lat[v][1];
      }
    } else {
      // the equilibrium needs the full {+-lambda e_k} set
      ok = in.d.nv == 2 * in.d.dim;
      for (int v = 0; v < in.d.nv; ++v)
        if (in.paxis[v] < 0) ok = false;
      const double lam = ok ? std::fabs(in.v[(size_t)0 * in.d.dim + in.paxis[0]]) : 0.0;
      int seen[3][2] = {{0, 0}, {0, 0}, {0, 0}};
      for (int v = 0; v < in.d.nv && ok; ++v) {
        const double sp = std::fabs(in.v[(size_t)v * in.d.dim + in.paxis[v]]);
        if (sp != lam) ok = false;
        rd.axis[v] = (int8_t)in.paxis[v];
        rd.sign[v] = (int8_t)in.psign[v];
        seen[in.paxis[v]][in.psign[v] > 0]++;
      }
      for (int k = 0; k < in.d.dim && ok; ++k)
        if (seen[k][0] != 1 || seen[k][1] != 1) ok = false;
      if (in.d.feq == PDG_FEQ_EULER && in.d.m != in.d.dim + 2) ok = false;
      if (in.d.feq != PDG_FEQ_EULER && in.d.feq != PDG_FEQ_ADVECTION) ok = false;
      rd.lambda = lam;
    }
    if (!ok) relax_ok = false;
    const int di = (int)rdesc.size();
    rdesc.push_back(rd);
    const std::array<int, 3> key{lattice, rd.nv, rd.m};
    const int64_t chunk = 4 * kBlock;
    for (int64_t n0 = 0; n0 < rd.nodes; n0 += chunk) {
      RelaxItem it;
      it.node0 = n0;
      it.desc = di;
      it.count = (int32_t)std::min<int64_t>(chunk, rd.nodes - n0);
      ritems_by[key].push_back(it);
    }
    // inflow points of every velocity; w_inflow holds nw moments per point
    for (int v = 0; v < in.d.nv; ++v) {
      InflowDesc idd;
      idd.per_comp = (in.fb_vel_off[v + 1] - in.fb_vel_off[v]) / in.d.m;
      idd.fb_base = in.fb_off + in.fb_vel_off[v];
      idd.w_base = w_inflow_off;
      idd.relax_desc = di;
      idd.vel = v;
      w_inflow_off += (int64_t)in.nw * idd.per_comp;
      if (idd.per_comp > 0) iby[key].push_back(idd);
    }
  }
  std::vector<RelaxItem> ritems;
  std::vector<RelaxGroup> rgroups, igroups;
  if (relax_ok) {
    for (auto &kv : ritems_by) {
      rgroups.push_back(RelaxGroup{kv.first[1], kv.first[2], (int64_t)ritems.size(), (int64_t)kv.second.size(),
                                   kv.first[0]});
      ritems.insert(ritems.end(), kv.second.begin(), kv.second.end());
    }
    for (auto &kv : iby) {
      igroups.push_back(RelaxGroup{kv.first[1], kv.first[2], (int64_t)idesc_all.size(), (int64_t)kv.second.size(),
                                   kv.first[0]});
      idesc_all.insert(idesc_all.end(), kv.second.begin(), kv.second.end());
    }
  }

  // ---- fused collision + x transport -------------------------------------
  // Opt-in (PDG_FUSED=1 at prepare): measured slower than the separate
  // collision and sweep passes on the 3D Euler workload (the pass holds a
  // row's d+1 nodes and all n_v m values per node, so fewer waves fit a CU).
  // Every instance: the {+-lambda e_k} velocity set of the relaxation on a
  // box mesh with uniform cells, rows short enough for one workgroup, node
  // offsets within 32 bits; otherwise the step keeps separate passes.
  std::vector<FusedDesc> fdesc_h;
  std::vector<FusedItem> fitems_h;
  std::vector<FusedGroup> fgroups_h;
  const char *fenv = std::getenv("PDG_FUSED");
  bool fused = relax_ok && dgroups.empty() && fenv && std::strcmp(fenv, "1") == 0;
  for (size_t ii = 0; ii < c->inst.size() && fused; ++ii) {
    const Instance &in = c->inst[ii];
    const int dim = in.d.dim;
    bool ok = in.d.feq != PDG_FEQ_D2Q9 && !in.affine && (int)vel_desc[ii].size() == in.d.nv &&
              fused_supported((int)in.np, in.d.nv, in.d.m, (int)in.n[0]) && in.nd * in.nc < ((int64_t)1 << 31);
    for (int a = 0; a < dim && ok; ++a) ok = !in.graded[a];
    int vx[2] = {-1, -1};
    for (int v = 0; v < in.d.nv && ok; ++v) {
      if (in.ndep[v] != 1 || vel_desc[ii][v] < 0) ok = false;
      else if (in.axis[v] == 0) vx[in.sign[v] > 0 ? 0 : 1] = v;
    }
    if (!ok || vx[0] < 0 || vx[1] < 0) {
      fused = false;
      break;
    }
    FusedDesc fd;
    std::memset(&fd, 0, sizeof(fd));
    fd.nc = in.nc;
    fd.rdesc = (int32_t)ii;
    fd.nx = (int32_t)in.n[0];
    fd.ntau = (int32_t)(in.nc / in.n[0]);
    fd.tnodes = 1;
    for (int k = 0; k < dim - 1; ++k) fd.tnodes *= (int32_t)in.np;
    for (int h = 0; h < 2; ++h) {
      fd.vx[h] = vx[h];
      fd.fb[h] = in.fb_off + in.fb_vel_off[vx[h]];
      fd.op[h] = sdesc[vel_desc[ii][vx[h]]].op;
    }
    fdesc_h.push_back(fd);
  }
  if (fused) {
    std::map<std::array<int, 4>, std::vector<FusedItem>> fby;
    for (size_t ii = 0; ii < c->inst.size(); ++ii) {
      const Instance &in = c->inst[ii];
      const FusedDesc &fd = fdesc_h[ii];
      const std::array<int, 4> key{(int)in.np, in.d.nv, in.d.m, fd.nx};
      for (int64_t r = 0; r < (int64_t)fd.tnodes * fd.ntau; ++r) {
        FusedItem fi;
        fi.desc = (int32_t)ii;
        fi.row0 = (int32_t)r;
        fby[key].push_back(fi);
      }
    }
    for (auto &kv : fby) {
      fgroups_h.push_back(FusedGroup{kv.first[0], kv.first[1], kv.first[2], kv.first[3], (int64_t)fitems_h.size(),
                                     (int64_t)kv.second.size()});
      fitems_h.insert(fitems_h.end(), kv.second.begin(), kv.second.end());
    }
  }
  c->fused = fused;
  c->fgroups = fgroups_h;
  c->desc_x.assign(sdesc.size(), 0);
  for (size_t k = 0; k < sdesc.size(); ++k) c->desc_x[k] = sdesc[k].x_kind == 1 ? 1 : 0;

  // ---- upload + device inversion ----------------------------------------
  hipError_t e;
#define PREP_TRY(call)                      \
  if ((e = (call)) != hipSuccess) {         \
    c->release_device();                    \
    return from_hip_at(e, #call);           \
  }
  PREP_TRY(c->ops.upload(ops))
  PREP_TRY(c->sdesc.upload(sdesc))
  PREP_TRY(c->rdesc.upload(rdesc))
  PREP_TRY(c->ritems.upload(ritems))
  PREP_TRY(c->idesc.upload(idesc_all))
  PREP_TRY(c->fdesc.upload(fdesc_h))
  PREP_TRY(c->fitems.upload(fitems_h))
  {
    const pdg_status us = upload_items(c, items);  // items, the mixed launch's order, statistics
    if (us != PDG_OK) {
      c->release_device();
      return us;
    }
  }
  PREP_TRY(launch_invert(c->ops.p, (int)ops.size(), st))
  PREP_TRY(hipStreamSynchronize(st))
  c->ops_h.resize(ops.size());
  PREP_TRY(hipMemcpy(c->ops_h.data(), c->ops.p, ops.size() * sizeof(OpEntry), hipMemcpyDeviceToHost))
  for (const OpEntry &o : c->ops_h)
    if (o.singular) {
      c->release_device();
      return PDG_ESINGULAR;
    }
  // dense path: tables, tiles, and the device inversion of the dense blocks
  PREP_TRY(c->ddesc.upload(ddesc))
  PREP_TRY(c->dfams.upload(dfam))
  PREP_TRY(c->dtiles.upload(dtile_sorted))
  PREP_TRY(c->dorder.upload(dorder))
  PREP_TRY(c->dtfams.upload(tfam))
  PREP_TRY(c->dtable.upload(dtable))
  PREP_TRY(c->dtraces.upload(std::vector<uint64_t>((size_t)trace_total, kDenseTraceEmpty)))
  PREP_TRY(c->dsync.upload(std::vector<int32_t>((size_t)sync_total, 0)))
  PREP_TRY(c->derr.upload(std::vector<int32_t>(1, 0)))
  PREP_TRY(hipHostMalloc(reinterpret_cast<void **>(&c->herr), sizeof(int32_t), hipHostMallocMapped))
  *c->herr = 0;
  PREP_TRY(hipHostGetDevicePointer(reinterpret_cast<void **>(&c->herr_dev), c->herr, 0))
  {
    // device address of this GPU's static scratch (once per device)
    int dev = 0;
    PREP_TRY(hipGetDevice(&dev))
    if (dev >= 0 && dev < kMaxDevices) {
      std::lock_guard<std::mutex> lock(g_scratch_mu);
      if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        PREP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)))
        g_scratch_ptr[dev] = ptr;
      }
    }
  }
  {
    // the dense trace wait bound; PDG_DENSE_WAIT_TICKS overrides it (tests of
    // the failure report use a bound of zero ticks)
    const char *wt = std::getenv("PDG_DENSE_WAIT_TICKS");
    c->wait_ticks = wt ? std::strtoull(wt, nullptr, 10) : 100000000ull;
  }
  if (!drow_off.empty()) {
    std::map<std::pair<int, int>, std::vector<size_t>> rows_by_shape;
    for (size_t r = 0; r < drow_off.size(); ++r) {
      rows_by_shape[ddshape[drow_desc[r]]].push_back(r);
    }
    for (auto &kv : rows_by_shape) {
      const int np2 = kv.first.first, dim2 = kv.first.second;
      const int n2 = dim2 == 2 ? np2 * np2 : np2 * np2 * np2;
      const int F2 = dim2 == 2 ? np2 : np2 * np2;
      std::vector<int64_t> ro;
      std::vector<int32_t> rd;
      std::vector<double> rc;
      for (size_t r : kv.second) {
        ro.push_back(drow_off[r]);
        rd.push_back(drow_desc[r]);
        for (int a = 0; a < 3; ++a) rc.push_back(drow_c0[3 * r + a]);
      }
      DevBuf<int64_t> d_ro;
      DevBuf<int32_t> d_rd, d_fl;
      DevBuf<double> d_rc;
      PREP_TRY(d_ro.upload(ro))
      PREP_TRY(d_rd.upload(rd))
      PREP_TRY(d_rc.upload(rc))
      PREP_TRY(d_fl.upload(std::vector<int32_t>(ro.size(), 0)))
      PREP_TRY(launch_dense_invert(c->dtable.p, d_ro.p, c->ddesc.p, d_rd.p, d_rc.p, d_fl.p, (int)ro.size(), n2, F2, st))
      // transfer operators of full tiles (two-dimensional velocities), from
      // the blocks just inverted
      if (dim2 == 2)
        PREP_TRY(launch_dense_transfer_operator(np2, c->dtable.p, d_ro.p, c->ddesc.p, d_rd.p, (int)ro.size(), st))
      PREP_TRY(hipStreamSynchronize(st))
      std::vector<int32_t> fl(ro.size());
      PREP_TRY(hipMemcpy(fl.data(), d_fl.p, fl.size() * sizeof(int32_t), hipMemcpyDeviceToHost))
      d_ro.release();
      d_rd.release();
      d_rc.release();
      d_fl.release();
      for (int32_t x : fl)
        if (x) {
          c->release_device();
          return PDG_ESINGULAR;
        }
    }
  }
  c->dgroups = dgroups;
  PREP_TRY(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking))
#undef PREP_TRY
  c->rgroups = rgroups;
  c->igroups = igroups;
  c->dt = dt;
  c->theta = theta;
  c->omega = omega;
  c->dts = dts;
  c->tau = tau;
  c->scheme = scheme;
  c->prec = prec;
  // Dense-tile schedule per launch group: the transfer schedule (three
  // launches that never wait: tiles with zero upwind inflow, the trace
  // wavefront on MFMA, tiles with their exact inflow) for two-dimensional
  // groups whose families all have full tiles; otherwise claimed tiles (one
  // launch, traces handed over between running tiles) except for the 8-node
  // cells of 3D degree 1, whose 4 x 4 x 4 tiles finish faster than a
  // hand-over through the device-scope atomics (measured on 2D and 3D
  // meshes), so one launch per tile diagonal serves them better.
  // PDG_DENSE_SCHEDULE=level, claim or transfer forces one schedule (transfer
  // only where a group allows it).
  {
    const char *ds = std::getenv("PDG_DENSE_SCHEDULE");
    const bool force_level = ds && std::strcmp(ds, "level") == 0;
    const bool force_claim = ds && std::strcmp(ds, "claim") == 0;
    c->dense_claim = false;
    for (DenseGroup &g : c->dgroups) {
      g.transfer = g.transfer_ok && !force_level && !force_claim;
      g.claim = !g.transfer && (force_claim || (!force_level && !(g.dim == 3 && g.np == 2)));
      c->dense_claim = c->dense_claim || g.claim;
    }
  }
  c->prepared = true;
  return PDG_OK;
}

}  // extern "C"

namespace {

DenseErr dense_err(const pdg_ctx *c) { return DenseErr{c->derr.p, c->herr_dev, c->wait_ticks}; }

// A dense-sweep failure already reported by a finished kernel (host-visible
// flag, read without synchronising): the state is invalid until the caller
// has seen it through pdg_sync_status, so the entry points refuse to go on.
bool dense_failed(const pdg_ctx *c) {
  if (!c->herr || *static_cast<volatile const int32_t *>(c->herr) == 0) return false;
  std::snprintf(g_detail, sizeof(g_detail), "%s",
                "dense sweep: an earlier sweep reported a failed trace wait; call pdg_sync_status");
  return true;
}

// Device scratch of one sweep: per-workgroup refinement statistics (2 doubles
// per work item), the dense inflow-trace slots and the tile-claim counters.
struct SweepScratch {
  double *stats;
  uint64_t *traces;
  int32_t *sync;
};

SweepScratch ctx_scratch(pdg_ctx *c) { return SweepScratch{c->stats.p, c->dtraces.p, c->dsync.p}; }

pdg_status do_sweep(pdg_ctx *c, void *f, const double *fb_old, const double *fb_new, int dt_idx,
                    hipStream_t st, const SweepScratch &sc) {
  if (c->mixed) {
    hipError_t e = launch_sweep_mixed(c->prec, c->smixed.p, (int)c->smixed.n, c->sdesc.p, c->ops.p, dt_idx,
                                      StateBuf{f, c->f_elems}, fb_old, fb_new, sc.stats + 2 * c->sitems.n, st);
    if (e != hipSuccess) return from_hip_at(e, "launch_sweep_mixed");
  }
  for (const Group &g : c->groups) {
    if (c->mixed && !g.graded) continue;
    hipError_t e = launch_sweep(c->prec, g.np, g.graded, g.wpos, c->sitems.p + g.first, (int)g.count, c->sdesc.p, c->ops.p, dt_idx, StateBuf{f, c->f_elems},
                                fb_old, fb_new, sc.stats + 2 * g.first, st);
    if (e != hipSuccess) {
      char what[96];
      std::snprintf(what, sizeof(what), "launch_sweep(np=%d,items=%lld)", g.np, (long long)g.count);
      return from_hip_at(e, what);
    }
  }
  if (c->dense_claim) {
    // every trace slot empty, every claim counter at zero (fill kernels, so
    // that the sequence can be captured into a graph)
    hipError_t e = launch_fill_u64(sc.traces, c->dtraces.n, kDenseTraceEmpty, st);
    if (e == hipSuccess) e = launch_fill_int(sc.sync, (int64_t)c->dgroups.size(), 0, st);
    if (e != hipSuccess) return from_hip_at(e, "dense sweep reset");
  }
  for (const DenseGroup &g : c->dgroups) {
    if (g.transfer) {
      // zero-inflow tiles (their outflow traces Z into the downwind slots), the
      // trace wavefront (slots: Z -> exact traces), tiles with exact inflow
      hipError_t e = launch_dense_sweep(c->prec, kDenseZero, g.np, g.dim, c->dtiles.p + g.first, c->dorder.p + g.first,
                                        (int)g.count, c->dfams.p, c->ddesc.p, c->dtable.p, dt_idx,
                                        StateBuf{f, c->f_elems}, fb_old, fb_new, sc.traces, sc.sync + g.sync_off,
                                        dense_err(c), st);
      if (e == hipSuccess)
        e = launch_dense_transfer(g.np, g.tmax_diag, c->dtiles.p + g.first, c->dfams.p, c->dtfams.p + g.tfam_first,
                                  (int)g.tfam_count, c->ddesc.p, c->dtable.p, dt_idx, sc.traces, st);
      if (e == hipSuccess)
        e = launch_dense_sweep(c->prec, kDenseFinal, g.np, g.dim, c->dtiles.p + g.first, c->dorder.p + g.first,
                               (int)g.count, c->dfams.p, c->ddesc.p, c->dtable.p, dt_idx, StateBuf{f, c->f_elems},
                               fb_old, fb_new, sc.traces, sc.sync + g.sync_off, dense_err(c), st);
      if (e != hipSuccess) return from_hip_at(e, "dense transfer schedule");
      continue;
    }
    if (!g.claim) {
      // one launch per tile diagonal: no tile ever waits
      for (size_t k = 0; k + 1 < g.level.size(); ++k) {
        hipError_t e = launch_dense_sweep(c->prec, kDenseLevel | (g.graded ? kDenseGraded : 0), g.np, g.dim,
                                          c->dtiles.p + g.first,
                                          c->dorder.p + g.first + g.level[k], (int)(g.level[k + 1] - g.level[k]),
                                          c->dfams.p, c->ddesc.p, c->dtable.p, dt_idx, StateBuf{f, c->f_elems}, fb_old, fb_new,
                                          sc.traces, sc.sync + g.sync_off, dense_err(c), st);
        if (e != hipSuccess) return from_hip_at(e, "launch_dense_sweep(level)");
      }
      continue;
    }
    hipError_t e = launch_dense_sweep(c->prec, kDenseClaim | (g.graded ? kDenseGraded : 0), g.np, g.dim,
                                      c->dtiles.p + g.first, c->dorder.p + g.first,
                                      (int)g.count, c->dfams.p, c->ddesc.p, c->dtable.p, dt_idx, StateBuf{f, c->f_elems}, fb_old, fb_new,
                                      sc.traces, sc.sync + g.sync_off, dense_err(c), st);
    if (e != hipSuccess) return from_hip_at(e, "launch_dense_sweep");
  }
  c->stats_valid = c->prec == PDG_FP32_REFINE || c->prec == PDG_FP32_REFINE_P48;
  c->last_stats = sc.stats;
  c->last_stream = st;
  return PDG_OK;
}

// The node-local part of a composition: S(h_pre) C(omega) S(h_post) (Sec. 3.2).
// The source terms act only on instances with a source (D2Q9 with gravity);
// with source_only the collision-only instances are left alone.
pdg_status do_local(pdg_ctx *c, void *f, double *w_out, double omega, double h_pre, double h_post,
                    bool source_only, hipStream_t st) {
  if (c->rgroups.empty()) return PDG_EUNSUPPORTED;
  for (const RelaxGroup &g : c->rgroups) {
    hipError_t e;
    if (g.lattice)
      e = launch_lattice(c->prec, c->ritems.p + g.first, (int)g.count, c->rdesc.p, StateBuf{f, c->f_elems}, w_out, nullptr, omega, h_pre,
                         h_post, 0, st);
    else if (source_only)
      e = hipSuccess;
    else
      e = launch_relax(c->prec, g.nv, g.m, c->ritems.p + g.first, (int)g.count, c->rdesc.p, StateBuf{f, c->f_elems}, w_out, nullptr,
                       omega, 0, st);
    if (e != hipSuccess) return from_hip(e);
  }
  return PDG_OK;
}

// The collision with factor omega followed by the transport sweep of
// sub-step dt_idx, as the fused pass (collision + chains along x) and the
// sweep of the other families.
pdg_status do_fused(pdg_ctx *c, void *f, const double *fb, int dt_idx, double omega, hipStream_t st) {
  const size_t off_yz = 2 * (c->sitems.n + c->smixed.n);
  const size_t off_f = off_yz + 2 * c->syz.n;
  for (const FusedGroup &g : c->fgroups) {
    hipError_t e = launch_relax_xsweep(c->prec, g.np, g.nv, g.m, g.nx, c->fitems.p + g.first, (int)g.count, c->fdesc.p,
                                       c->rdesc.p, c->ops.p, dt_idx, StateBuf{f, c->f_elems}, fb, fb, omega,
                                       c->stats.p + off_f + 2 * g.first, st);
    if (e != hipSuccess) return from_hip_at(e, "launch_relax_xsweep");
  }
  hipError_t e = launch_sweep_mixed(c->prec, c->syz.p, (int)c->syz.n, c->sdesc.p, c->ops.p, dt_idx,
                                    StateBuf{f, c->f_elems}, fb, fb, c->stats.p + off_yz, st);
  if (e != hipSuccess) return from_hip_at(e, "launch_sweep_mixed (fused step)");
  c->stats_valid = c->prec == PDG_FP32_REFINE || c->prec == PDG_FP32_REFINE_P48;
  c->last_stats = c->stats.p;
  c->last_stream = st;
  return PDG_OK;
}

struct StepOp {
  int kind;       // 0: transport sweep, 1: node-local step S(h_pre) C(omega) S(h_post), 2: C(omega) then
                  // the sweep (fused pass)
  int dt_idx;     // sweep: index into the prepared sub-steps
  double omega;   // relaxation factor
  double h_pre;   // source sub-steps around the collision
  double h_post;
};

pdg_status run_ops(pdg_ctx *c, const std::vector<StepOp> &ops, void *f, const double *fb, hipStream_t st) {
  for (const StepOp &o : ops) {
    const pdg_status s = o.kind == 0   ? do_sweep(c, f, fb, fb, o.dt_idx, st, ctx_scratch(c))
                         : o.kind == 2 ? do_fused(c, f, fb, o.dt_idx, o.omega, st)
                                       : do_local(c, f, nullptr, o.omega, o.h_pre, o.h_post, false, st);
    if (s != PDG_OK) return s;
  }
  return PDG_OK;
}

}  // namespace

extern "C" {

pdg_status pdg_transport_sweep(pdg_ctx *c, void *f, const double *fb_old, const double *fb_new, double dt_sub,
                               void *stream) {
  if (!c || !f || (c->fb_elems > 0 && (!fb_old || !fb_new))) return PDG_EINVAL;
  if (!c->prepared) return PDG_ESTATE;
  if (dense_failed(c)) return PDG_EDEVICE;
  int dt_idx = -1;
  for (size_t i = 0; i < c->dts.size(); ++i)
    if (dt_sub == c->dts[i]) {
      dt_idx = (int)i;
      break;
    }
  if (dt_idx < 0) return PDG_ESTATE;
  return do_sweep(c, f, fb_old, fb_new, dt_idx, static_cast<hipStream_t>(stream), ctx_scratch(c));
}

pdg_status pdg_transport_sweep_static(pdg_ctx *c, void *f, const double *fb_old, const double *fb_new,
                                      double dt_sub, void *stream) {
  if (!c || !f || (c->fb_elems > 0 && (!fb_old || !fb_new))) return PDG_EINVAL;
  if (!c->prepared) return PDG_ESTATE;
  if (dense_failed(c)) return PDG_EDEVICE;
  int dt_idx = -1;
  for (size_t i = 0; i < c->dts.size(); ++i)
    if (dt_sub == c->dts[i]) {
      dt_idx = (int)i;
      break;
    }
  if (dt_idx < 0) return PDG_ESTATE;
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  void *base = (dev >= 0 && dev < kMaxDevices) ? g_scratch_ptr[dev] : nullptr;
  if (!base) {
    std::snprintf(g_detail, sizeof(g_detail), "pdg_transport_sweep_static: no static scratch on device %d "
                  "(prepare the context on this device)", dev);
    return PDG_ESTATE;
  }
  // [stats: 2 doubles per work item][trace slots][claim counters], 256-byte aligned parts
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t b_stats = up(2 * (c->sitems.n + c->smixed.n) * sizeof(double));
  const size_t b_traces = up(c->dtraces.n * sizeof(uint64_t));
  const size_t b_sync = up(c->dgroups.size() * sizeof(int32_t));
  if (b_stats + b_traces + b_sync > kStaticScratchBytes) {
    std::snprintf(g_detail, sizeof(g_detail), "pdg_transport_sweep_static: this problem needs %zu bytes of "
                  "scratch, the static scratch holds %zu", b_stats + b_traces + b_sync, kStaticScratchBytes);
    return PDG_EUNSUPPORTED;
  }
  unsigned char *p = static_cast<unsigned char *>(base);
  const SweepScratch sc{reinterpret_cast<double *>(p), reinterpret_cast<uint64_t *>(p + b_stats),
                        reinterpret_cast<int32_t *>(p + b_stats + b_traces)};
  return do_sweep(c, f, fb_old, fb_new, dt_idx, static_cast<hipStream_t>(stream), sc);
}

pdg_status pdg_relax(pdg_ctx *c, void *f, double *w_out, void *stream) {
  if (!c || !f) return PDG_EINVAL;
  if (!c->prepared) return PDG_ESTATE;
  if (dense_failed(c)) return PDG_EDEVICE;
  return do_local(c, f, w_out, c->omega, 0.0, 0.0, false, static_cast<hipStream_t>(stream));
}

pdg_status pdg_source(pdg_ctx *c, void *f, double h, void *stream) {
  if (!c || !f || !is_finite(h)) return PDG_EINVAL;
  if (!c->prepared) return PDG_ESTATE;
  if (dense_failed(c)) return PDG_EDEVICE;
  if (h == 0.0) return PDG_OK;
  return do_local(c, f, nullptr, 0.0, h, 0.0, true, static_cast<hipStream_t>(stream));
}

pdg_status pdg_equilibrium(pdg_ctx *c, const double *w, void *f, void *stream) {
  if (!c || !w || !f) return PDG_EINVAL;
  if (!c->prepared) return PDG_ESTATE;
  if (c->rgroups.empty()) return PDG_EUNSUPPORTED;
  for (const RelaxGroup &g : c->rgroups) {
    hipError_t e = g.lattice ? launch_lattice(c->prec, c->ritems.p + g.first, (int)g.count, c->rdesc.p, StateBuf{f, c->f_elems}, nullptr,
                                              w, 1.0, 0.0, 0.0, 1, static_cast<hipStream_t>(stream))
                             : launch_relax(c->prec, g.nv, g.m, c->ritems.p + g.first, (int)g.count, c->rdesc.p, StateBuf{f, c->f_elems},
                                            nullptr, w, 1.0, 1, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return from_hip(e);
  }
  return PDG_OK;
}

pdg_status pdg_state_to_f64(pdg_ctx *c, const void *f, double *x, void *stream) {
  if (!c || !f || !x) return PDG_EINVAL;
  if (!c->prepared) return PDG_ESTATE;
  const hipError_t e = launch_convert(c->prec, StateBuf{const_cast<void *>(f), c->f_elems}, x, true,
                                      static_cast<hipStream_t>(stream));
  return e == hipSuccess ? PDG_OK : from_hip_at(e, "launch_convert");
}

pdg_status pdg_state_from_f64(pdg_ctx *c, const double *x, void *f, void *stream) {
  if (!c || !f || !x) return PDG_EINVAL;
  if (!c->prepared) return PDG_ESTATE;
  const hipError_t e = launch_convert(c->prec, StateBuf{f, c->f_elems}, const_cast<double *>(x), false,
                                      static_cast<hipStream_t>(stream));
  return e == hipSuccess ? PDG_OK : from_hip_at(e, "launch_convert");
}

pdg_status pdg_inflow_equilibrium(pdg_ctx *c, const double *w_inflow, double *fb, void *stream) {
  if (!c || !w_inflow || !fb) return PDG_EINVAL;
  if (!c->prepared) return PDG_ESTATE;
  if (c->igroups.empty()) return PDG_EUNSUPPORTED;
  for (const RelaxGroup &g : c->igroups) {
    hipError_t e = g.lattice ? launch_lattice_inflow(c->idesc.p + g.first, (int)g.count, c->rdesc.p, w_inflow, fb,
                                                     static_cast<hipStream_t>(stream))
                             : launch_inflow_eq(g.nv, g.m, c->idesc.p + g.first, (int)g.count, c->rdesc.p, w_inflow,
                                                fb, static_cast<hipStream_t>(stream));
    if (e != hipSuccess) return from_hip(e);
  }
  return PDG_OK;
}

static pdg_status step_impl(pdg_ctx *c, void *f, const double *fb, int32_t n_steps, void *stream) {
  if (!c || !f || n_steps < 0 || (c->fb_elems > 0 && !fb)) return PDG_EINVAL;
  if (!c->prepared) return PDG_ESTATE;
  if (c->rgroups.empty()) return PDG_EUNSUPPORTED;
  if (dense_failed(c)) return PDG_EDEVICE;
  if (n_steps == 0) return PDG_OK;
  hipStream_t st = static_cast<hipStream_t>(stream);
  // prologue, interior (repeated), epilogue: sweeps by sub-step index, relaxations by omega
  std::vector<StepOp> pro, body, epi;
  int reps = n_steps;
  const double w = c->omega;
  auto om = [c](double h) { return c->tau == 0.0 ? 2.0 : 2.0 * h / (2.0 * c->tau + h); };
  // With a source every collision C(h) becomes S(a) C(h) S(b) (Sec. 3.2, Sec. 5.1):
  // Lie T(dt) S(dt) C(dt); Strang T(dt/2) S(dt/2) C(dt) S(dt/2) T(dt/2); each
  // C(h/2) of M_2^kin(h) becomes S(h/4) C(h/2) S(h/4).  Without a source the
  // source fractions are ignored.
  const double dt = c->dt;
  switch (c->scheme) {
    case PDG_LIE: body = {{0, 0, 0.0, 0.0, 0.0}, {1, 0, w, dt, 0.0}}; break;
    case PDG_STRANG: body = {{0, 1, 0.0, 0.0, 0.0}, {1, 0, w, 0.5 * dt, 0.5 * dt}, {0, 1, 0.0, 0.0, 0.0}}; break;
    case PDG_STRANG_COLLAPSED:
      // T(dt/2) C [T(dt) C]^(N-1) T(dt/2), or with the fused passes
      // T(dt/2) [C T(dt)]^(N-1) C T(dt/2)
      if (c->fused) {
        pro = {{0, 1, 0.0, 0.0, 0.0}};
        body = {{2, 0, w, 0.0, 0.0}};
        epi = {{2, 1, w, 0.0, 0.0}};
      } else {
        pro = {{0, 1, 0.0, 0.0, 0.0}, {1, 0, w, 0.5 * dt, 0.5 * dt}};
        body = {{0, 0, 0.0, 0.0, 0.0}, {1, 0, w, 0.5 * dt, 0.5 * dt}};
        epi = {{0, 1, 0.0, 0.0, 0.0}};
      }
      reps = n_steps - 1;
      break;
    case PDG_KIN: {
      // M_2^kin(dt) = T(dt/4) C(dt/2) T(dt/2) C(dt/2) T(dt/4)
      const double wc = om(0.5 * dt), q = 0.25 * dt;
      body = {{0, 2, 0.0, 0.0, 0.0}, {1, 0, wc, q, q}, {0, 1, 0.0, 0.0, 0.0}, {1, 0, wc, q, q}, {0, 2, 0.0, 0.0, 0.0}};
      break;
    }
    case PDG_KIN4: {
      // M_2^kin(g1 dt) M_2^kin(g2 dt) M_2^kin(g1 dt); sub-steps 2..5 = g1/4, g1/2, g2/4, g2/2
      const double g[3] = {kTripleJump1, kTripleJump2, kTripleJump1};
      const int q[3] = {2, 4, 2};
      for (int j = 0; j < 3; ++j) {
        const double wc = om(0.5 * g[j] * dt), hq = 0.25 * g[j] * dt;
        body.push_back({0, q[j], 0.0, 0.0, 0.0});
        body.push_back({1, 0, wc, hq, hq});
        body.push_back({0, q[j] + 1, 0.0, 0.0, 0.0});
        body.push_back({1, 0, wc, hq, hq});
        body.push_back({0, q[j], 0.0, 0.0, 0.0});
      }
      break;
    }
    default: return PDG_ESTATE;
  }
  pdg_status s;
  if ((s = run_ops(c, pro, f, fb, st)) != PDG_OK) return s;
  if (reps > 0) {
    const bool use_graph = std::getenv("PDG_NO_GRAPH") == nullptr;
    if (use_graph && (c->gexec == nullptr || c->g_f != f || c->g_fb != fb)) {
      if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
      c->gexec = nullptr;
      hipGraph_t graph = nullptr;
      hipError_t e = hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal);
      if (e != hipSuccess) return from_hip_at(e, "hipStreamBeginCapture");
      pdg_status s2 = run_ops(c, body, f, fb, c->cap_stream);
      e = hipStreamEndCapture(c->cap_stream, &graph);
      if (s2 != PDG_OK) {
        if (graph) (void)hipGraphDestroy(graph);
        return s2;
      }
      if (e != hipSuccess) return from_hip_at(e, "hipStreamEndCapture");
      e = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
      (void)hipGraphDestroy(graph);
      if (e != hipSuccess) {
        c->gexec = nullptr;
        return from_hip_at(e, "hipGraphInstantiate");
      }
      c->g_f = f;
      c->g_fb = fb;
    }
    for (int32_t i = 0; i < reps; ++i) {
      if (use_graph) {
        hipError_t e = hipGraphLaunch(c->gexec, st);
        if (e != hipSuccess) return from_hip_at(e, "hipGraphLaunch");
      } else if ((s = run_ops(c, body, f, fb, st)) != PDG_OK) {
        return s;
      }
    }
    c->stats_valid = c->prec == PDG_FP32_REFINE || c->prec == PDG_FP32_REFINE_P48;
    c->last_stats = c->stats.p;
    c->last_stream = st;
  }
  return run_ops(c, epi, f, fb, st);
}

namespace {

// Re-upload the item array after a tile change; grows the per-workgroup
// statistics buffer if needed and drops the cached step graph.
pdg_status upload_items(pdg_ctx *c, const std::vector<SweepItem> &items) {
  hipError_t e = c->sitems.upload(items);
  if (e != hipSuccess) return from_hip_at(e, "upload items");
  // the mixed launch: every uniform-mesh item, longest first across node counts
  int n_uniform_groups = 0;
  for (const Group &g : c->groups) n_uniform_groups += g.graded ? 0 : 1;
  const char *mx = std::getenv("PDG_SWEEP_MIXED");
  c->mixed = n_uniform_groups >= 2 && !(mx && std::strcmp(mx, "0") == 0);
  std::vector<SweepItem> mixed_items;
  if (c->mixed) {
    std::vector<std::pair<int, int64_t>> order;
    for (const Group &g : c->groups)
      if (!g.graded)
        for (int64_t i = g.first; i < g.first + g.count; ++i) order.push_back({c->item_cost[i], i});
    std::stable_sort(order.begin(), order.end(),
                     [](const std::pair<int, int64_t> &a, const std::pair<int, int64_t> &b) { return a.first > b.first; });
    for (const auto &o : order) mixed_items.push_back(items[o.second]);
  }
  e = c->smixed.upload(mixed_items);
  if (e != hipSuccess) return from_hip_at(e, "upload mixed items");
  // the fused step's sweep: every family not along x in one launch, longest first
  std::vector<SweepItem> yz_items;
  if (c->fused) {
    std::vector<std::pair<int, int64_t>> order;
    for (size_t i = 0; i < items.size(); ++i)
      if (!c->desc_x[items[i].desc]) order.push_back({c->item_cost[i], (int64_t)i});
    std::stable_sort(order.begin(), order.end(),
                     [](const std::pair<int, int64_t> &a, const std::pair<int, int64_t> &b) { return a.first > b.first; });
    for (const auto &o : order) yz_items.push_back(items[o.second]);
  }
  e = c->syz.upload(yz_items);
  if (e != hipSuccess) return from_hip_at(e, "upload fused-step sweep items");
  // statistics: [items | mixed items | fused-step sweep items | fused items]
  const size_t n_stats = 2 * (items.size() + mixed_items.size() + yz_items.size() + c->fitems.n);
  if (c->stats.n < std::max<size_t>(2, n_stats)) {
    std::vector<double> zeros(std::max<size_t>(2, n_stats), 0.0);
    e = c->stats.upload(zeros);
    if (e != hipSuccess) return from_hip_at(e, "upload stats");
  }
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  c->gexec = nullptr;
  c->g_f = nullptr;
  c->g_fb = nullptr;
  return PDG_OK;
}

bool tile_valid(const LaunchClass &k, int C, int S) {
  if (C < 1 || C > kBlock || S < 1 || S > class_smax(k.np, k.x_kind)) return false;
  if (k.x_kind == 1 && S == 1) return (int64_t)C * k.n_max < 65536;
  return kBlock % C == 0;
}

}  // namespace

static pdg_status autotune_impl(pdg_ctx *c, void *f, const double *fb, int32_t reps, void *stream) {
  if (!c || !f || (c->fb_elems > 0 && !fb) || reps < 1) return PDG_EINVAL;
  if (!c->prepared) return PDG_ESTATE;
  c->stats_valid = false;  // the work items change below
  hipStream_t st = static_cast<hipStream_t>(stream);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  std::vector<SweepItem> items;
  pdg_status status = PDG_OK;
  for (size_t ki = 0; ki < c->classes.size() && status == PDG_OK; ++ki) {
    LaunchClass &k = c->classes[ki];
    std::vector<std::pair<int, int>> cands;
    if (k.x_kind == 1) {
      for (int C = 1; C <= 64; C <<= 1) cands.push_back({C, 1});
      // the segment mapping too: rows of C lanes' chains, S cells per thread
      for (int C = 8; C <= 64; C <<= 1)
        for (int S = 2; S <= class_smax(k.np, k.x_kind); S <<= 1) cands.push_back({C, S});
    } else {
      for (int C = 8; C <= 64; C <<= 1)
        for (int S = 1; S <= class_smax(k.np, k.x_kind); S <<= 1) cands.push_back({C, S});
    }
    int bestC = k.C, bestS = k.S;
    float best = 1e30f;
    for (const auto &cs : cands) {
      if (!tile_valid(k, cs.first, cs.second)) continue;
      k.C = cs.first;
      k.S = cs.second;
      build_items(c, items);
      if ((status = upload_items(c, items)) != PDG_OK) break;
      const Group &g = c->groups[k.group];
      hipError_t e = hipSuccess;
      for (int r = 0; r <= reps && e == hipSuccess; ++r) {
        if (r == 1) e = hipEventRecord(e0, st);
        if (e == hipSuccess)
          e = launch_sweep(c->prec, g.np, g.graded, g.wpos, c->sitems.p + k.first, (int)k.count, c->sdesc.p, c->ops.p, 0, StateBuf{f, c->f_elems}, fb, fb,
                           c->stats.p + 2 * k.first, st);
      }
      if (e == hipSuccess) e = hipEventRecord(e1, st);
      if (e == hipSuccess) e = hipEventSynchronize(e1);
      float ms = 0.f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
      if (e != hipSuccess) {
        status = from_hip_at(e, "autotune timing");
        break;
      }
      if (ms < best) {
        best = ms;
        bestC = cs.first;
        bestS = cs.second;
      }
    }
    k.C = bestC;
    k.S = bestS;
  }
  if (status == PDG_OK) {
    build_items(c, items);
    status = upload_items(c, items);
  }
  // dense launch groups: time every schedule a group allows (levelled,
  // claimed, transfer) over whole sweeps and keep the fastest;
  // PDG_DENSE_SCHEDULE, when set, keeps the prepared choice
  if (status == PDG_OK && !std::getenv("PDG_DENSE_SCHEDULE")) {
    auto set_claim_flag = [c]() {
      c->dense_claim = false;
      for (const DenseGroup &h : c->dgroups) c->dense_claim = c->dense_claim || h.claim;
    };
    for (DenseGroup &g : c->dgroups) {
      std::vector<int> cands = {0, 1};  // levelled, claimed
      if (g.transfer_ok) cands.push_back(2);
      int best_s = g.transfer ? 2 : (g.claim ? 1 : 0);
      float best = 1e30f;
      for (int sch : cands) {
        g.claim = sch == 1;
        g.transfer = sch == 2;
        set_claim_flag();
        hipError_t e = hipSuccess;
        pdg_status ss = PDG_OK;
        for (int r = 0; r <= reps && ss == PDG_OK && e == hipSuccess; ++r) {
          if (r == 1) e = hipEventRecord(e0, st);
          if (e == hipSuccess) ss = do_sweep(c, f, fb, fb, 0, st, ctx_scratch(c));
        }
        if (ss != PDG_OK) {
          status = ss;
          break;
        }
        if (e == hipSuccess) e = hipEventRecord(e1, st);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
        if (e != hipSuccess) {
          status = from_hip_at(e, "autotune timing (dense schedules)");
          break;
        }
        if (dense_failed(c)) {  // a claimed wait gave up: the timing is invalid
          status = PDG_EDEVICE;
          break;
        }
        if (ms < best) {
          best = ms;
          best_s = sch;
        }
      }
      g.claim = best_s == 1;
      g.transfer = best_s == 2;
      set_claim_flag();
      if (status != PDG_OK) break;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->stats_valid = false;
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);  // the step graph holds the old schedules
  c->gexec = nullptr;
  c->g_f = nullptr;
  c->g_fb = nullptr;
  return status;
}

pdg_status pdg_get_tiles(const pdg_ctx *c, int32_t *n_classes, int32_t *tiles) {
  if (!c || !n_classes) return PDG_EINVAL;
  if (!c->prepared) return PDG_ESTATE;
  if (tiles) {
    for (size_t k = 0; k < c->classes.size() && (int32_t)k < *n_classes; ++k) {
      tiles[4 * k + 0] = c->classes[k].np;
      tiles[4 * k + 1] = c->classes[k].x_kind;
      tiles[4 * k + 2] = c->classes[k].C;
      tiles[4 * k + 3] = c->classes[k].S;
    }
  }
  *n_classes = (int32_t)c->classes.size();
  return PDG_OK;
}

static pdg_status set_tiles_impl(pdg_ctx *c, int32_t n_classes, const int32_t *tiles) {
  if (!c || (n_classes > 0 && !tiles) || n_classes < 0) return PDG_EINVAL;
  if (!c->prepared) return PDG_ESTATE;
  for (int32_t i = 0; i < n_classes; ++i) {
    bool found = false;
    for (const LaunchClass &k : c->classes)
      if (k.np == tiles[4 * i] && k.x_kind == tiles[4 * i + 1]) {
        found = true;
        if (!tile_valid(k, tiles[4 * i + 2], tiles[4 * i + 3])) return PDG_EINVAL;
      }
    if (!found) return PDG_EINVAL;
  }
  for (int32_t i = 0; i < n_classes; ++i)
    for (LaunchClass &k : c->classes)
      if (k.np == tiles[4 * i] && k.x_kind == tiles[4 * i + 1]) {
        k.C = tiles[4 * i + 2];
        k.S = tiles[4 * i + 3];
      }
  std::vector<SweepItem> items;
  build_items(c, items);
  return upload_items(c, items);
}

static pdg_status last_refine_correction_impl(const pdg_ctx *c, double *max_rel_correction) {
  if (!c || !max_rel_correction) return PDG_EINVAL;
  if (!c->prepared || !c->stats_valid) return PDG_ESTATE;
  hipError_t e = hipStreamSynchronize(c->last_stream);
  if (e != hipSuccess) return from_hip(e);
  const size_t n = c->last_stats == c->stats.p ? c->stats.n : 2 * (c->sitems.n + c->smixed.n);
  std::vector<double> h(n);
  e = hipMemcpy(h.data(), c->last_stats, h.size() * sizeof(double), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return from_hip(e);
  double cm = 0.0, ym = 0.0;
  for (size_t i = 0; i + 1 < h.size(); i += 2) {
    cm = std::max(cm, h[i]);
    ym = std::max(ym, h[i + 1]);
  }
  *max_rel_correction = ym > 0 ? cm / ym : 0.0;
  return PDG_OK;
}

pdg_status pdg_sync_status(pdg_ctx *c) {
  if (!c) return PDG_EINVAL;
  if (!c->prepared) return PDG_ESTATE;
  HIP_TRY(hipStreamSynchronize(c->last_stream));
  HIP_TRY(hipGetLastError());
  int32_t err = 0;
  HIP_TRY(hipMemcpy(&err, c->derr.p, sizeof(err), hipMemcpyDeviceToHost));
  if (c->herr) *c->herr = 0;
  if (err) {
    const int32_t zero = 0;
    HIP_TRY(hipMemcpy(c->derr.p, &zero, sizeof(zero), hipMemcpyHostToDevice));
    std::snprintf(g_detail, sizeof(g_detail), "%s",
                  (err & 2) ? "dense sweep: tile-claim counter overrun"
                            : "dense sweep: a wait for an upwind trace timed out");
    return PDG_EDEVICE;
  }
  return PDG_OK;
}

// Host allocation failures (std::bad_alloc) are reported as PDG_ENOMEM; no
// exception crosses the C ABI.
pdg_status pdg_topo_levels(int32_t n_nodes, int64_t n_edges, const int32_t *src, const int32_t *dst,
                           int32_t *level) {
  try {
    return topo_levels_impl(n_nodes, n_edges, src, dst, level);
  } catch (const std::bad_alloc &) {
    return PDG_ENOMEM;
  }
}

pdg_status pdg_setup_mesh(const pdg_instance_desc *descs, int32_t n_inst, pdg_ctx **out) {
  try {
    return setup_mesh_impl(descs, n_inst, out);
  } catch (const std::bad_alloc &) {
    return PDG_ENOMEM;
  }
}

pdg_status pdg_node_coords(const pdg_ctx *c, int32_t inst, double *vol_xyz, double *inflow_xyz) {
  try {
    return node_coords_impl(c, inst, vol_xyz, inflow_xyz);
  } catch (const std::bad_alloc &) {
    return PDG_ENOMEM;
  }
}

pdg_status pdg_levels(const pdg_ctx *c, int32_t inst, int32_t vel, int32_t *level) {
  try {
    return levels_impl(c, inst, vel, level);
  } catch (const std::bad_alloc &) {
    return PDG_ENOMEM;
  }
}

pdg_status pdg_prepare(pdg_ctx *c, double dt, double theta, double omega, pdg_scheme scheme, pdg_precision prec,
                       void *stream) {
  try {
    return prepare_impl(c, dt, theta, omega, scheme, prec, stream);
  } catch (const std::bad_alloc &) { if (c) c->release_device();
    return PDG_ENOMEM;
  }
}

pdg_status pdg_step(pdg_ctx *c, void *f, const double *fb, int32_t n_steps, void *stream) {
  try {
    return step_impl(c, f, fb, n_steps, stream);
  } catch (const std::bad_alloc &) {
    return PDG_ENOMEM;
  }
}

pdg_status pdg_autotune(pdg_ctx *c, void *f, const double *fb, int32_t reps, void *stream) {
  try {
    return autotune_impl(c, f, fb, reps, stream);
  } catch (const std::bad_alloc &) {
    return PDG_ENOMEM;
  }
}

pdg_status pdg_set_tiles(pdg_ctx *c, int32_t n_classes, const int32_t *tiles) {
  try {
    return set_tiles_impl(c, n_classes, tiles);
  } catch (const std::bad_alloc &) {
    return PDG_ENOMEM;
  }
}

pdg_status pdg_last_refine_correction(const pdg_ctx *c, double *max_rel_correction) {
  try {
    return last_refine_correction_impl(c, max_rel_correction);
  } catch (const std::bad_alloc &) {
    return PDG_ENOMEM;
  }
}

void pdg_destroy(pdg_ctx *c) {
  if (!c) return;
  c->release_device();
  delete c;
}

}  // extern "C"
