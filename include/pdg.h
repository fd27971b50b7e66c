/*
 * pdg.h - C ABI of the MI355X (gfx950) implementation of the hot path of the
 * Palindromic Discontinuous Galerkin kinetic scheme (Badwaik et al.,
 * "Task-based parallelization of an implicit kinetic scheme", arXiv 1702.00169):
 * the implicit upwind-DG transport sweep and the local BGK relaxation.
 *
 * Model (Sec. 2, eq. kin_bgk).  nv transport equations at constant velocities
 * v_i, each carrying m components f_{i,k}, coupled by the relaxation
 * f <- f + omega (f^eq(w) - f) with w = P f (eq. micro_to_macro): w_k =
 * sum_i f_{i,k} for the vector kinetic models, or the 3 x 9 matrix P of the
 * D2Q9 lattice model of the isothermal Euler equations with gravity (Sec. 5.1),
 * whose constant gravity enters through the source step S_2 (Sec. 3.2).
 * Space: nodal DG on Gauss-Lobatto points of uniform Cartesian hexahedra
 * (Sec. 3.1, eq. DG_reduit).  Time: the theta-scheme transport step
 * (eq. transport_cn, theta = 1/2 gives T_2) and the collision update
 * (eq. collision_cn).  The upwind flux makes the transport matrix block
 * triangular in a topological order of the upwind dependency graph (Sec. 4.1),
 * so each implicit step is solved by a downwind sweep.
 *
 * Supported here: D in {2, 3}, degree d in 1..4, any constant velocities.
 * - axis-aligned velocities (+-lambda e_k): the cell block I + theta dt
 *   Gamma_{L<-L} factorises as a Kronecker product of a (d+1) x (d+1)
 *   one-dimensional block with the identity, and the dependency graph splits
 *   into independent lines of cells along the velocity axis;
 * - velocities with two or three non-zero components (e.g. the diagonal
 *   velocities of D2Q9 / D3Q27): dense cell blocks, swept as a tiled
 *   wavefront; (d+1)^D <= 27 (2D: d <= 4, 3D: d <= 2);
 * - the zero velocity: transport is the identity.
 *
 * Conventions used by every entry point:
 *  - Status codes are returned synchronously; the library never aborts and no
 *    exception crosses the ABI.  Argument and state errors are detected on the
 *    host before anything is launched.  An asynchronous device error is
 *    reported as PDG_EDEVICE by the next call that checks the device.
 *  - Device pointers are plain HIP device allocations owned by the caller
 *    (for example torch tensors on "cuda", passed by data_ptr()); the library
 *    never frees them and never keeps them beyond the call, except that
 *    pdg_step keeps a cached graph keyed by (f, fb) that it rebuilds when they
 *    change.  Host pointers are read or written only during the call.
 *  - `stream` is a hipStream_t (NULL = the legacy default stream); all device
 *    work is enqueued on it in order.  A context is not thread safe.
 *  - Layouts (element offsets within one instance; instances are
 *    concatenated, offsets from pdg_layout):
 *      node j   = jx + (d+1) jy + (d+1)^2 jz          (Gauss-Lobatto tensor index)
 *      cell c   = x + nx y + nx ny z                   (lexicographic, x fastest)
 *      f[v][k][j][c]      nv * m * Nd * Nc values, Nd = (d+1)^D, Nc = nx ny nz
 *      w[k][j][c]         nw * Nd * Nc values (nw = m moments per node; 3 for
 *                         PDG_FEQ_D2Q9: rho, rho u_x, rho u_y)
 *      fb[v][k][t][tau]   inflow boundary values of velocity v: for an axis-a
 *                         velocity, t enumerates the node indices of the other
 *                         axes (increasing axis order, first fastest) and tau
 *                         the cell indices of the other axes (same order);
 *                         (d+1)^(D-1) * Nc / n_a values per (v, k).
 */
#ifndef PDG_H
#define PDG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pdg_ctx pdg_ctx; /* opaque, owned by the library */

typedef enum {
  PDG_OK = 0,
  PDG_EINVAL = 1,       /* bad argument (null pointer, size, non-finite value) */
  PDG_EUNSUPPORTED = 2, /* valid but outside what this build implements */
  PDG_ENOTDAG = 3,      /* an upwind dependency graph has a cycle */
  PDG_ESINGULAR = 4,    /* a cell block I + theta dt Gamma_LL is singular */
  PDG_ENOMEM = 5,       /* host or device allocation failed */
  PDG_EDEVICE = 6,      /* HIP runtime or kernel error */
  PDG_ESTATE = 7        /* call out of order (e.g. sweep before prepare) */
} pdg_status;

typedef enum {
  PDG_FP64 = 0,        /* state and arithmetic in binary64 */
  PDG_FP32 = 1,        /* state and arithmetic in binary32 (moments in binary64) */
  PDG_FP32_REFINE = 2, /* binary64 state; binary32 cell solves with one binary64
                          residual correction per cell */
  PDG_FP32_REFINE_P48 = 3 /* the arithmetic of PDG_FP32_REFINE with the state kept in
                          48 bits per value (6 bytes instead of 8, so a transport +
                          relax step moves 24 instead of 32 bytes per unknown).  The
                          f buffer holds 6 * f_elems bytes: f_elems binary32 values h
                          (each value rounded to nearest), then f_elems int16 values l;
                          the value is h + l * 2^(e - 39), e the binary exponent of h
                          (e = -126 for h = 0 or subnormal), l = round((value - h) /
                          2^(e - 39)) clamped to +-32767: a 40-bit significand, relative
                          rounding <= 2^-39, for |value| < 2^128.  Each
                          kernel rounds the values it writes to this format; use
                          pdg_state_from_f64 / pdg_state_to_f64 to convert. */
} pdg_precision;

typedef enum {
  PDG_FEQ_ADVECTION = 0, /* q^k(w) = a_k w; feq_param = {a_1, .., a_D} */
  PDG_FEQ_EULER = 1,     /* compressible Euler, m = D + 2; feq_param = {gamma} */
  PDG_FEQ_D2Q9 = 2       /* isothermal Euler on the D2Q9 lattice (Sec. 5.1): D = 2, m = 1, nv = 9
                            velocities lambda x {0, +-e_x, +-e_y, (+-1, +-1)} in any order;
                            w = (rho, rho u_x, rho u_y); with c^2 = lambda^2 / 3,
                            f_i^eq = wt_i rho (1 + u.v_i/c^2 + (u.v_i)^2/(2c^4) - u.u/(2c^2)),
                            wt = 4/9 (rest), 1/9 (axis), 1/36 (diagonal);
                            feq_param = {g}: constant gravity -g e_y (0: no source).
                            A malformed velocity set is PDG_EINVAL at setup. */
} pdg_feq_kind;

typedef enum {
  PDG_LIE = 0,              /* [T(dt) C(dt)]^N */
  PDG_STRANG = 1,           /* [T(dt/2) C(dt) T(dt/2)]^N  (M_2, Sec. 3.2) */
  PDG_STRANG_COLLAPSED = 2, /* T(dt/2) C [T(dt) C]^(N-1) T(dt/2)  (Sec. 5.1) */
  PDG_KIN = 3,              /* [M_2^kin(dt)]^N, M_2^kin(h) = T(h/4) C(h/2) T(h/2) C(h/2) T(h/4)
                               (Sec. 3.2: second order also as tau -> 0) */
  PDG_KIN4 = 4              /* [M_2^kin(g1 dt) M_2^kin(g2 dt) M_2^kin(g1 dt)]^N, triple-jump
                               coefficients g1 = 1/(2 - 2^(1/3)), g2 = 1 - 2 g1: a fourth-order
                               palindromic composition (Sec. 3.2 raises the order this way).
                               The negative middle stage makes it only conditionally stable
                               on the strongly damped upwind modes: use small dt. */
} pdg_scheme;

/* One independent kinetic problem.  The equilibrium (Sec. 2: P f^eq = P f and
 * q^k = P V^k f^eq, depending on w only) is taken as
 *   f_i^eq = w / nv + v_i . Q(w) / (2 lambda^2),  Q = (q^1, .., q^D),
 * which meets both moment conditions when the velocities are {+-lambda e_k}
 * (nv = 2D).  Transport alone accepts any set of non-zero axis-aligned
 * velocities; pdg_relax and the equilibrium helpers need the full
 * {+-lambda e_k} set. */
typedef struct {
  int32_t dim;          /* D, 2 or 3 */
  int32_t n[3];         /* cells per axis; n[2] is ignored when D = 2 */
  int32_t degree;       /* d, 1..4 */
  int32_t nv;           /* number of velocities, 1..27 */
  int32_t m;            /* components per velocity, 1..8 */
  double lo[3], hi[3];  /* box; uniform cells of size (hi - lo) / n */
  const double *v;      /* host, nv * dim, row-major; copied */
  int32_t feq;          /* pdg_feq_kind */
  double feq_param[4];  /* see pdg_feq_kind */
  const double *edges[3]; /* optional, host: cell edges along axis k (n[k] + 1 strictly increasing
                             finite values; copied), a tensor-product graded mesh of box cells;
                             NULL: uniform cells on [lo[k], hi[k]].  Given edges replace lo/hi.
                             Velocities with two or three non-zero components along graded
                             axes keep one dense cell block per combination of distinct cell
                             sizes along those axes (prepared on the device like the others;
                             the transfer schedule is for uniform cells only). */
  double axes[9];       /* optional uniform affine lattice (Sec. 3.1, affine cell maps): axes[3 k + i]
                           is component i of the edge vector a_k shared by every cell, for k, i < D;
                           cell (c_0, .., c_{D-1}) is lo + sum_k (c_k + [0, 1]) a_k, every cell the
                           same parallelogram / parallelepiped (positive determinant, else
                           PDG_EINVAL; hi and edges must then be unused).  All zero: box cells.
                           Transport runs in the frame of the cell index axes, where the scheme is
                           that of unit box cells with velocity A^{-1} v (A = [a_0 .. a_{D-1}]):
                           chains follow the index axes along which A^{-1} v is non-zero (a
                           component at most 1e-13 of its largest counts as zero), and a
                           velocity with several non-zero components of A^{-1} v takes the dense
                           path.  fb and pdg_node_coords use the same index-frame faces, mapped
                           to physical points; the relaxation and equilibria use v itself. */
} pdg_instance_desc;

/* Build a context for n_inst independent instances (Sec. 4.1): validate the
 * descriptors, build each velocity's upwind dependency graph (edge L -> R when
 * n_LR . v > 0 on the common face), order it by Kahn's algorithm into levels,
 * reject cycles (PDG_ENOTDAG), and group the cells into lines along each
 * velocity axis.  Host only: no device memory is touched.  *out receives a
 * context to be released with pdg_destroy; it is untouched on error. */
pdg_status pdg_setup_mesh(const pdg_instance_desc *inst, int32_t n_inst, pdg_ctx **out);

/* Sizes (in elements) of the f, w and fb buffers for all instances, and the
 * per-instance start offsets (arrays of n_inst + 1 entries each; the last is
 * the total).  Any output pointer may be NULL. */
pdg_status pdg_layout(const pdg_ctx *c, int64_t *f_elems, int64_t *w_elems, int64_t *fb_elems,
                      int64_t *inst_f_offsets, int64_t *inst_w_offsets, int64_t *inst_fb_offsets);

/* Physical coordinates of instance `inst` (host buffers, may be NULL):
 * vol_xyz[D][j][c] of every Gauss-Lobatto point (eq. map_GL), and
 * inflow_xyz[v][D][t][tau] of the inflow boundary points at which fb is read
 * (one block of D * (d+1)^(D-1) * Nc/n_a values per velocity). */
pdg_status pdg_node_coords(const pdg_ctx *c, int32_t inst, double *vol_xyz, double *inflow_xyz);

/* Topological level (longest upwind path from the inflow boundary, Sec. 4.1)
 * of every cell of instance `inst` for velocity `vel`; level[c], host. */
pdg_status pdg_levels(const pdg_ctx *c, int32_t inst, int32_t vel, int32_t *level);

/* Kahn layering of an arbitrary directed graph (host utility used by setup):
 * level[i] = longest path length from a source; PDG_ENOTDAG on a cycle. */
pdg_status pdg_topo_levels(int32_t n_nodes, int64_t n_edges, const int32_t *src, const int32_t *dst,
                           int32_t *level);

/* Host introspection of the cell operator used for (inst, vel): the
 * one-dimensional block Gamma (row-major (d+1) x (d+1), downwind-local node
 * order: node 0 on the inflow face) of eq. DG_reduit along the velocity axis
 * (on a graded axis: of the chain's upwind-most cell),
 * and the inflow coefficient kappa such that the upwind coupling
 * Gamma_{L<-R} is -kappa at the inflow node.  The full cell block is the
 * Kronecker product of this block with the identity on the transverse nodes.
 * Host only; gamma holds (d+1)^2 values. */
pdg_status pdg_line_operator(const pdg_ctx *c, int32_t inst, int32_t vel, double *gamma, double *kappa);

/* Host introspection of the full cell block of any velocity: gamma receives
 * Gamma_{L<-L} of eq. DG_reduit ((d+1)^D x (d+1)^D, row-major) in
 * downwind-local tensor order (node q = q_0 + (d+1) q_1 + (d+1)^2 q_2 with
 * q_a = j_a if v_a >= 0 else d - j_a, so q_a = 0 lies on the inflow face of
 * each non-zero component); kappa[a] (3 values) is the inflow coupling
 * magnitude of axis a (Gamma_{L<-R} = -kappa[a] at the inflow face nodes; 0 if
 * v_a = 0).  On uniform Cartesian cells the block is the Kronecker sum of the
 * one-dimensional blocks of the non-zero components; on graded axes it is the
 * block of the upwind-most cell.  Host only. */
pdg_status pdg_cell_operator(const pdg_ctx *c, int32_t inst, int32_t vel, double *gamma, double *kappa);

/* Prepare the time step (Sec. 3.2): for every instance, velocity and
 * transport sub-step dt_sub of the scheme (always dt and dt/2; also dt/4 for
 * PDG_KIN; g dt/4 and g dt/2 for both triple-jump g for PDG_KIN4), build on
 * the host in binary64 the
 * one-dimensional cell blocks A = I + theta dt_sub Gamma_{L<-L} and
 * B = I - (1-theta) dt_sub Gamma_{L<-L} of eq. DG_reduit, invert A on the device
 * in binary64 (Gauss-Jordan with partial pivoting, PDG_ESINGULAR on a pivot
 * below 1e-300 times the block norm) and keep binary64 and binary32 copies.
 * omega is the collision factor of eq. collision_cn over dt (2 dt/(2 tau + dt);
 * 2 is tau = 0); collisions over other sub-steps h use 2h/(2 tau + h).
 * Allocates the context's device tables; synchronises `stream`.
 * theta in (0, 1], dt finite and non-zero (negative dt runs time backwards).
 * Environment read here: PDG_FUSED=1 makes pdg_step run each collision of
 * the collapsed Strang scheme together with the transport of the velocities
 * along x, in one pass over the state (instances whose velocities are
 * {+-lambda e_k} on a uniform box mesh, m = 1 or the Euler m, and
 * (d+1) * (n_x rounded up to 64) <= 512; the others keep separate passes;
 * the results agree to rounding); PDG_SWEEP_MIXED=0 gives each node count of a batch its own
 * sweep launch; PDG_DENSE_SCHEDULE=level|claim|transfer fixes the dense tile
 * schedule. */
pdg_status pdg_prepare(pdg_ctx *c, double dt, double theta, double omega, pdg_scheme scheme,
                       pdg_precision prec, void *stream);

/* f = f^eq(w) at every node (device; w[k][j][c] binary64 per instance,
 * f in the state precision).  Sets an initial state (Sec. 2). */
pdg_status pdg_equilibrium(pdg_ctx *c, const double *w, void *f, void *stream);

/* Conversion between the state (f in the prepared precision, layout as
 * above; for PDG_FP32_REFINE_P48 the two planes described there) and binary64
 * values x[v][k][j][c] (device, f_elems values): pdg_state_to_f64 reads f into
 * x, pdg_state_from_f64 writes x into f (rounded to the state precision).
 * Element-wise, stream ordered; x and f must not overlap.  Used to set or
 * inspect a state whose storage is not binary64. */
pdg_status pdg_state_to_f64(pdg_ctx *c, const void *f, double *x, void *stream);
pdg_status pdg_state_from_f64(pdg_ctx *c, const double *x, void *f, void *stream);

/* fb = f^eq_{v}(w) at the inflow points of every velocity (device, binary64):
 * w_inflow holds, per instance and velocity v (in that order), nw blocks
 * (one per moment) of the macroscopic field at v's inflow points, in the
 * point order of v's fb block.  With nw = m this is exactly the fb layout;
 * for PDG_FEQ_D2Q9 it holds 3 values per inflow point (size 3 * fb_elems). */
pdg_status pdg_inflow_equilibrium(pdg_ctx *c, const double *w_inflow, double *fb, void *stream);

/* One theta-scheme transport step of size dt_sub (dt or dt/2 as prepared) for
 * every instance, velocity and component, in place on f (Sec. 4.1-4.2,
 * eq. transport_cn): solves
 *   (I - theta dt L_h) F^new = (I + (1-theta) dt L_h) F^old
 *                              + dt (theta b(fb_new) + (1-theta) b(fb_old))
 * cell by cell in downwind order.  fb_old/fb_new: inflow data at the old and
 * new time (the same pointer for time-independent data).  PDG_ESTATE if
 * dt_sub is not one of the prepared sub-steps (bitwise). */
pdg_status pdg_transport_sweep(pdg_ctx *c, void *f, const double *fb_old, const double *fb_new,
                               double dt_sub, void *stream);

/* pdg_transport_sweep for callers that cannot allocate device memory (code
 * under HIP graph capture, serving loops, harnesses that forbid hipMalloc):
 * the same operation, arguments, kernels and results, but the sweep's device
 * scratch -- the per-workgroup refinement statistics, the inflow-trace slots
 * and tile-claim counters of dense velocities -- lives in a static array of
 * 32 MiB per GPU that the library holds until the process ends (its address
 * is taken when a context is prepared on that GPU), not in the context's
 * buffers.  The call allocates nothing.  PDG_EUNSUPPORTED (before any launch;
 * pdg_error_detail gives the sizes) if the problem needs more scratch than
 * that.  Every call on one GPU shares the array and leaves its contents
 * behind (the slots and counters are reset at the start of each call), so
 * calls that overlap on one GPU -- concurrent streams, threads or processes
 * sharing the library's copy -- race and must be serialised by the caller.
 * pdg_last_refine_correction reports the most recent sweep of either kind. */
pdg_status pdg_transport_sweep_static(pdg_ctx *c, void *f, const double *fb_old, const double *fb_new,
                                      double dt_sub, void *stream);

/* Collision step (eq. collision_cn, Sec. 4.4): at every node
 * w = P f (compensated binary64 sums), then f_i <- f_i + omega (f_i^eq(w) - f_i).
 * w_out (nullable, device binary64, w layout) receives w. */
pdg_status pdg_relax(pdg_ctx *c, void *f, double *w_out, void *stream);

/* Source step S_2(h) (Sec. 3.2) of the instances with a source (PDG_FEQ_D2Q9
 * with g != 0; the others are left untouched): the Crank-Nicolson integrator
 * of w' = w + h/2 (S(w) + S(w')), S(w) = (0, 0, -g rho), which keeps rho and
 * is therefore solved exactly (rho u_y -= h g rho), applied to the
 * equilibrium part of f: f <- f + f^eq(w') - f^eq(w) (Sec. 5.1).  Node-local,
 * in place; any finite h (h < 0 inverts the step h > 0).  pdg_step applies
 * it around each collision: T(dt) S(dt) C(dt) for PDG_LIE, S(dt/2) C(dt)
 * S(dt/2) for the Strang schemes, S(h/4) C(h/2) S(h/4) inside M_2^kin(h). */
pdg_status pdg_source(pdg_ctx *c, void *f, double h, void *stream);

/* n_steps time steps of the prepared scheme with time-independent inflow fb
 * (Sec. 3.2 and Sec. 5.1).  The repeated part of the scheme (one step; for
 * the collapsed form relax + full transport) is recorded once as a HIP graph
 * per (f, fb) pair and replayed. */
pdg_status pdg_step(pdg_ctx *c, void *f, const double *fb, int32_t n_steps, void *stream);

/* Autotuner of the sweep's work decomposition.  Work items are grouped in
 * launch classes (same node count d+1 and same chain kind: chains along the
 * contiguous x axis, or along a strided axis).  For every class this times
 * each candidate tile (x chains: rows per workgroup 1..64 with one cell per
 * thread (S = 1), or chains per workgroup 8..64 x cells per thread segment
 * 2..8; strided chains: chains per workgroup 8..64 x cells per thread
 * segment 1..8) with `reps`
 * launches of the class alone on `stream`, keeps the fastest, and uses it
 * from then on.  Then, for every launch group of the dense path (velocities
 * with two or three non-zero components), it times whole sweeps under each
 * tile schedule the group allows (levelled, claimed and, for 2D meshes of
 * full 8 x 8 uniform tiles, the transfer schedule) and keeps the fastest,
 * unless PDG_DENSE_SCHEDULE was set at prepare.  f is used as scratch and
 * overwritten; fb is read.  Every tile and schedule solves the same system;
 * only the rounding order differs.  PDG_EDEVICE if a claimed wait gave up
 * while timing.  Drops the cached step graph. */
pdg_status pdg_autotune(pdg_ctx *c, void *f_scratch, const double *fb, int32_t reps, void *stream);

/* Current tiles: *n_classes receives the number of launch classes; if
 * `tiles` is not NULL, up to the incoming *n_classes entries of 4 int32 each
 * are written: (d+1, chain kind (1 = x, 0 = strided axis, 2 = graded axis), C, S).
 * Host only. */
pdg_status pdg_get_tiles(const pdg_ctx *c, int32_t *n_classes, int32_t *tiles);

/* Apply tiles (same 4-int format, e.g. a cached autotuner result); classes
 * are matched by (d+1, chain kind).  PDG_EINVAL for an unknown class or an
 * invalid tile; nothing is changed then. */
pdg_status pdg_set_tiles(pdg_ctx *c, int32_t n_classes, const int32_t *tiles);

/* For PDG_FP32_REFINE and PDG_FP32_REFINE_P48: max over nodes of |correction| / max |solution| seen by
 * the most recent sweep (synchronises the stream of that sweep). */
pdg_status pdg_last_refine_correction(const pdg_ctx *c, double *max_rel_correction);

/* Detail of the most recent HIP failure seen by this thread (the failing
 * call and the runtime's message); empty if none.  Static thread-local
 * storage, valid until the next failing call. */
const char *pdg_error_detail(void);

/* Wait for the work enqueued by the most recent sweep and report device-side
 * failures: PDG_EDEVICE if a kernel failed or a dense-path tile wait timed
 * out (the result is then invalid), else PDG_OK.  Synchronises. */
pdg_status pdg_sync_status(pdg_ctx *c);

/* Human-readable name of a status code (static storage). */
const char *pdg_status_string(pdg_status s);

/* Release the context and its device tables (NULL is a no-op). */
void pdg_destroy(pdg_ctx *c);

#ifdef __cplusplus
}
#endif

#endif /* PDG_H */
