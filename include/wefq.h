/*
 * wefq: Wigner-Eckart factorized spectral Boltzmann collision operator
 * on AMD Instinct MI355X (gfx950).  C ABI.
 *
 * The operator (Sections 2.1-2.3 of the paper): for a distribution
 * f = M~ sum_alpha c_alpha phi_alpha in the Laguerre x real-spherical-harmonic
 * basis alpha = (k, l, m), the Galerkin collision term is
 *     Q_alpha1(c) = sum_{alpha2, alpha3} C_{alpha1 alpha2 alpha3} c_alpha2 c_alpha3,
 * with C the 8-D weak form of Q(f, f) for the kernel B = b0 u^gamma.  Via the
 * Wigner-Eckart factorization (eq. wigner-eckart-factorization, Section 4.1)
 * C = R^{(l1 l2 l3)}_{k1 k2 k3} g(q1, q2, q3), where g is the real Gaunt
 * weight and R the dense radial kinematic core.
 *
 * Conventions shared by every entry point:
 *   q = l*l + l + m (0-based), flat mode index n = q * (Kmax+1) + k,
 *   N = (Kmax+1)(Lmax+1)^2 modes per cell (box truncation, Section 4.6).
 *   Coefficient batches are row-major [B][ld] with the N modes of one cell
 *   contiguous.  phi_000 = 1, so the unit Maxwellian is c = e_0.
 *
 * Error behaviour: every call returns a wefq_status and never aborts; no C++
 * exception crosses the ABI.  wefq_last_error() returns a thread-local message
 * describing the last non-OK status of the calling thread.  Device faults of
 * asynchronous launches surface at the caller's next synchronization.
 */
#ifndef WEFQ_H
#define WEFQ_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct wefq_core* wefq_handle;
typedef struct wefq_plan_s* wefq_plan;

typedef enum {
  WEFQ_OK = 0,
  WEFQ_EINVAL = 1,        /* bad argument (null pointer, size, layout, precision) */
  WEFQ_ENOMEM = 2,        /* device or host allocation failed */
  WEFQ_EHIP = 3,          /* HIP runtime error */
  WEFQ_EUNSUPPORTED = 4,  /* truncation or precision not supported by this build */
  WEFQ_EBUDGET = 5        /* request does not fit the given memory budget */
} wefq_status;

typedef enum {
  WEFQ_MAXWELL = 0,       /* gamma = 0  (Maxwell molecules) */
  WEFQ_HARD_SPHERE = 1,   /* gamma = 1 */
  WEFQ_VHS = 2            /* variable hard sphere, gamma from the descriptor */
} wefq_model;

typedef enum {
  WEFQ_FP64 = 1,          /* FP64 angular coupling + FP64 MFMA radial contraction; double */
  WEFQ_FP32 = 2,          /* FP32 angular coupling + FP32 MFMA radial contraction; float */
  WEFQ_BF16X3 = 4,        /* FP32 angular coupling + split hi/lo BF16 MFMA (3 products,
                             FP32 accumulation); f and Q are float */
  WEFQ_FP64_NAIVE = 8,    /* the paper's naive ordering of the factorized sum (Section 4.5.2):
                             every COO row contracts its full K^3 block, FP64, one thread per
                             output; a reference ordering, memory-bound on R; double */
  WEFQ_PREP_BILINEAR = 16,/* not a precision: in wefq_core_desc.precisions, also prepare the
                             tables of the non-symmetric bilinear form (wefq_apply_Qfg) for the
                             FP64 / FP32 precisions requested */
  WEFQ_PREP_RADIAL = 32   /* not a precision: also prepare the tables of the radial-first
                             ordering (wefq_apply_Q_radial); implies WEFQ_FP64 */
} wefq_precision;

/* Most Legendre coefficients of an angular factor (degree <= 32). */
#define WEFQ_MAX_BETA 33

/* Descriptor of a radial core.  The collision kernel (Section 2.1, Grad cut-off) is
 *   B(u, cos chi) = b0 u^gamma beta(cos chi),  beta(t) = sum_{j < n_beta} beta[j] P_j(t),
 * with chi the deflection angle between the pre- and post-collision relative velocities
 * and P_j the Legendre polynomials.  n_beta = 0 (beta may then be NULL) is the isotropic
 * kernel beta = 1; a zero-initialized descriptor tail selects it.  b0 <= 0 selects
 * b0 = 1/(4 pi), for which int B du' = 4 pi b0 beta[0] u^gamma = beta[0] u^gamma.  beta is
 * read during the call and not kept; physical kernels have beta >= 0 on [-1, 1], which is
 * not checked.  With n_beta >= 1 the gain sphere average is integrated by a direct
 * beta-weighted rule at every node (exact for a polynomial beta), which costs more build
 * time than the isotropic closed form.  Only the even part of beta enters Q(f, f); the
 * whole of it enters the bilinear form Q(f, g).  precisions is a bitmask of
 * wefq_precision values to prepare. */
typedef struct {
  int32_t model;
  double gamma;           /* used when model == WEFQ_VHS; must be in [0, 2] */
  double b0;
  int32_t Kmax;           /* 0 <= Kmax <= 16 */
  int32_t Lmax;           /* 0 <= Lmax <= 16 */
  uint32_t precisions;
  int32_t device;         /* HIP device ordinal */
  int32_t n_beta;         /* 0 <= n_beta <= WEFQ_MAX_BETA; finite coefficients */
  const double* beta;     /* host pointer, n_beta doubles (Legendre coefficients) */
  int32_t rad_pad;        /* 0 <= pad <= 64 extra points in each radial Gauss rule, and */
  int32_t ang_pad;        /* in each angular one, beyond the counts that are exact for the
                             polynomial degree of the integrand (Sections 3.3 and 5.1: padding
                             for the self-convergence study); 0 is the exact rule */
} wefq_core_desc;

typedef struct {
  int64_t N, NK, NQ;      /* modes, radial and angular sizes */
  int64_t N_T, N_G, N_S;  /* channels, COO rows, (channel, q1) slices (Section 4.7) */
  int64_t N_T_merged, N_G_merged, N_S_merged; /* after pairing (q1,q2,q3) with (q1,q3,q2) */
  int64_t quad_nodes;     /* quadrature nodes used to integrate the core */
  int64_t device_bytes;   /* device memory held by the handle */
  double flop_alg_per_cell; /* 2 NK^2 N_G + 2 NK^3 N_S (Section 4.7, angular-first count) */
  double gamma, b0;
  int64_t model;          /* wefq_model of the core */
  int64_t n_beta;         /* angular factor: Legendre coefficients beta[0 .. n_beta) */
  double beta[WEFQ_MAX_BETA];
  int64_t radial_groups;  /* distinct (channel, q2, q3) triples of the table when the
                             radial-first tables are prepared, else 0 */
  int64_t rad_pad, ang_pad; /* quadrature padding of the build (0 for a core loaded from file) */
} wefq_core_info;

/* Build the radial core R (Sections 3.2-3.3, 4.3-4.4) on the GPU in FP64 and the
 * routing tables (Sections 4.1-4.2).  R is integrated by an exact Gauss rule in
 * centre-of-mass / relative-velocity variables, then its collision-invariant rows
 * (mass, momentum, energy) and the detailed-balance vector are set to exactly 0
 * (Section 4.4).  Synchronous: returns when the handle is ready.  stream may be
 * NULL (the default stream).  On success *out owns all device memory of the core;
 * release it with wefq_destroy.  The handle is read-only afterwards and may be
 * used concurrently from several streams.  EINVAL for n_beta outside
 * [0, WEFQ_MAX_BETA], a NULL beta with n_beta > 0 or a non-finite coefficient. */
wefq_status wefq_build_core(const wefq_core_desc* desc, void* stream, wefq_handle* out);

/* Sizes and parameters of a built core (the counts of Sections 4.6-4.7 and Table 6, the
 * merged counts of this implementation, device memory held, the angular factor).  Host
 * only; info is caller-owned.  EINVAL for a null argument. */
wefq_status wefq_core_info_get(wefq_handle h, wefq_core_info* info);

/* Flat index of the basis function phi_klm (Section 2.2) in a core's coefficient vectors:
 * *n = (l*l + l + m) * NK + k.  EINVAL unless 0 <= k <= Kmax, 0 <= l <= Lmax, |m| <= l.
 * Host only. */
wefq_status wefq_mode_index(wefq_handle h, int32_t k, int32_t l, int32_t m, int64_t* n);

/* Copy the zeroed FP64 core to host memory: R[c][k1][k2][k3], c in the paper's
 * channel order (l1 outer, l2, l3 inner), count = N_T * NK^3 doubles. */
wefq_status wefq_core_download_R(wefq_handle h, double* host_R, int64_t count);

/* Write the core to a file: its parameters and the radial tensor before the invariant-row
 * zeroing (N_T * NK^3 doubles, paper channel order), with a checksum, so that
 * wefq_core_load can rebuild the handle without the quadrature.  Host only. */
wefq_status wefq_core_save(wefq_handle h, const char* path);

/* Build a core from a file written by wefq_core_save: model, gamma, b0, the angular
 * factor, Kmax and Lmax come from the file; precisions (as in wefq_core_desc) and device are chosen here.  The
 * tables and results are bitwise those of the saved core.  EINVAL for a missing,
 * truncated or corrupted file (header, size and checksum are checked before any device
 * work). */
wefq_status wefq_core_load(const char* path, uint32_t precisions, int32_t device, void* stream, wefq_handle* out);

/* Q = Q(f, f) for B independent cells (eq. full_discrete_sum, Section 4.5).
 * f and Q are device pointers, row-major [B][ld_f] / [B][ld_q], ld >= N,
 * double for WEFQ_FP64 / WEFQ_FP64_NAIVE and float otherwise, aligned to the
 * element size, not aliasing.  Requesting WEFQ_FP64_NAIVE needs the WEFQ_FP64 tables.
 * Q is overwritten (not accumulated).  B == 0 is a no-op.  Asynchronous on
 * stream; allocates nothing.  For finite f the mass, momentum and energy rows of Q
 * are exactly 0 in every precision: those rows of the core are zero (Section 4.4), so
 * every product on them is 0 x finite; they are stored as computed, not overwritten.
 * NaN/Inf in f propagate, into those rows too. */
wefq_status wefq_apply_Q(wefq_handle h, int32_t precision, const void* f, void* Q,
                         int64_t B, int64_t ld_f, int64_t ld_q, void* stream);

/* Workspace of wefq_apply_Q_radial for chunks of `chunk` cells (rounded up to a multiple
 * of 64): chunk * (N + radial_groups * NK) * 8 bytes.  EINVAL if the core was built without
 * WEFQ_PREP_RADIAL or chunk < 1. */
wefq_status wefq_radial_workspace(wefq_handle h, int64_t chunk, int64_t* bytes);

/* Q = Q(f, f) in FP64 by the radial-first ordering of the factorized sum (Section 4.5.3): for
 * every distinct (channel c, q2, q3) of the table the dense intermediate
 *   Psi^{k1}_{q2 q3 c} = sum_{k2, k3} R^{(c)}_{k1 k2 k3} f_{k2 q2} f_{k3 q3}
 * is written to the workspace, then one pass over the table grouped by output state forms
 * Q_{k1 q1} = sum_z g_z Psi^{k1}_{q2z q3z c_z}.  A reference ordering for comparison with
 * wefq_apply_Q (the angular-first ordering); the results agree to FP64 rounding.
 * f, Q: device pointers to double, row-major [B][ld], ld >= N, not overlapping each other or
 * the workspace.  work: caller-owned device memory, 256-byte aligned, of work_bytes bytes;
 * the batch runs in chunks of the largest multiple of 64 cells whose workspace
 * (wefq_radial_workspace) fits work_bytes, at most 65,536.  Concurrent calls need separate
 * workspaces.  The invariant rows of Q are exactly 0.  Needs a core built with
 * WEFQ_PREP_RADIAL.  EINVAL for bad pointers or sizes, or a workspace smaller than one
 * 64-cell chunk.  Asynchronous on stream; allocates nothing.  B == 0 is a no-op. */
wefq_status wefq_apply_Q_radial(wefq_handle h, const double* f, double* Q, int64_t B, int64_t ld_f,
                                int64_t ld_q, void* work, int64_t work_bytes, void* stream);

/* ---- the dense Cartesian contraction (Section 4.5.1), the paper's comparison baseline ---- */

/* Bytes of the dense weak-form tensor C of a core for wefq_dense_assemble:
 * 16 ceil(N/16) * N * 4 ceil(N/4) doubles (7.6 GB at Kmax = 4, Lmax = 13).  EINVAL without the
 * WEFQ_FP64 tables; EUNSUPPORTED for N > 1280 (the contraction stages a 16-cell tile of f in LDS). */
wefq_status wefq_dense_bytes(wefq_handle h, int64_t* bytes);

/* Assemble the full tensor C_{a1 a2 a3} = g_{q1 q2 q3} R^{(c)}_{k1 k2 k3} (the factorization of
 * Section 4.1 undone; zero where no Gaunt row exists) into C, caller-owned device memory of at
 * least wefq_dense_bytes bytes, 256-byte aligned, in the layout of the contraction's matrix-core
 * operand (documented in dense.hip).  Asynchronous on stream; allocates nothing. */
wefq_status wefq_dense_assemble(wefq_handle h, void* C, int64_t C_bytes, void* stream);

/* Q = Q(f, f) by the dense Cartesian contraction Q_a1 = sum_{a2, a3} C_{a1 a2 a3} f_a2 f_a3 in
 * FP64 (Section 4.5.1): a reference ordering for comparison with wefq_apply_Q, 2 N^3 flops per
 * cell.  C as assembled by wefq_dense_assemble; f, Q as for wefq_apply_Q in FP64 (double,
 * [B][ld], ld >= N); Q must not overlap f or C.  Its invariant rows are exactly 0 for finite f
 * (those rows of C are zero).  Asynchronous on stream; allocates nothing.  B == 0 is a no-op. */
wefq_status wefq_apply_Q_dense(wefq_handle h, const void* C, int64_t C_bytes, const double* f, double* Q, int64_t B,
                               int64_t ld_f, int64_t ld_q, void* stream);

/* Jacobian-vector product out = J(c) d = Q(c, d) + Q(d, c), the derivative of Q(f, f)
 * at f = c in the direction d, where Q(f, g) = sum C_{a1 a2 a3} f_a2 g_a3 is the
 * bilinear form of Section 2.3 (so J(c) c = 2 Q(c, c) and J(e_000) is the linearized
 * operator).  c, d, out: device pointers, row-major [B][ld], ld >= N, double for
 * WEFQ_FP64 and float for WEFQ_FP32 (the two precisions offered), aligned to the
 * element size; c and d may alias each other but not out.  out is overwritten, its
 * invariant rows are exactly 0.  Asynchronous on stream; allocates nothing.  Both
 * inputs are staged in LDS, so the cell tile is at most half that of wefq_apply_Q: FP64
 * at Kmax = Lmax >= 13 runs tiles of 2 cells with 8 output states per column group, which
 * fit up to 16.  WEFQ_EUNSUPPORTED when even those do not fit LDS. */
wefq_status wefq_apply_J(wefq_handle h, int32_t precision, const void* c, const void* d, void* out, int64_t B,
                         int64_t ld_c, int64_t ld_d, int64_t ld_out, void* stream);

/* The bilinear form itself: out = Q(f, g) = sum C_{a1 a2 a3} f_a2 g_a3 (Section 2.3; f is
 * the particle whose distribution the loss term depletes, g its collision partner), so
 * Q(f, f) is wefq_apply_Q and Q(f, g) + Q(g, f) = wefq_apply_J.  Arguments as for
 * wefq_apply_J; the core must have been built with WEFQ_PREP_BILINEAR in its precisions
 * (otherwise EINVAL).  Two launches on stream: the symmetric part, then the antisymmetric
 * part added into out.  The mass row of out is exactly 0; the momentum and energy rows are
 * not zero in general (only Q(f, g) + Q(g, f) conserves them), and they come from the core
 * before the invariant-row zeroing of Section 4.4. */
wefq_status wefq_apply_Qfg(wefq_handle h, int32_t precision, const void* f, const void* g, void* out, int64_t B,
                           int64_t ld_f, int64_t ld_g, int64_t ld_out, void* stream);

/* FP64 check of the five collision-invariant rows (Section 4.4) of a computed Q:
 * *max_abs = max over cells of |Q| on those rows (exactly 0 when conservation
 * holds; NaN if any of them is NaN).  Q as for wefq_apply_Q with the same precision.
 * Synchronizes stream.  The per-block partial maxima go to a small device buffer
 * owned by the handle, so checks on one handle must not run concurrently. */
wefq_status wefq_check_conservation(wefq_handle h, int32_t precision, const void* Q,
                                    int64_t B, int64_t ld_q, double* max_abs, void* stream);

/* Release every device and host resource of a core.  The caller must have synchronized
 * the streams that used it (plans built on it must be destroyed first).  EINVAL for NULL. */
wefq_status wefq_destroy(wefq_handle h);

/* Message of the last non-OK status returned on the calling thread (thread-local; valid
 * until the thread's next failing call).  Never NULL. */
const char* wefq_last_error(void);

/* Tile shape used by wefq_apply_Q for one precision of a core: slots = output
 * states sharing the 16 MFMA columns (1, 2 or 4; the cell tile is 16/slots cells
 * and must fit in LDS), block = threads per workgroup (256, 512, 768 or 1024; 768 and 1024 run
 * kernel instances built for 12 and 16 waves, with fewer registers per lane; 1024 exists for
 * quadrants up to 5x5, H = ceil((Kmax+1)/2) <= 5).  Results are bitwise independent of the
 * shape.  The default, set by wefq_build_core, is the largest tile that fits in LDS with a
 * kernel that spills at most 128 bytes of registers per lane; 256 threads when a tile holds
 * fewer than 16 work units of up to 4 output states each, else the block among 512, 768 and
 * 1024 whose instance spills at most 64 bytes and keeps the most waves resident per compute
 * unit (the larger on a tie); the autotuner may replace it.  Each precision keeps its own
 * shape.  EINVAL for an unknown precision, slots or block, or a block with no instance for
 * the shape.
 * Setting a shape also re-derives how small batches split their tiles over workgroups
 * (a residency query of the kernel on the core's device, which the call makes current).
 * EUNSUPPORTED when the tile does not fit in LDS; EHIP when the device cannot be selected.
 * Not thread-safe with concurrent applies of the same core. */
wefq_status wefq_tune_set(wefq_handle h, int32_t precision, int32_t slots, int32_t block);
/* The shape wefq_apply_Q currently uses for a precision.  EINVAL for a null argument or a
 * precision without tiles. */
wefq_status wefq_tune_get(wefq_handle h, int32_t precision, int32_t* slots, int32_t* block);

/* ---- uneven batches in one persistent launch (captured in a HIP graph) ---- */

/* One segment of an uneven batch: B cells of core `core` with coefficients f
 * and outputs Q (device pointers, layout as for wefq_apply_Q).  slots = 0 uses
 * the core's current tile shape. */
typedef struct {
  wefq_handle core;
  int32_t precision;      /* one precision for the whole plan: FP32, BF16X3 or FP64 */
  int32_t slots;
  const void* f;
  void* Q;
  int64_t B, ld_f, ld_q;
} wefq_segment;

/* Build a plan: one work item per (segment, cell tile), or several per tile when a tile
 * costs more than a third of a workgroup's fair share of the plan (each then takes every
 * n-th work unit of the tile), largest first, served by a persistent kernel whose
 * workgroups pull items from a device counter; the counter
 * reset and the kernel are captured once in a HIP graph.  Per-cell results equal
 * those of wefq_apply_Q bitwise.  Buffers and cores must outlive the plan; the plan
 * owns a small device work list.  Synchronizes stream.  block: 256 or 512 threads (the
 * 8-wave kernel, every tile shape), or 768 (a 12-wave kernel, three waves per SIMD, for FP32
 * plans whose segments all have the shapes of one of its two builds: quadrants up to 5x5 or
 * 7x7 with one output state per MFMA column group or 9x9 with two, the default FP32 shapes of
 * K = 0..9, 12 and 16; or 6x6 with one and 7x7 or 8x8 with two, those of K = 10, 11 and
 * 13..15.  EINVAL otherwise).  BF16X3 and FP64 plans whose segments all have their precision's default tile
 * shapes run an 8-wave build of those shapes only, which spills fewer registers. */
wefq_status wefq_plan_create(int32_t nseg, const wefq_segment* segs, int32_t block, void* stream,
                             wefq_plan* out);
/* Replay the captured graph on stream (asynchronous).  Concurrent launches of one
 * plan race on its counter: serialize them on one stream. */
wefq_status wefq_plan_launch(wefq_plan p, void* stream);
/* The same two kernels launched directly, without the graph. */
wefq_status wefq_plan_launch_direct(wefq_plan p, void* stream);
/* The plan's work list length, dynamic LDS per workgroup and persistent grid size; any output
 * pointer may be NULL.  EINVAL for a null plan. */
wefq_status wefq_plan_info(wefq_plan p, int64_t* work_items, int64_t* lds_bytes, int64_t* grid);
/* Release the plan (its graph and device work list); the caller synchronizes first. */
wefq_status wefq_plan_destroy(wefq_plan p);

/* ---- runners: one persistent launch per call over any mix of segments (serving) ---- */

typedef struct wefq_runner_s* wefq_runner;

/* A runner launches the persistent kernel of wefq_plan_create once per wefq_runner_launch over
 * the segments of that call, with no graph and no allocation per call: the scheduling tick of
 * a continuous-batching server, where the set of (core, cells) changes from one launch to the
 * next (the spatial batching of Section 4.5 over requests of several truncations and models).
 * It owns a ring of 4 slots, each a device work list of max_segments descriptors and max_items
 * work items with a pinned host staging copy.  precision: FP32, BF16X3 or FP64 for every
 * segment; block: 256, 512 or 768 threads (768: FP32 only, the 12-wave kernel of
 * wefq_plan_create for launches whose segments all have its tile shapes, the 8-wave kernel of
 * 512 threads for the others).  EINVAL for bad arguments, ENOMEM when the slots cannot be
 * allocated. */
wefq_status wefq_runner_create(int32_t device, int32_t precision, int32_t max_segments, int32_t max_items,
                               int32_t block, wefq_runner* out);

/* One persistent launch over nseg segments (layout, rules and per-cell results as for
 * wefq_plan_create: bitwise those of wefq_apply_Q).  Builds the work list on the host, copies it
 * into the next ring slot and enqueues the counter reset and the kernel on stream; returns without
 * waiting, except when the slot's previous launch is still running (then it waits for that one).
 * Segment buffers must stay valid until the launch completes.  EBUDGET when the batch needs more
 * work items than max_items; nseg = 0 or a batch without cells launches nothing. */
wefq_status wefq_runner_launch(wefq_runner r, int32_t nseg, const wefq_segment* segs, void* stream);

/* Wait for the runner's launches and release it.  EINVAL for NULL. */
wefq_status wefq_runner_destroy(wefq_runner r);

/* ---- time integration: batched explicit Runge-Kutta stepping of dc/dt = Q(c) ---- */

/* With the identity mass matrix the Galerkin weak form is an ODE system per cell
 * (Section 2.3); the relaxation experiments of Section 5 integrate it with an
 * explicit Runge-Kutta scheme.  Schemes: forward Euler, Heun (2 stages), the
 * three-stage strong-stability-preserving scheme, and the classic four-stage one. */
typedef enum {
  WEFQ_RK_EULER = 1,
  WEFQ_RK_HEUN = 2,
  WEFQ_RK_SSP3 = 3,
  WEFQ_RK_CLASSIC4 = 4
} wefq_rk_scheme;

/* Device workspace (bytes) that wefq_rk_integrate needs for B cells: 256 bytes of
 * check state plus (stages + 1) compact [B][N] buffers of the precision's element. */
wefq_status wefq_rk_workspace(wefq_handle h, int32_t precision, int32_t scheme, int64_t B, int64_t* bytes);

/* Advance the device coefficients c ([B][ld], ld >= N, element as for wefq_apply_Q)
 * in place by nsteps steps of size dt of the given scheme.  Every stage evaluates Q
 * with wefq_apply_Q's kernels on the whole batch, followed by fused element-wise
 * combinations.  work is a caller-owned device buffer of at least wefq_rk_workspace
 * bytes, 256-byte aligned, not overlapping c; nothing is allocated.  When max_invariant
 * is not NULL it receives the FP64 maximum of |Q| over the five invariant rows of every
 * stage evaluation (exactly 0 when conservation holds; then the invariant coefficients
 * of c are unchanged bit for bit), and the call synchronizes stream; otherwise it is
 * asynchronous.  Per-cell results do not depend on the batch. */
wefq_status wefq_rk_integrate(wefq_handle h, int32_t precision, int32_t scheme, void* c, int64_t B, int64_t ld,
                              double dt, int32_t nsteps, void* work, int64_t work_bytes, double* max_invariant,
                              void* stream);

/* Bytes of the fixed device scratch that wefq_rk_integrate_noalloc uses (64 MiB per device). */
#define WEFQ_RK_NOALLOC_BYTES (64u << 20)

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * time-stepping or serving loops, harnesses that forbid allocation): wefq_rk_integrate without
 * a workspace argument.  The check state and the stage buffers live in a fixed device array of
 * WEFQ_RK_NOALLOC_BYTES inside the library, one per device that the library runs on, held until
 * the process ends; its device address is looked up on the first call on each device.  The call
 * itself allocates nothing (no hipMalloc, hipFree or allocating library routine).  Arguments,
 * results and errors as for wefq_rk_integrate, and WEFQ_EBUDGET when the workspace that
 * wefq_rk_workspace reports for (precision, scheme, B) exceeds WEFQ_RK_NOALLOC_BYTES.  The check
 * state is cleared by a kernel at the start of every call.  Every call on one device shares that
 * device's scratch, which keeps the last call's contents: calls that overlap on one device
 * (several streams or threads) race, so the caller serializes them.  Under graph capture pass
 * max_invariant = NULL (the readback synchronizes the stream). */
wefq_status wefq_rk_integrate_noalloc(wefq_handle h, int32_t precision, int32_t scheme, void* c, int64_t B,
                                      int64_t ld, double dt, int32_t nsteps, double* max_invariant, void* stream);

/* ---- measurement helper ---- */

/* What the rate probe measures. */
typedef enum {
  WEFQ_PROBE_MFMA_F32 = 0,   /* matrix cores, 16x16x4 FP32 */
  WEFQ_PROBE_MFMA_F64 = 1,   /* matrix cores, 16x16x4 FP64 */
  WEFQ_PROBE_MFMA_BF16 = 2,  /* matrix cores, 16x16x32 BF16 with FP32 accumulation */
  WEFQ_PROBE_VALU_F32 = 3,   /* vector ALU, unpacked FP32 fused multiply-add */
  WEFQ_PROBE_VALU_F64 = 4    /* vector ALU, FP64 fused multiply-add */
} wefq_probe_kind;

/* Attainable arithmetic rate of one device, measured so that a kernel's algorithmic rate can
 * be set against a measured peak as well as the datasheet one (not part of the operator).
 * Runs kernels of a few milliseconds that chain independent instructions of the given kind
 * and touch memory only for one store per lane, on 8 workgroups of 256 threads per compute
 * unit, and stores in *tflops the best of five launches in TFLOP/s (a multiply-add counts 2).
 * It allocates and frees a small device buffer, so it is not for graph capture, and it
 * synchronizes stream.  EINVAL for an unknown kind, a null tflops or a bad device ordinal;
 * EHIP on a HIP failure. */
wefq_status wefq_peak_probe(int32_t device, int32_t kind, double* tflops, void* stream);

/* ---- host-only helpers (no device needed), used to test the host tables ---- */

/* Real-Gaunt COO table (Table 1 order: q3 slowest, q1 fastest, 0-based).  Call
 * with null arrays to get *count; then again with arrays of *count entries. */
wefq_status wefq_host_coo(int32_t Lmax, int64_t* count, int32_t* q1, int32_t* q2,
                          int32_t* q3, int32_t* channel, double* g);

/* Gauss rule: kind 0 Gauss-Legendre on [-1,1]; kind 1 generalized Gauss-Laguerre
 * with weight x^alpha e^{-x}.  x and w have n entries. */
wefq_status wefq_host_gauss(int32_t kind, int32_t n, double alpha, double* x, double* w);

#ifdef __cplusplus
}
#endif
#endif /* WEFQ_H */
