/*
 * fmm.h -- C ABI of libfmm_mi355x.so, a fast multipole evaluation of the
 * velocity induced by N two-dimensional vortex particles, written for the
 * AMD Instinct MI355X (gfx950).
 *
 * What one evaluation computes (Cruz, Knepley & Barba, "PetFMM"):
 *   u(x_i) = sum_{j != i} gamma_j K(x_i - x_j)                    (Section 3, eq. 9)
 * where K is the Gaussian-regularised Biot-Savart kernel of eq. 8,
 *   K_sigma(x) = (-x2, x1) (1 - exp(-|x|^2 / (2 sigma^2))) / (2 pi |x|^2),
 * for pairs whose leaves touch, and the singular kernel of eq. 7 (through
 * its multipole and local expansions) for every other pair -- the kernel
 * substitution described after eq. 9.  The tree is a uniform quadtree of
 * depth L over a square domain (Section 2.1); the steps are the upward sweep
 * (P2M, M2M), the downward sweep (M2L over the interaction list, L2L) and
 * the evaluation step (L2P plus near-field direct interactions), Section 2.2
 * and Fig. 2.  Expansions have p complex terms, k = 0 .. p-1 ("truncated
 * after p terms", Section 2; 16p bytes per box in Table 1).
 * A plan may choose another kernel (fmm_params.kernel, Sections 6.1 and 8):
 * the singular kernel of eq. 7 in the near field, Lennard-Jones forces (near
 * field only), or the discrete Gauss transform by the fast Gauss transform.
 * The fmm3d_* entry points at the end carry the method to three dimensions
 * (Section 8): a uniform octree with the Laplace kernel 1/r.
 *
 * Conventions shared by every entry point:
 *   - Every function returns an fmm_status; no C++ exception crosses the ABI.
 *   - "Device pointer" means memory on the current HIP device (hipMalloc or a
 *     PyTorch CUDA/HIP tensor).  The library never frees caller memory.
 *   - "stream" is a hipStream_t passed as void* (NULL = the default stream).
 *     fmm_evaluate, fmm_evaluate_at, fmm_evaluate_batch and fmm3d_evaluate only enqueue work on
 *     it (the batched form as one table kernel and one graph launch): they never
 *     synchronise, never allocate device memory and never read device data
 *     back to the host.
 *   - A plan is not re-entrant: two evaluations of one plan must not overlap
 *     (they share the workspace).  Separate plans are independent.
 *   - Self-interaction and coincident particles contribute exactly 0 (the
 *     kernel of eq. 8 tends to 0 at the origin).  The boundary is free space.
 *   - Outputs are written (not accumulated) in the caller's input order.
 */
#ifndef FMM_MI355X_H
#define FMM_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fmm_plan_s* fmm_plan_t;          /* opaque host handle */

typedef enum {
    FMM_OK = 0,
    FMM_E_ARG = -1,          /* invalid argument (checked on the host, synchronously) */
    FMM_E_CAPACITY = -2,     /* n larger than the plan's capacity, or workspace too small */
    FMM_E_DOMAIN = -3,       /* fmm_get_status: particles outside the explicit domain or NaN
                                (or all of them, the bounding square being wider than 1e36) */
    FMM_E_NOMEM = -4,        /* host allocation failed */
    FMM_E_DEVICE = -5,       /* a HIP runtime call failed */
    FMM_E_UNSUPPORTED = -6   /* valid but not supported combination (e.g. p too large for FP32) */
} fmm_status;

typedef enum {
    FMM_PREC_FP64 = 0,       /* every stage in FP64 */
    FMM_PREC_MIXED = 1       /* FP32 near field and fine-level M2L; FP64 shifts and coarse M2L */
} fmm_precision;

/* Pair kernel of the near field.  Section 6.1 templates the evaluator over
 * its kernel so that one equation can replace another; Section 8 names
 * further kernels, among them the Lennard-Jones potential of molecular
 * dynamics.  For the two vortex kernels the far field uses the expansions of
 * the singular kernel (Section 3, text after eq. 9), so the choice only
 * changes the direct sum over touching leaves. */
typedef enum {
    FMM_KERNEL_GAUSSIAN = 0, /* regularised Biot-Savart kernel of eq. 8, core sigma > 0 */
    FMM_KERNEL_SINGULAR = 1, /* singular Biot-Savart kernel of eq. 7 (point vortices); sigma is
                                ignored; a pair at zero distance contributes nothing */
    FMM_KERNEL_LENNARD_JONES = 2,
                             /* Lennard-Jones force, V(r) = 4 eps ((s/r)^12 - (s/r)^6) for
                                0 < r < cutoff, 0 beyond (truncated, not shifted): d_u, d_v
                                receive the force sum_j 24 eps (2 (s/r)^12 - (s/r)^6) (x_i -
                                x_j) / r^2; s = sigma > 0, eps = lj_epsilon > 0, d_gamma is
                                ignored.  Short range, so there is no far field: the tree
                                serves as a cell list, and the cutoff may not exceed the leaf
                                width width / 2^depth (else FMM_E_UNSUPPORTED; a pair closer
                                than the cutoff by no more than a rounding error at a leaf
                                edge may be missed).  Needs an explicit square and FP64;
                                fmm_evaluate and the batched form only */
    FMM_KERNEL_GAUSS_TRANSFORM = 3
                             /* the discrete Gauss transform (Section 8 names the fast
                                Gauss transform): d_u receives G_i = sum_j gamma_j
                                exp(-|x_i - x_j|^2 / (2 sigma^2)) (the term j = i
                                included), d_v is cleared.  Computed by Greengard and
                                Strain's fast Gauss transform on the 4^depth leaf boxes:
                                p Hermite terms per axis (p <= 16) for every box, Hermite
                                to Taylor translation between boxes within Chebyshev
                                distance nc = ceil(sqrt(ln 1e16) sqrt(2) sigma / w) (w the
                                leaf width; a left-out term is below 1e-16 of its source's
                                strength), Taylor evaluation at the particles.  The error
                                falls with p and with w / sigma: w <= sigma and p = 12-16
                                give 1e-10 to 1e-14 relative.  Needs an explicit square,
                                FP64, a single-instance plan, nc <= 63 (else
                                FMM_E_UNSUPPORTED); fmm_evaluate, and fmm_evaluate_at
                                for the transform at target points.  Stage timing
                                reports the transform's three launches under "p2m_m2m" */
} fmm_kernel;

/* Problem parameters, following the paper's problem statement: positions
 * and circulations (eq. 9), one core size sigma for all particles
 * (Section 7.1), expansion order p and tree level (Section 7.2). */
typedef struct {
    int64_t n_max;            /* capacity: largest n passed to fmm_evaluate (>= 0, < 2^31) */
    double  sigma;            /* Gaussian core size, >= 1e-30 (eqs. 5 and 8); ignored by the singular
                                 kernel; the length s of the Lennard-Jones kernel; the width
                                 of the Gauss transform's exp(-r^2 / (2 sigma^2)) */
    int32_t p;                /* number of expansion terms, 1 <= p <= 32 (<= 22 in mixed mode;
                                 Hermite terms per axis, <= 16, for the Gauss transform) */
    int32_t depth;            /* leaf level L, 0 <= L <= 13; levels 0..L, 4^L leaves */
    double  x0, y0, width;    /* domain [x0, x0+width]^2, width <= 1e36; width <= 0 selects
                                 the bounding square of the particles, recomputed at every
                                 evaluation (one wider than 1e36 counts every particle as
                                 outside, FMM_E_DOMAIN) */
    int32_t precision;        /* an fmm_precision value */
    int32_t fp32_fine_levels; /* mixed mode: M2L at levels > L - fp32_fine_levels runs in
                                 FP32 (0 .. L-1); ignored in FP64 mode */
    int64_t m_max;            /* capacity: largest m passed to fmm_evaluate_at (>= 0, < 2^31);
                                 0 = no target points.  Single-instance plans only */
    int32_t kernel;           /* an fmm_kernel value (0: the Gaussian kernel of eq. 8) */
    double  lj_epsilon;       /* Lennard-Jones energy eps (kernel FMM_KERNEL_LENNARD_JONES only) */
    double  cutoff;           /* Lennard-Jones cutoff (kernel FMM_KERNEL_LENNARD_JONES only) */
    int32_t max_instances;    /* 0 or 1: the single form (fmm_evaluate); 2 .. 65536: the batched
                                 form (fmm_evaluate_batch), at most this many instances per call;
                                 n_max then caps their total particle count and depth their
                                 deepest tree */
    int64_t max_leaves;       /* batched form: capacity for sum over a call's instances of
                                 4^depth_i (leaf boxes; the expansions of all levels are sized
                                 from it); 0 = max_instances * 4^depth, the worst case */
} fmm_params;

/* Number of bytes of device workspace a plan with these parameters needs
 * (either form, after prm->max_instances).  Host only; touches no device.  Errors: FMM_E_ARG for invalid parameters
 * or a NULL pointer, FMM_E_UNSUPPORTED for p > 22 in mixed mode and for the
 * kernel-specific limits listed with fmm_kernel. */
fmm_status fmm_workspace_size(const fmm_params* prm, size_t* bytes);

/* Create a plan.  d_workspace: caller-owned device buffer of at least
 * fmm_workspace_size() bytes, 256-byte aligned, kept alive and unused by
 * anyone else until fmm_destroy.  The operator tables (M2M, L2L shifts and
 * the M2L translation data, derived from the expansions of 1/z) are built on
 * the host in FP64 and copied into the workspace on `stream`.  *out receives a
 * host handle.  Errors: FMM_E_ARG (NULL pointers, invalid parameters),
 * FMM_E_CAPACITY (bytes too small), FMM_E_NOMEM, FMM_E_DEVICE. */
fmm_status fmm_plan(const fmm_params* prm, void* d_workspace, size_t bytes,
                    void* stream, fmm_plan_t* out);

/* One full FMM evaluation: tree build (z-order keys, stable radix sort by
 * leaf, leaf ranges), P2M, M2M, M2L, L2L, L2P and P2P (Section 2.2).
 *   n                  number of particles, 0 <= n <= n_max
 *   d_x, d_y, d_gamma  device FP64 arrays [n]: positions and circulations
 *   d_u, d_v           device FP64 arrays [n]: velocity components (eq. 9),
 *                      overwritten, in input order (with the Lennard-Jones
 *                      kernel: the force, after the tree and the near field
 *                      alone)
 * Asynchronous on `stream`; kernels only (no allocation, no memset, no
 * synchronisation), so a caller may capture it into a graph.  Particles outside an explicit domain (or with a
 * NaN coordinate) are clamped into the nearest leaf and counted; read the
 * count with fmm_get_status.  Errors (synchronous): FMM_E_ARG (NULL plan or
 * pointers with n > 0), FMM_E_CAPACITY (n > n_max), FMM_E_DEVICE. */
fmm_status fmm_evaluate(fmm_plan_t plan, int64_t n,
                        const double* d_x, const double* d_y, const double* d_gamma,
                        double* d_u, double* d_v, void* stream);

/* The velocity at m target points distinct from the particles: the sum of
 * eq. 1 with the regularised kernel (eqs. 5 and 8), evaluated by the same
 * FMM.  The target points are sorted into the particles' tree; each takes
 * L2P from its leaf's local expansion and the regularised near field from
 * the particles of its leaf and the touching leaves (Section 2.2).  A point
 * on top of a particle gets nothing from it (the regularised kernel
 * vanishes at zero distance).
 *   n, d_x, d_y, d_gamma  particles as for fmm_evaluate, 0 <= n <= n_max
 *   m                     number of target points, 0 <= m <= m_max
 *   d_tx, d_ty            device FP64 arrays [m]: target positions
 *   d_u, d_v              device FP64 arrays [m]: velocity at the points,
 *                         overwritten, in input order (zero when n == 0)
 * With the bounding-square domain (width <= 0) the square bounds the
 * particles and the points together.  Points outside an explicit domain or
 * with a NaN coordinate are clamped into the nearest leaf and counted with
 * the particles (fmm_get_status).  m == 0 does nothing.  Asynchronous on
 * `stream`.  FP64 single-instance plans only.  Errors (synchronous):
 * FMM_E_ARG (NULL plan or pointers, negative counts, a batched plan),
 * FMM_E_UNSUPPORTED (a mixed-precision or Lennard-Jones plan), FMM_E_CAPACITY
 * (n > n_max or m > m_max), FMM_E_DEVICE.  A Gauss transform plan writes the
 * transform at the points into d_u (d_v cleared). */
fmm_status fmm_evaluate_at(fmm_plan_t plan, int64_t n, const double* d_x, const double* d_y,
                           const double* d_gamma, int64_t m, const double* d_tx, const double* d_ty,
                           double* d_u, double* d_v, void* stream);

/* Batched form (Sections 4 and 5.2: many trees of uneven size, and sizes
 * that change from call to call): a plan made with prm->max_instances >= 2
 * fixes capacities only -- n_max particles in total, max_instances
 * instances, trees no deeper than prm->depth, max_leaves leaf boxes in
 * total -- and every call evaluates the instance set it is given, each
 * instance exactly as fmm_evaluate would (the same operation and kernels,
 * the same results bit for bit), sharing sigma, p, precision, kernel and one
 * explicit square [x0, x0+width]^2 (width <= 0: FMM_E_UNSUPPORTED; m_max
 * must be 0, else FMM_E_ARG; the Gauss transform: FMM_E_UNSUPPORTED;
 * ceil(log2 max_instances) + 2 depth <= 32, else FMM_E_UNSUPPORTED).
 *   n_inst      instances of this call, 1 <= n_inst <= max_instances (host)
 *   d_offsets   device int64 [n_inst + 1]: CSR offsets into the arrays below;
 *               instance i owns entries [d_offsets[i], d_offsets[i+1]),
 *               d_offsets[0] = 0, non-decreasing
 *   d_depths    device int32 [n_inst]: tree depth of every instance, 0 .. depth
 *   d_x .. d_v  device FP64 arrays of d_offsets[n_inst] entries, as for
 *               fmm_evaluate, results in the same order
 * The instance table is read on the device: one kernel validates it against
 * the capacities, lays out the instances' segments, orders them by the
 * paper's work estimate (eqs. 13-15, heaviest first; see
 * fmm_work_estimate) and writes the work tables of every launch; the stage
 * kernels are launched with grids sized for the capacities, and a
 * workgroup past its launch's work returns at once.  The first call with a
 * given set of the five arrays captures those launches into a HIP graph (on
 * a stream the plan owns); later calls with the same arrays -- whatever
 * their instance sets -- run the table kernel and replay the graph on
 * `stream`.  An instance set that does not fit the capacities, or is
 * malformed, computes nothing (d_u, d_v are left as they were) and
 * fmm_get_status then returns FMM_E_CAPACITY or FMM_E_ARG.  Calls on one
 * plan must not overlap.  Errors (synchronous): FMM_E_ARG (a single-instance
 * plan, n_inst out of range, NULL pointers), FMM_E_DEVICE.
 * fmm_get_status and fmm_debug_dump (KEYS and PERM over n_max entries,
 * LEAF_START over the leaf capacity: the segments of the call's instances,
 * 4^depth_i + 1 entries each, come first) work as for a single plan.  With
 * stage timing on (fmm_set_timing) the launches are enqueued eagerly, with
 * the stage events between them, instead of replayed. */
fmm_status fmm_evaluate_batch(fmm_plan_t plan, int32_t n_inst, const int64_t* d_offsets, const int32_t* d_depths,
                              const double* d_x, const double* d_y, const double* d_gamma, double* d_u, double* d_v,
                              void* stream);

/* Vortex-method time stepping (Section 3, eq. 6: in ideal 2D flow every
 * particle moves with its velocity and keeps its circulation).  Advances
 * d_x, d_y (device FP64 [n], in place; d_gamma unchanged) by n_steps steps
 * of the explicit midpoint rule, the paper naming no integrator:
 *   x_mid = x + dt/2 u(x),   x <- x + dt u(x_mid),
 * each velocity a full evaluation of this plan (tree rebuilt every stage).
 * d_scratch: caller-owned device FP64 [4 n] (stage velocities and midpoint
 * positions), overwritten.  A single-instance plan only; use the bounding-
 * square domain (width <= 0) or an explicit square the particles stay in
 * (escapes are counted as by fmm_evaluate: fmm_get_status reports the last
 * evaluation).  The first call for a given set of arrays, n and dt captures
 * one step into a HIP graph (on a stream the plan owns); every step is a
 * replay of it on `stream`.  Asynchronous.  Errors: FMM_E_ARG (batched plan,
 * NULL pointers, n < 0, n_steps < 0, dt not finite), FMM_E_CAPACITY,
 * FMM_E_DEVICE. */
fmm_status fmm_advance_rk2(fmm_plan_t plan, int64_t n, double* d_x, double* d_y, const double* d_gamma,
                           double dt, int32_t n_steps, double* d_scratch, void* stream);

/* Launch shapes.  p2p_waves: leaves (one wavefront each) per P2P workgroup,
 * 2 or 4 (default 4).  m2l_split_max: M2L levels <= min(L, m2l_split_max)
 * split each box's interaction list over two or three wavefronts (more
 * parallelism on levels with few boxes), 0 .. 8 (default 8; below 2: never).
 * m2l_mfma: 1 runs the FP32 M2L levels of the mixed form whose lists are not
 * split (those above m2l_split_max) on the matrix cores (MFMA), 0 (default)
 * on the vector units with the interaction-list members taken in symmetric
 * pairs, as the FP64 levels and all split levels always are.  work_order (batched plans): 1 (default) launches the
 * instances of every stage in decreasing order of the paper's work estimate
 * (eqs. 13-15, see fmm_work_estimate), so the heaviest workgroups are
 * dispatched first; 0 keeps the input order.  p2p_block chooses how a
 * near-field wavefront lays out a chunk of t target particles (t <= 64):
 * R targets per lane, TG = ceil(t / R) lanes per target group and S source
 * slices (S x TG <= 64 lanes); 0 (the default of a mixed plan) pads t to a
 * power of two (R = 4 at 64 targets, 2 at 32, else 1), 1 (the default of an
 * FP64 plan) keeps the most lanes on real pairs (largest t S / (64 R), the
 * larger R on a tie).  Results are identical up
 * to the summation order (bit for bit for work_order).
 * fmm_set_tuning synchronises `stream`.  fmm_autotune times candidates from
 * p2p_waves in {2, 4} x p2p_block in {0, 1}, m2l_split_max in {0, 5, 8} and, for a mixed plan,
 * m2l_mfma in {0, 1} on the caller's data (reps timed evaluations each,
 * after one warm-up; the output arrays are overwritten) and keeps the
 * fastest.  The search is seeded by the paper's work model (Section 5.2):
 * the estimate of eqs. 13-15 is split into its near-field part (n_nd N_i^2
 * and 2 N_i p per leaf) and its far-field part (p^2 (2 n_c + n_IL) per
 * non-leaf box, p^2 n_IL per leaf); starting from the current shape, the
 * knobs of the larger part (near field: p2p_waves, p2p_block; far field: the M2L
 * knobs) are searched first, those of the smaller part only when it holds at
 * least 10 % of the estimate.  The environment variable
 * FMM_AUTOTUNE_EXHAUSTIVE=1 times the whole grid instead.  When
 * FMM_AUTOTUNE_CACHE names a file, the choice is looked up there first and
 * appended after a search (one line per choice: the problem's signature,
 * then p2p_waves, m2l_split_max, m2l_mfma and p2p_block; the last line with
 * the signature wins).  For batched plans n is ignored and the instance set of the plan's
 * last fmm_evaluate_batch call is timed (FMM_E_ARG before the first call). */
fmm_status fmm_get_tuning(fmm_plan_t plan, int32_t* p2p_waves, int32_t* m2l_split_max, int32_t* m2l_mfma,
                          int32_t* work_order, int32_t* p2p_block);
fmm_status fmm_set_tuning(fmm_plan_t plan, int32_t p2p_waves, int32_t m2l_split_max, int32_t m2l_mfma,
                          int32_t work_order, int32_t p2p_block, void* stream);
fmm_status fmm_autotune(fmm_plan_t plan, int64_t n, const double* d_x, const double* d_y,
                        const double* d_gamma, double* d_u, double* d_v, void* stream, int32_t reps);
/* The plan's last fmm_autotune: the number of candidates it timed (0 when
 * the choice came from the cache) and the near-field share of the work
 * model's estimate that ordered the search.  Host only. */
fmm_status fmm_autotune_report(fmm_plan_t plan, int32_t* candidates_timed, double* near_share);

/* The paper's work model (Section 5.2) for every instance of the plan, in
 * input order: non-leaf boxes p^2 (2 n_c + n_IL) each (eq. 13), leaves
 * 2 N_i p + p^2 n_IL + n_nd N_i^2 each (eq. 14), summed over the tree of
 * depth L (eq. 15), with n_c = 4, n_IL = 27, n_nd = 9 and the mean leaf
 * occupancy N_i = N / 4^L (N = n_max for a single-instance plan; for a
 * batched plan the instances of its last fmm_evaluate_batch call, whose
 * estimates the device computed for the launch order: the call waits for
 * that call's stream).  Writes min(n_out, instances) values; *n_written (may
 * be NULL) gets that count. */
fmm_status fmm_work_estimate(fmm_plan_t plan, double* work, int32_t n_out, int32_t* n_written);

/* Synchronises `stream` and reports the number of particles of the last
 * evaluation (with fmm_evaluate_at: particles and target points) that fell
 * outside the explicit domain or had a NaN coordinate.
 * Returns FMM_OK if there were none, FMM_E_DOMAIN otherwise; for a batched
 * plan whose last call's instance set was rejected on the device,
 * FMM_E_CAPACITY or FMM_E_ARG (with *n_bad = 0). */
fmm_status fmm_get_status(fmm_plan_t plan, void* stream, int64_t* n_bad);

/* Stage timing.  fmm_set_timing(plan, 1) clears the totals; every later
 * evaluation records HIP events on its own stream between its stages (no
 * synchronisation: a ring of 32 event sets is drained as it wraps).
 * fmm_stats synchronises and writes, for up to n_stages stages in the order
 * of fmm_stage_name, the average GPU time in milliseconds over every timed
 * evaluation since fmm_set_timing(plan, 1); *n_written gets the number of
 * stages written and *n_evaluations (may be NULL) the number of evaluations
 * averaged.  FMM_E_ARG if nothing was timed. */
fmm_status fmm_set_timing(fmm_plan_t plan, int32_t on);
fmm_status fmm_stats(fmm_plan_t plan, double* stage_ms, int32_t n_stages, int32_t* n_written,
                     int64_t* n_evaluations);
const char* fmm_stage_name(int32_t stage);

/* Parity inspection (not on the hot path).  Waits for the stream of the
 * plan's last evaluation (before any: the stream given to fmm_plan) and
 * copies one of the plan's device arrays from that evaluation into host_buf,
 * on that stream; it allocates no device memory:
 *   FMM_DUMP_KEYS       uint32 [n]      leaf z-order key of every particle (input order)
 *   FMM_DUMP_PERM       uint32 [n]      sorted position -> input index
 *   FMM_DUMP_LEAF_START int32 [4^L+1]   sorted range of every leaf, z-order (batched:
 *                                       the segments of all instances, 4^L_i+1 each)
 *   FMM_DUMP_ME         complex128 [Lambda][p] scaled multipole coefficients
 *   FMM_DUMP_LE         complex128 [Lambda][p] scaled local coefficients
 *   FMM_DUMP_DOMAIN     double [4]      x0, y0, width, 2^L / width
 *   FMM_DUMP_ILIST      int32 [Lambda][27]  interaction list of every box as
 *                       global box ids, -1 padded, as the M2L kernel walks it
                       (single-instance plans; written in chunks into the
                       workspace's sort temporaries, which every tree build
                       rewrites, and copied out chunk by chunk)
 *   FMM_DUMP_TKEYS, FMM_DUMP_TPERM, FMM_DUMP_TLEAF_START  the same three
 *                       arrays for the m target points of the last
 *                       fmm_evaluate_at (empty after other evaluations)
 * Boxes are numbered per level in z-order from (4^l - 1)/3 (the global box
 * numbering of Section 6.2).  Scaled coefficients: a_k = ahat_k * w_l^k and
 * b_l = bhat_l / w_l^(l+1), w_l the box width at level l.  If bytes is too
 * small, *needed is set and FMM_E_CAPACITY returned. */
enum {
    FMM_DUMP_KEYS = 0, FMM_DUMP_PERM = 1, FMM_DUMP_LEAF_START = 2,
    FMM_DUMP_ME = 3, FMM_DUMP_LE = 4, FMM_DUMP_DOMAIN = 5, FMM_DUMP_ILIST = 6,
    FMM_DUMP_TKEYS = 7, FMM_DUMP_TPERM = 8, FMM_DUMP_TLEAF_START = 9
};
fmm_status fmm_debug_dump(fmm_plan_t plan, int32_t what, void* host_buf,
                          size_t bytes, size_t* needed);

/* For callers that cannot allocate device memory (code under graph capture,
 * tight serving loops, harnesses that forbid allocation): one full
 * evaluation exactly as fmm_plan + fmm_evaluate compute it with the same
 * parameters (same kernels, same results bit for bit), whose workspace is a
 * fixed array of FMM_STATIC_SCRATCH_BYTES bytes of device memory that the
 * library holds on every GPU it is loaded on until the process ends.  It
 * allocates no device memory and creates no plan handle for the caller.
 *   prm                single-instance parameters as for fmm_plan; the
 *                      workspace they need (fmm_workspace_size) must fit in
 *                      FMM_STATIC_SCRATCH_BYTES, else FMM_E_CAPACITY (checked
 *                      on the host, nothing enqueued)
 *   n, d_x .. d_v      as for fmm_evaluate (0 <= n <= prm->n_max)
 * The first call on a device, and every call whose parameters differ from
 * the previous call's on that device, uploads the operator tables into the
 * array on `stream` and waits for it; later calls with the same parameters
 * only enqueue kernels.  All calls on one GPU share its array: calls whose
 * work overlaps on one GPU (other streams, other host threads) race and
 * their results are undefined.  No stage timing, status word or inspection.
 * Errors: FMM_E_ARG, FMM_E_CAPACITY, FMM_E_UNSUPPORTED and FMM_E_DEVICE as
 * for fmm_plan and fmm_evaluate. */
#define FMM_STATIC_SCRATCH_BYTES (64u << 20)
fmm_status fmm_evaluate_static(const fmm_params* prm, int64_t n, const double* d_x, const double* d_y,
                               const double* d_gamma, double* d_u, double* d_v, void* stream);

/* Release the host handle, its HIP events, captured graph and private
 * stream.  Never frees the workspace or any other caller memory.  NULL is
 * accepted. */
fmm_status fmm_destroy(fmm_plan_t plan);

/* Static description of a status code. */
const char* fmm_status_string(fmm_status s);

/* ---- 3D form ------------------------------------------------------------
 * The method on a uniform octree (Section 8: in 3D the tree, the sweeps and
 * the lists stay; the kernel, its series expansions and translation
 * operators change), for the Laplace kernel 1/r:
 *     phi(x_i)      = sum_{j != i} q_j / |x_i - x_j|
 *     grad phi(x_i) = sum_{j != i} -q_j (x_i - x_j) / |x_i - x_j|^3
 * (pairs at zero distance contribute nothing).  Near field = the leaf and
 * the 26 leaves touching it, evaluated directly; interaction list = the up
 * to 189 boxes of the same level whose parents touch the box's parent but
 * which do not touch the box.  Far field through Cartesian Taylor
 * expansions of total degree <= p ((p+1)(p+2)(p+3)/6 terms per box): P2M,
 * M2M, M2L, L2L, L2P.  FP64 throughout.  The 3D vortex velocity is the curl
 * of three such potentials (one per vorticity component); that combination
 * is left to the caller.
 *
 * Particles must lie in the cube [x0, x0 + width)^3; one outside it (or with
 * a NaN coordinate) gets zero outputs, acts on nothing and is counted by
 * fmm3d_get_status.  Same workspace, stream and error conventions as the 2D
 * entry points: the caller owns the 256-byte aligned device workspace; the
 * evaluation only enqueues work on the stream. */
typedef struct fmm3d_plan_s* fmm3d_plan_t;     /* opaque host handle */

typedef struct {
    int64_t n_max;      /* particle capacity, 0 .. 2^31 - 1 */
    int32_t p;          /* expansion degree, 0 .. 9 (FMM_E_UNSUPPORTED above) */
    int32_t depth;      /* octree depth L, 0 .. 7 (8^L leaves; FMM_E_UNSUPPORTED above);
                           L <= 1 leaves no far field: the direct sum */
    double x0, y0, z0;  /* lower corner of the cube */
    double width;       /* its side, > 0 */
} fmm3d_params;

/* Bytes of device workspace a plan with these parameters needs.  Host only.
 * Errors: FMM_E_ARG (NULL, negative or non-finite values), FMM_E_UNSUPPORTED
 * (p > 9 or depth > 7). */
fmm_status fmm3d_workspace_size(const fmm3d_params* prm, size_t* bytes);

/* Bind the parameters to a workspace of at least fmm3d_workspace_size bytes
 * (256-byte aligned, else FMM_E_ARG; smaller: FMM_E_CAPACITY).  Uploads the
 * M2L derivative table on `stream` and waits for it. */
fmm_status fmm3d_plan(const fmm3d_params* prm, void* d_workspace, size_t bytes, void* stream,
                      fmm3d_plan_t* out);

/* Potential and gradient at the n particles (device FP64 arrays of length
 * n, outputs in input order).  n > n_max: FMM_E_CAPACITY.  Enqueues only. */
fmm_status fmm3d_evaluate(fmm3d_plan_t plan, int64_t n, const double* d_x, const double* d_y,
                          const double* d_z, const double* d_q, double* d_phi, double* d_gx,
                          double* d_gy, double* d_gz, void* stream);

/* Waits for `stream` and reports the particles the last evaluation found
 * outside the cube: FMM_E_DOMAIN if there were any. */
fmm_status fmm3d_get_status(fmm3d_plan_t plan, void* stream, int64_t* n_outside);

/* Parity inspection of the last evaluation's tree (waits for the device):
 *   FMM_DUMP_KEYS        uint32 [n]        3D Morton leaf key per input particle
 *                        (2^(3 depth) for one outside the cube)
 *   FMM_DUMP_PERM        uint32 [n]        sorted position -> input index (stable)
 *   FMM_DUMP_LEAF_START  int32 [8^depth+1] first sorted position of every leaf;
 *                        the last entry counts the particles inside the cube
 * Other kinds: FMM_E_ARG.  If bytes is too small, *needed is set and
 * FMM_E_CAPACITY returned. */
fmm_status fmm3d_debug_dump(fmm3d_plan_t plan, int32_t what, void* host_buf, size_t bytes, size_t* needed);

/* Release the host handle (never the workspace).  NULL is accepted. */
fmm_status fmm3d_destroy(fmm3d_plan_t plan);

#ifdef __cplusplus
}
#endif

#endif /* FMM_MI355X_H */
