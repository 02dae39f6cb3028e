/*
 * hamls.h -- C ABI of the HAMLS hot path on AMD Instinct MI355X (gfx950).
 *
 * HAMLS (harmonic approximation via moving least squares; Hielscher, Poeschl,
 * Wuensche, "Fast and Stable Harmonic Approximation from Ill-distributed Data
 * using Moving Least Squares") turns scattered samples (x_i, y_i) on S2, SO(3)
 * or T3 into the harmonic coefficients of a band-limited approximation
 * (Alg. 1):
 *   step 1  an exact product quadrature grid (Sec. 2.1)
 *   step 2  a moving-least-squares value at every grid node, each from its own
 *           small regularized local polynomial fit (Sec. 2.2, 2.3)
 *   step 3  the adjoint Fourier transform of the quadrature rule (eq. (25))
 *
 * Plain C: no HIP or torch types cross this boundary.  Device buffers are raw
 * pointers into device memory of the current HIP device; streams are passed as
 * void* (a hipStream_t, NULL = the default stream).  All array arguments are
 * FP64 and C-contiguous.  Every call returns a status and never throws; a
 * non-OK status leaves outputs unspecified and plan state unchanged, and
 * hamls_last_error() describes it (thread-local).  Work is enqueued on the
 * given stream and is asynchronous unless a call says otherwise.
 */
#ifndef HAMLS_H
#define HAMLS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    HAMLS_OK = 0,
    HAMLS_ERR_INVALID_ARG = -1,   /* argument outside its documented range */
    HAMLS_ERR_UNSUPPORTED = -2,   /* valid request the library does not handle */
    HAMLS_ERR_OUT_OF_MEMORY = -3, /* device or host allocation failed */
    HAMLS_ERR_DEVICE = -4,        /* HIP runtime error (message in hamls_last_error) */
    HAMLS_ERR_DOMAIN = -5,        /* geometric precondition violated */
    HAMLS_ERR_NOT_EXACT_GRID = -6 /* grid_shape not exact on Pi_{2N} */
} hamls_status;

typedef enum { HAMLS_S2 = 0, HAMLS_SO3 = 1, HAMLS_T3 = 2 } hamls_domain;

/* Regularization of the local problems (Sec. 2.3):
 *  NONE        tau = 0 (plain MLS, eq. (15))
 *  FIXED       tau = tau_fixed for every centre in eq. (22)
 *  CHI_TARGET  tau = 0 where chi <= chi_target; otherwise the tau with
 *              chi_tau = chi_target (eq. (23)), blended in smoothly between
 *              chi_target and chi_full. */
typedef enum { HAMLS_REG_NONE = 0, HAMLS_REG_FIXED = 1, HAMLS_REG_CHI_TARGET = 2 } hamls_reg;

/* Arithmetic of step 2 (and step 3):
 *  FP64   every step in double precision
 *  MIXED  Gram assembly in FP32 with one FP64 residual refinement; centres
 *         that are regularized, ill-conditioned (condition above ~1e4) or
 *         degenerate are solved in FP64 (every domain); on S2 the step-3
 *         contraction in FP32 on the matrix cores (tables generated in FP64).
 *         hamls_plan_tune may keep FP64 kernels for step 2 where they are
 *         faster.  Within 1e-6 relative L2 of FP64. */
typedef enum { HAMLS_FP64 = 0, HAMLS_MIXED = 1 } hamls_precision;

/* Per-centre status bits returned by hamls_diagnostics. */
#define HAMLS_ST_REGULARIZED 1u    /* tau > 0 was used */
#define HAMLS_ST_UNDERDETERMINED 2u /* fewer than m nodes or singular local system: Shepard mean */
#define HAMLS_ST_EMPTY 4u          /* no node inside the support: value NaN */
#define HAMLS_ST_HEMISPHERE 8u     /* support radius clamped (S2: pi/2, SO3: pi) */
#define HAMLS_ST_ILLCOND 16u       /* solved in double-double precision: the FP64 local system was
                                      ill-conditioned, or (one-field FP64 fits, adaptive radius on S2)
                                      the search predicted it from the node's nearest neighbour lying
                                      beyond 0.7 d_n */

typedef struct hamls_params {
    int32_t struct_size;     /* = sizeof(hamls_params); set by hamls_params_init */
    int32_t domain;          /* hamls_domain */
    int32_t bandwidth;       /* N >= 0 (the paper's L) */
    int32_t degree;          /* K in [0, 4] (S2), [0, 3] (SO3, T3); m = C(K+d, d) */
    double support_radius;   /* delta_0 > 0 enables a fixed radius (S2: arc length in rad;
                                SO3: rotation angle in rad; T3: torus units) */
    int32_t knn_count;       /* n >= m enables the adaptive radius of eq. (12) */
    int32_t wendland;        /* weight profile (eq. (6)): 1 = phi_{3,1}, 2 = phi_{3,2} */
    double knn_eps;          /* epsilon > 0 of eq. (12) */
    int32_t reg;             /* hamls_reg */
    int32_t precision;       /* hamls_precision */
    double tau_fixed;        /* tau for HAMLS_REG_FIXED (>= 0) */
    double chi_target;       /* chi_T > 1 */
    double chi_full;         /* chi_full > chi_T */
    int32_t grid_shape[3];   /* 0 = the paper's minimal exact grid; otherwise checked for
                                exactness. S2 (n_theta, n_phi, -), SO3 (n_beta, n_alpha,
                                n_gamma), T3 (n, n, n) */
    int32_t smooth_aux;      /* S2, knn_count > 0, no fixed radius: > 0 smooths the adaptive
                                radius (Sec. 2.2, after eq. (12)): d_n is evaluated on a
                                Fibonacci grid of smooth_aux points and replaced by its
                                degree-zero MLS approximation (Wendland weights, support
                                three mean spacings sqrt(4 pi / smooth_aux)); delta = (1+eps)
                                times that.  0: eq. (12) as it stands */
} hamls_params;

typedef struct hamls_plan_info {
    int32_t domain;
    int32_t bandwidth;
    int32_t degree;
    int32_t m;               /* local ansatz dimension */
    int32_t grid_dims[3];
    int32_t precision;
    int64_t num_grid;        /* M_Q */
    int64_t num_coeffs;      /* length of one field's coefficient vector */
    int64_t num_nodes;       /* M of the bound node set */
    int64_t node_capacity;   /* largest M hamls_plan_rebind accepts without reallocating */
    int64_t resident_bytes;  /* device memory held by the plan */
    int64_t num_cells;       /* binning cells */
} hamls_plan_info;

typedef struct hamls_plan_s* hamls_plan_t;

/* Fill *p with defaults: S2, N = 16, K = 2, kNN n = 4m, eps = 0.05,
 * phi_{3,1}, CHI_TARGET with chi_T = 10, chi_full = 20, FP64. */
hamls_status hamls_params_init(hamls_params* p);

/* Step 1 of Alg. 1 plus the node-side set-up of step 2 (Sec. 2.1, eq. (5),
 * (12)): builds the quadrature grid and its transform tables, bins and sorts
 * the nodes by cell key and computes every grid node's support radius.
 *  nodes        device, M x 3 (S2 unit vectors, T3 points in [0,1)) or M x 4
 *               (SO3 unit quaternions w,x,y,z; q and -q are the same rotation)
 *  node_weights device, M (e.g. Voronoi areas, Sec. 2.2) or NULL for all ones
 *  M            >= 1 and >= knn_count; capacity for later rebinds is M
 * The plan copies what it needs; nodes are not referenced after return.
 * Errors: INVALID_ARG (bad parameters), NOT_EXACT_GRID, DOMAIN (fixed
 * radius: S2 >= pi/2, SO3 > pi, T3 >= 1/2), UNSUPPORTED (degree above 4 on
 * S2 or 3 on SO3 / T3, knn_count above 512 on S2 or 416 on SO3 / T3),
 * OUT_OF_MEMORY, DEVICE. */
hamls_status hamls_plan(const hamls_params* p, const double* nodes, int64_t M,
                        const double* node_weights, void* stream, hamls_plan_t* out);

/* Replace the plan's node set (same parameters) without allocating:
 * M <= node_capacity.  Re-bins, re-sorts and recomputes the radii. */
hamls_status hamls_plan_rebind(hamls_plan_t plan, const double* nodes, int64_t M,
                               const double* node_weights, void* stream);

/* Step 2 of Alg. 1: the MLS value at every grid node (eq. (4), (14)-(23)).
 *  values       device, F rows of M node values; row f starts at values + f*ld
 *  F            1 <= F <= 4096 real fields (complex data: two fields),
 *               solved 16 per pass over the neighbours
 *  ld           >= M
 *  grid_values  device, F x M_Q (row-major, grid order of hamls_plan_grid)
 * Per-centre diagnostics are kept for hamls_diagnostics. */
hamls_status hamls_mls_to_grid(hamls_plan_t plan, const double* values, int32_t F, int64_t ld,
                               double* grid_values, void* stream);

/* Generating functions of MLS (Rem. 2.5), all domains.  The MLS value at a grid
 * node is a linear functional of the data, M_y(q_j) = sum_i a*_ji y_i, whose
 * weights a*_ji depend on the nodes, the radius rule and the regularization
 * only (tau is chosen from the geometry, eq. (23)).  hamls_gen_build computes
 * them for the bound node set (FP64, ill-conditioned nodes in double-double
 * as in hamls_mls_to_grid; also refreshes hamls_diagnostics) and keeps them in
 * the plan as CSR over the grid (one entry per (grid node, neighbour) pair, 12
 * bytes); it synchronizes the stream once (the entry count sizes the
 * storage) and allocates on first use or growth.  A rebind invalidates them.
 * Errors: OUT_OF_MEMORY, DEVICE. */
hamls_status hamls_gen_build(hamls_plan_t plan, void* stream);

/* hamls_mls_to_grid through the generating functions: grid_values[f][j] =
 * sum_i a*_ji values[f][i] (NaN where X(q_j) is empty), one sparse product per
 * 16 fields that reads values in place; same arguments and layouts as
 * hamls_mls_to_grid, equal to it up to rounding (the sums run in another
 * order).  INVALID_ARG if
 * hamls_gen_build has not run since the last bind. */
hamls_status hamls_gen_apply(hamls_plan_t plan, const double* values, int32_t F, int64_t ld,
                             double* grid_values, void* stream);

/* The generating functions as host CSR over the grid: row_ptr (M_Q + 1, equal
 * to that of hamls_plan_neighbors), idx (original node indices ascending per
 * row) and val (a*_ji); idx and val may be NULL.  Synchronizes the device. */
hamls_status hamls_gen_get(hamls_plan_t plan, int64_t* row_ptr, int32_t* idx, double* val);

/* Step 3 of Alg. 1: fhat = F^H W f by the quadrature rule (eq. (25)).
 *  grid_values  device, F x M_Q real
 *  coeffs       device, F x num_coeffs x 2 (re, im).  Index of a coefficient:
 *               S2   n*n + n + k                       (|k| <= n <= N)
 *               SO3  sum_{l<n}(2l+1)^2 + (k+n)(2n+1) + (k'+n)
 *               T3   ((k0+h)*n + (k1+h))*n + (k2+h), h = n/2, k_d in [-h, n-1-h]
 * Bases: S2 orthonormal spherical harmonics with Condon-Shortley phase;
 * SO3 sqrt((2n+1)/8pi^2) e^{-ik alpha} d^n_{k,k'}(beta) e^{-ik' gamma}
 * (Euler ZYZ); T3 e^{2 pi i k.x}. */
hamls_status hamls_grid_to_coeffs(hamls_plan_t plan, const double* grid_values, int32_t F,
                                  double* coeffs, void* stream);

/* Synthesis: out[f*P + i] = Re sum_k fhat_{f,k} phi_k(points_i).
 *  points  device, P x 3 (S2, T3) or P x 4 (SO3) */
hamls_status hamls_eval(hamls_plan_t plan, const double* coeffs, int32_t F, const double* points,
                        int64_t P, double* out, void* stream);

hamls_status hamls_plan_destroy(hamls_plan_t plan);

/* Skewed neighbour counts (ill-distributed nodes under a fixed or hybrid
 * radius: from none in holes to thousands at cluster modes) make a few grid
 * nodes far costlier than the rest; in grid order they can trail at the end
 * of a launch.  hamls_plan_tune measures the one-field assembly pass (FP64,
 * or the mixed FP32 pass with its FP64 list) on the bound nodes in its launch
 * forms -- grid order (0); blocks dispatched in order of decreasing member
 * count (1); on FP64 S2 also a persistent work queue
 * with per-XCD counters handing out grid nodes in that order, at 8 and 12
 * blocks per CU (the block count) -- and keeps the fastest for the plan's
 * later passes (best of three timings each, HIP events on `stream`;
 * synchronizes).  With form 1 the support-radius search of later binds also
 * runs in cost order.  The order is that of the node set at tuning; rebinds
 * keep it (any order gives the same results, only the balance changes).
 * Results are identical in every form.  *queue_blocks receives the choice and
 * times_ms, if not NULL, the four timings in milliseconds (-1 for forms the
 * plan lacks).  On a MIXED plan it also times step 2 (one field, without the
 * extended-precision re-solve) by the FP32-Gram pass with its FP64 list
 * (times_ms[2]) and by the FP64 kernels (times_ms[3]), and runs later step-2
 * calls with the faster; step 3 stays FP32 on the matrix cores.  (Without
 * packed FP32 instructions the FP32 vector rate equals the FP64 rate, so the
 * FP32 Gram pass pays only where it saves memory traffic.)  Both choices are
 * within the mixed bar of the FP64 path. */
hamls_status hamls_plan_tune(hamls_plan_t plan, void* stream, int32_t* queue_blocks, float* times_ms);
/* Routing of predicted ill-conditioned centres (S2, adaptive radius of eq.
 * (12), one-field FP64 step 2, degree >= 1).  The support-radius search flags
 * a centre whose nearest node lies beyond 0.7 d_n: its members form a thin
 * shell (a hole of the node set), the setting in which the FP64 solve hands
 * the centre to the double-double re-solve.  With routing on, a fit's
 * one-field FP64 pass sends the flagged centres to the re-solve without
 * assembling them in FP64 first; the values stay within the FP64 bar either
 * way (only the precision in which a centre is solved changes, and such
 * centres carry HAMLS_ST_ILLCOND).  It pays where most flagged centres need
 * the re-solve anyway.  Off for a new plan; hamls_plan_tune times step 2
 * without and with it on the bound nodes and keeps the faster.  The flags
 * come from the search, which computes them only on plans that route (it
 * costs the search a few percent): switching routing on here takes effect
 * from the next bind (hamls_plan_rebind), switching it off at once.
 *  set       -1 query, 0 off, 1 on
 *  enabled   out (may be NULL): the state after the call
 *  times_ms  out (may be NULL), 2 floats: the tuner's step-2 times without
 *            and with routing, -1 where it did not time them
 * INVALID_ARG for a null plan or set outside {-1, 0, 1}. */
hamls_status hamls_plan_routing(hamls_plan_t plan, int32_t set, int32_t* enabled, float* times_ms);
/* Sets the launch form directly: 0 = grid order, 1 = cost-ordered dispatch,
 * >= 8 = the work queue with that many blocks (the order computed from the
 * bound nodes as in hamls_plan_tune).  INVALID_ARG for 2..7 (the queue needs a
 * block for each of its 8 partitions); UNSUPPORTED for the queue on SO3, T3
 * and mixed plans. */
hamls_status hamls_plan_assembly_form(hamls_plan_t plan, void* stream, int32_t queue_blocks);

/* Introspection of the cost order behind forms >= 1: order (host, M_Q int32)
 * receives the grid nodes by decreasing member count -- buckets of
 * floor(log2(n_j + 1)), heaviest first, grid order within a bucket -- as
 * computed from the member counts of the node set at tuning.  Synchronizes
 * the device.  INVALID_ARG for a null argument or a plan that has no order
 * yet (never tuned nor set to a form >= 1). */
hamls_status hamls_plan_cost_order(hamls_plan_t plan, int32_t* order);

/* ---- captured fits (HIP graphs) ----
 * Steps 2 and 3 on a resident plan have fixed shapes: a fit whose buffers do
 * not change between calls (repeated fields on one node set, a served plan)
 * can be captured once and replayed as one graph launch instead of ~15 kernel
 * launches.  hamls_fit_capture records hamls_mls_to_grid(values, F, ld,
 * grid_values) followed by hamls_grid_to_coeffs(grid_values, F, coeffs) on
 * `stream`, which must not be the default stream, and instantiates the graph
 * (it synchronizes the stream first; step-3 work buffers for F fields are
 * allocated before the capture, and the captured work records no memset).
 * Each hamls_graph_launch reads what values holds when it runs and rewrites
 * grid_values, coeffs and the diagnostics, with the same results as the
 * eager calls.  The graph refers to the plan's buffers: a rebind to the same
 * M that keeps node weights present (or absent) keeps it valid; after a
 * rebind to another M, or one that adds or drops node weights,
 * hamls_graph_launch returns INVALID_ARG.  Destroy graphs before their
 * plan. */
typedef struct hamls_graph_s* hamls_graph_t;
hamls_status hamls_fit_capture(hamls_plan_t plan, const double* values, int32_t F, int64_t ld,
                               double* grid_values, double* coeffs, void* stream, hamls_graph_t* out);
hamls_status hamls_graph_launch(hamls_graph_t graph, void* stream);
hamls_status hamls_graph_destroy(hamls_graph_t graph);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc):
 * hamls_grid_to_coeffs with its step-3 work memory (ring spectra, axis-pass
 * buffers, folded FP32 spectra) taken from a static device array of
 * hamls_noalloc_scratch_bytes() bytes (128 MiB) that each GPU the library runs
 * on holds until the process ends, instead of the plan's own work memory,
 * which hamls_grid_to_coeffs grows (allocates) with the largest F it sees.
 * Arguments, layouts and results as hamls_grid_to_coeffs (the same kernels);
 * the plan's device must be current.  Calls no hipMalloc, hipFree or other
 * allocating routine and records no timing events.  Every call on one GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams or
 * threads) race and must be serialized by the caller.
 * Errors: INVALID_ARG (null pointers, F outside [1, 4096], F whose work
 * memory exceeds the array -- a clear message names the bytes needed -- or a
 * current device other than the plan's), UNSUPPORTED (device index >= 64),
 * DEVICE. */
hamls_status hamls_grid_to_coeffs_noalloc(hamls_plan_t plan, const double* grid_values, int32_t F,
                                          double* coeffs, void* stream);
size_t hamls_noalloc_scratch_bytes(void);

/* Node weights of the paper's ill-distributed recipe (Sec. 2.2, the remark
 * after Thm. 2.1: the weight function rescaled by each node's Voronoi-cell
 * volume; Sec. 3: the data weighted by Voronoi areas): the area of the
 * spherical Voronoi cell {y : y.x_i >= y.x_j for every j} of every bound node,
 * exact up to rounding.
 *  areas   device, M doubles in the caller's node order (sum 4 pi); NaN for a
 *          cell that reaches ~89.99 degrees from its node, holds more than 28
 *          vertices, or belongs to a duplicated node
 * Pass them back as node_weights (hamls_plan_rebind) to weight the fit.
 * Asynchronous on stream.  Errors: INVALID_ARG, UNSUPPORTED (SO3, T3), DEVICE. */
hamls_status hamls_plan_voronoi_areas(hamls_plan_t plan, double* areas, void* stream);

/* Device bytes a plan of these parameters holds for M nodes after a
 * hamls_grid_to_coeffs call with F fields: the sum of its allocations (the
 * capacity of a serving-loop plan, below, counts as M).  Host only; no device
 * call.  Errors: INVALID_ARG, NOT_EXACT_GRID, UNSUPPORTED as for hamls_plan. */
hamls_status hamls_plan_footprint(const hamls_params* p, int64_t M, int32_t F, int64_t* bytes);

/* ---- introspection (host outputs; these calls synchronize the stream) ---- */
hamls_status hamls_plan_info_get(hamls_plan_t plan, hamls_plan_info* out);

/* Grid points (M_Q x 3, or x 4 for SO3) and quadrature weights (M_Q); either
 * pointer may be NULL. */
hamls_status hamls_plan_grid(hamls_plan_t plan, double* points, double* weights);

/* Neighbour sets X(q_j) of eq. (5) as CSR over the grid: row_ptr (M_Q + 1)
 * and idx (row_ptr[M_Q] entries, original node indices ascending per row).
 * Pass idx = NULL to obtain row_ptr only. */
hamls_status hamls_plan_neighbors(hamls_plan_t plan, int64_t* row_ptr, int32_t* idx);

/* Per grid node support radius delta_j and membership threshold c_j
 * (S2: dot > c; SO3: |dot| > c; T3: squared distance < c). */
hamls_status hamls_plan_radii(hamls_plan_t plan, double* delta, double* threshold);

/* Diagnostics of the last hamls_mls_to_grid: neighbour count, chi (eq. (17)),
 * tau, status bits.  Any pointer may be NULL. */
hamls_status hamls_diagnostics(hamls_plan_t plan, int32_t* n, double* chi, double* tau,
                               uint8_t* status);

/* ---- per-phase timing (HIP events on the caller's stream) ----
 * With timing enabled every later call records a start and an end event around
 * each phase it launches.  hamls_timing_read synchronizes, returns the number
 * of launches and the summed event time of one phase, and clears that phase.
 * Phases: HAMLS_PHASE_* below. */
#define HAMLS_PHASE_BINNING 0   /* keys, radix sort, cell table, node gather */
#define HAMLS_PHASE_RADIUS 1    /* support radius / kNN select */
#define HAMLS_PHASE_ASSEMBLE 2  /* local Gram assembly */
#define HAMLS_PHASE_SOLVE 3     /* local regularized solve */
#define HAMLS_PHASE_RING_DFT 4  /* step 3: periodic-angle transforms */
#define HAMLS_PHASE_CONTRACT 5  /* step 3: Legendre / Wigner contraction */
#define HAMLS_PHASE_GATHER 6    /* value gather into sorted order */
#define HAMLS_PHASE_GEN_APPLY 7 /* sparse product with the generating functions */
#define HAMLS_PHASE_RESOLVE 8   /* re-solve of the ill-conditioned centres (extended precision) */
#define HAMLS_PHASE_FOLD 9      /* step 3, S2 mixed: spectra folded into the FP32 contraction blocks and
                                   the blocks unfolded into the coefficient layout */
#define HAMLS_NUM_PHASES 10
hamls_status hamls_timing_enable(hamls_plan_t plan, int32_t enable);
/* Restricts the timing to the phases whose bit (1 << phase) is set in mask
 * (every phase by default): events are recorded around those phases only,
 * since each event pair costs a few microseconds of GPU time. */
hamls_status hamls_timing_phases(hamls_plan_t plan, uint32_t mask);
hamls_status hamls_timing_read(hamls_plan_t plan, int32_t phase, int64_t* launches,
                               double* total_ms);

/* ---- serving loop: continuous batching over resident plans ----
 * The serving extension of Alg. 1: many independent fits (requests), each
 * steps 2 and 3 (hamls_mls_to_grid then hamls_grid_to_coeffs) on its own
 * nodes and parameters, arriving while others run.
 *
 * A server owns `slots` worker threads on the HIP device that is current at
 * creation, each with its own stream (default priority), so the device work of
 * up to `slots` requests overlaps.  Requests wait in arrival order; a free
 * worker admits the oldest one as soon as its device footprint
 * (hamls_plan_footprint at the plan's capacity, plus F x M_Q doubles of grid
 * values) fits within hbm_budget next to the plans of running requests and
 * the idle resident plans; idle plans are evicted, least recently used first,
 * to make room.  While the oldest request cannot fit until running requests
 * finish, a later one (among the next 32) that fits now is admitted ahead of
 * it (backfilling), at most 8 times per waiting request, so that none is
 * starved.  A request whose parameters equal those of an idle resident
 * plan with enough node capacity (at most four times what a new plan would
 * get, since the cell grid follows a plan's first node set) rebinds it (hamls_plan_rebind: no allocation,
 * no grid or table generation); otherwise a plan is built with its capacity
 * rounded up to a power of two (at least 16384 nodes) and stays resident, with
 * its Legendre / Wigner tables, after the request.  A request whose footprint
 * alone exceeds the budget completes with OUT_OF_MEMORY.
 *
 * Inputs (nodes, weights, values) must be complete in device memory when the
 * request is submitted (the workers' streams do not wait for other streams),
 * and must stay valid and unchanged, and coeffs must not be read, until the
 * request's completion is returned.  Results
 * equal those of the plain one-request calls up to rounding of the summation
 * order (a rebound plan keeps the cell grid of its first node set). */
typedef struct hamls_request {
    int32_t struct_size;         /* = sizeof(hamls_request) */
    int32_t F;                   /* fields, 1 <= F <= 4096 */
    hamls_params params;         /* as for hamls_plan */
    const double* nodes;         /* device, as for hamls_plan */
    const double* node_weights;  /* device, M, or NULL */
    int64_t M;
    const double* values;        /* device, F x M (ld = M) */
    double* coeffs;              /* device, F x num_coeffs x 2 (as hamls_grid_to_coeffs) */
    uint64_t tag;                /* returned with the completion */
} hamls_request;

typedef struct hamls_completion {
    uint64_t tag;
    int32_t status;       /* hamls_status of the request */
    int32_t plan_reused;  /* 1: an idle resident plan was rebound */
    double t_submit;      /* seconds on hamls_server_clock: queued */
    double t_admit;       /* admitted by a worker */
    double t_done;        /* coefficients complete in device memory */
} hamls_completion;

typedef struct hamls_server_s* hamls_server_t;

/* slots in [1, 64]; hbm_budget in bytes, <= 0 for 80% of the device memory
 * free at creation. */
hamls_status hamls_server_create(int32_t slots, int64_t hbm_budget, hamls_server_t* out);
/* Queue a request (copied; never blocks on the device).  INVALID_ARG for a
 * malformed request (null pointers, F or M out of range); parameter errors
 * come back in the completion. */
hamls_status hamls_server_submit(hamls_server_t server, const hamls_request* request);
/* Up to max completions, oldest first, into out; *count receives how many.
 * Blocks until at least one is available or timeout_s seconds have passed
 * (timeout_s <= 0: do not block). */
hamls_status hamls_server_wait(hamls_server_t server, hamls_completion* out, int32_t max,
                               int32_t* count, double timeout_s);
/* Requests queued or running, and device bytes committed to plans. */
hamls_status hamls_server_load(hamls_server_t server, int32_t* in_flight, int64_t* committed_bytes,
                               int32_t* resident_plans);
/* Finishes every queued request, then frees the plans, streams and threads.
 * Completions not yet collected are discarded. */
hamls_status hamls_server_destroy(hamls_server_t server);
/* Monotonic clock (seconds) of the completion time stamps. */
double hamls_server_clock(void);

const char* hamls_status_string(hamls_status s);
const char* hamls_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HAMLS_H */
