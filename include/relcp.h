/*
 * relcp.h -- C ABI of the MI355X ReLCP time-step library (librelcp.so).
 *
 * One ReLCP time-step for frictionless contact between smooth rigid bodies
 * (ellipsoids, spherocylinders), after Palmer, Aktulga, Gao, "Smooth-Rigid-
 * Body Contact as a ReLCP" (arXiv 2506.14097): Alg. 1 (overdamped) and Eq.
 * relcp_inertial (inertial).  Each call states the passage it implements.
 *
 * Conventions
 *  - Every call returns an int status: RELCP_OK (0) or a negative RELCP_E_*.
 *    Nothing is thrown across the ABI; relcp_last_error() gives a message.
 *  - The library owns the context and all of its device buffers.  Inputs
 *    are copied at create / set time; the caller may free them afterwards.
 *  - Host arrays are array-of-structs per body in double precision: x[3i+k],
 *    q[4i+k] with the scalar part first (q = [s, w]), velocities u[3i+k]
 *    (translation) and w[3i+k] (world-frame angular velocity).  Functions
 *    with the _device suffix take device pointers of the same layout and work
 *    on the context's stream.
 *  - One context per stream; calls on one context are not thread-safe.
 *  - Units are the caller's; all lengths, times and forces consistent.
 *  - Errors leave the state untouched: a step commits only on acceptance.
 *  - relcp_step and relcp_affine_rescale may return before the last of
 *    their device work has run (it is ordered on the context's stream);
 *    every call that reads results back waits for it.
 */
#ifndef RELCP_H
#define RELCP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#ifndef RELCP_API
#define RELCP_API __attribute__((visibility("default")))
#endif

typedef struct relcp_ctx relcp_ctx;

enum {
    RELCP_OK = 0,
    RELCP_E_INVALID = -1,       /* bad argument: NaN, non-unit quaternion, bad shape, box too small */
    RELCP_E_OOM = -2,           /* device allocation failed */
    RELCP_E_DEVICE = -3,        /* HIP runtime error */
    RELCP_E_LCP_MAXITER = -4,   /* projected gradient did not reach lcp_tol within lcp_max_iters */
    RELCP_E_RECURSION_CAP = -5, /* more than max_recursions augmentations (Alg. 1 while-loop) */
    RELCP_E_SKIN = -6,          /* a trial moved a surface point by more than skin/2 */
    RELCP_E_NAN = -7,           /* non-finite value produced during the step */
    RELCP_E_CAPACITY = -8       /* contact or pair buffer would exceed the configured maximum */
};

enum { RELCP_ELLIPSOID = 0, RELCP_SPHEROCYLINDER = 1, RELCP_TORUS = 2 };
enum { RELCP_OVERDAMPED = 0, RELCP_INERTIAL = 1 };
enum { RELCP_WS_COLD = 0, RELCP_WS_PREV = 1, RELCP_WS_LEARNED = 2 };

/* Bodies (generalized configuration C, Sec. 2.1.1): n bodies in n_batch
 * independent systems ("packings").  Bodies of packing p are
 * [batch_off[p], batch_off[p+1]).  box[3p+k] is the periodic box edge of
 * packing p along k, 0 for an open direction.  u, w may be NULL (at rest).
 * batch_off may be NULL when n_batch == 1. */
typedef struct {
    int32_t n;
    const double *x, *q, *u, *w;
    int32_t n_batch;
    const int32_t *batch_off;
    const double *box;
} relcp_bodies;

/* Shapes: kind[i] = RELCP_ELLIPSOID with p[3i..] = semiaxes (a, b, c) along
 * the body x, y, z axes; or RELCP_SPHEROCYLINDER with p[3i..] = (r, l, 0):
 * cap radius r and cylinder length l, axis along body x (Sec. 5.3); or
 * RELCP_TORUS with p[3i..] = (R, r, 0): centre-circle (major) radius R >= 0
 * and tube (minor) radius r > 0, symmetry axis along body z (the rings of
 * Sec. 6; SNSD = distance between the centre circles minus both minor
 * radii; overdamped only, not in a monolayer, no learned warm start).
 * rho_or_xi[i] = density (inertial) or drag coefficient xi (overdamped, Eq.
 * ellipsoid_mobility; mobility length L = 2 max semiaxis, l + 2 r or
 * 2 (R + r)).  One packing holds one kind only. */
typedef struct {
    const int32_t *kind;
    const double *p;
    const double *rho_or_xi;
} relcp_shapes;

/* Parameters.  precision: 64 = FP64 LCP iterations; 32 = FP32 products and
 * projection with an FP64 residual, FP64 polish and FP64 acceptance.
 * max_recursions: cap on Alg. 1 augmentations (0 = the plain single-
 * constraint SNSD LCP, first trial always accepted).  lcp_max_iters: cap on
 * projected-gradient iterations per LCP (0 = 100000).  skin: near-contact
 * distance delta_c: pairs with Phi_0 <= skin start in A_0 (the candidate
 * search examines pairs whose bounding spheres and whose support gap along
 * the centre line, a lower bound of Phi, are both within 2 skin, and keeps
 * that list while a bound on the bodies' displacement allows).  warm_start: start
 * of the iteration-0 LCP, RELCP_WS_COLD (zero) or RELCP_WS_PREV (the pair's
 * previous-step multiplier sum, the default); RELCP_WS_LEARNED is selected
 * with relcp_set_warm_start once a model is installed.  stream: a
 * hipStream_t, NULL = the library creates its own. */
typedef struct {
    int32_t dynamics, precision, warm_start, planar;
    int32_t max_recursions, lcp_max_iters, lcp_fixed_iters;
    double skin;
    void *stream;
} relcp_params;

#define RELCP_MAX_RECORDED 65

/* Statistics of one step.  For batched contexts the counts are totals over
 * packings and recursions/iterations are maxima over packings. */
typedef struct {
    int32_t recursions;          /* augmentations before acceptance */
    int32_t lcp_iters_total;     /* projected-gradient iterations over all recursions */
    int32_t n_pairs;             /* pairs of the candidate list: bounding-sphere gap and centre-line
                                    support gap (a lower bound of Phi) <= 2 skin when built */
    int32_t n_contacts_final;    /* rows at acceptance */
    int32_t n_contacts[RELCP_MAX_RECORDED];
    int32_t lcp_iters[RELCP_MAX_RECORDED];   /* iterations per recursion (all precisions) */
    int32_t lcp_iters64[RELCP_MAX_RECORDED]; /* of which FP64 (the FP32 path's polish) */
    double W[RELCP_MAX_RECORDED];        /* gamma_n^T A_n gamma_n (work, non-decreasing) */
    double margin[RELCP_MAX_RECORDED];   /* min |Phi(C_{n+1}) + overlap_tol| over pairs */
    double residual_fp64;        /* scaled natural residual max|min(A_aa g_a, w_a)| of the accepted LCP */
    double residual_lowp;        /* the same in the iteration precision before the FP64 polish */
    double max_overlap;          /* max over pairs of -Phi at the accepted configuration (>= 0) */
    double max_disp;             /* largest surface-point displacement bound of the accepted trial */
    double t_narrow, t_lcp, t_other; /* milliseconds (host clock, stream-synchronised) */
    int32_t rowgraph_entries[RELCP_MAX_RECORDED]; /* off-diagonal entries of A over rows per recursion (row-graph LCP mode; 0 otherwise) */
    int32_t pairs_rebuilt;       /* 1 if the candidate list was rebuilt at this step (it is kept while valid) */
    int32_t n_waits;             /* host waits during the step (polls of results the kernels write to
                                    host-mapped memory, or stream synchronisations) */
    double t_wait;               /* milliseconds of host clock spent in those waits */
    int32_t rowgraph_restarts;   /* row-graph assemblies that overflowed their entry slots and were
                                    re-sized, their solve restarted from the same start */
} relcp_step_stats;

/* Create a context (Sec. 2.1.1 state, Sec. 2.1.2 laws of motion).  Validates
 * the inputs (RELCP_E_INVALID), allocates device buffers (RELCP_E_OOM) and
 * uploads the state once.  *out is set on success only.
 * Environment read here (not in the paper: execution only; every setting
 * gives the same results, bit for bit, and exists to test one path against
 * the other or to force a rare one): RELCP_REDUCE_SPLIT_BLOCKS (see
 * relcp_set_lcp_config); RELCP_RG_SLOTS_PER_ROW, the row graph's first
 * stride of entry slots per row (default 16; a row with more entries raises
 * it and restarts the solve); RELCP_FIRST_LISTS = 0 builds the iteration-0 rows'
 * incidence lists from the rows (atomic slots and a sort) instead of
 * filtering the candidate pairs' lists (1, default); RELCP_FUSED_SELECT = 0
 * compacts the iteration-0 pairs before building their rows instead of
 * selecting and building them in one pass (1, default). */
RELCP_API int relcp_create(const relcp_bodies *bodies, const relcp_shapes *shapes, const relcp_params *params,
                 relcp_ctx **out);
/* Release a context and all of its device buffers (not in the paper:
 * resource handling).  NULL is ignored. */
RELCP_API void relcp_destroy(relcp_ctx *ctx);
/* Message of the last failed call on this context (not in the paper); the
 * string is owned by the context and valid until its next call. */
RELCP_API const char *relcp_last_error(const relcp_ctx *ctx);

/* External wrench F_ext (6n host doubles: force then torque per body, world
 * frame), or NULL for none (Alg. 1 input F_ext). */
RELCP_API int relcp_set_external(relcp_ctx *ctx, const double *f);

/* One time-step: Alg. 1 (overdamped) or Eq. relcp_inertial (inertial) with
 * overlap tolerance eps_NCP = overlap_tol (Eq. gap_stopping_rule) and LCP
 * tolerance lcp_tol on the scaled natural residual.  stats may be NULL. */
RELCP_API int relcp_step(relcp_ctx *ctx, double dt, double overlap_tol, double lcp_tol, relcp_step_stats *stats);

/* State read-back (Alg. 1 output C^{k+1}; inertial runs also U^{k+1}, Eq.
 * relcp_inertial) into caller buffers in the caller's body order (x 3n,
 * q 4n, u 3n, w 3n; any may be NULL).  u, w are the last accepted velocity
 * V_n = U_free + K D gamma.  relcp_get_state takes host buffers and waits;
 * relcp_get_state_device takes device buffers, is ordered on the context's
 * stream and waits for it.  RELCP_E_INVALID for a NULL context. */
RELCP_API int relcp_get_state(const relcp_ctx *ctx, double *x, double *q, double *u, double *w);
RELCP_API int relcp_get_state_device(const relcp_ctx *ctx, double *x, double *q, double *u, double *w);

/* Replace the state C^k (Alg. 1 input; inertial runs also U^k) with the
 * same layout as relcp_create: the same or new body counts (the context is
 * re-sized), shapes and drag or density included.  Validated as at create
 * (RELCP_E_INVALID leaves the old state); clears the warm-start history and
 * the external wrenches.  Used to inject a state (parity checks) and by
 * the colony's division. */
RELCP_API int relcp_set_state(relcp_ctx *ctx, const relcp_bodies *bodies, const relcp_shapes *shapes);

/* Isotropic affine compression x <- s x, box <- s box of all packings, the
 * compression of the compacting suspension between steps (Sec. 5.2).
 * RELCP_E_INVALID for s <= 0 or a box that would become smaller than
 * 2 (R_max + skin).  Ordered on the stream (no wait). */
RELCP_API int relcp_affine_rescale(relcp_ctx *ctx, double s);
/* The same with one factor per packing (host array of n_batch values;
 * waits for the stream). */
RELCP_API int relcp_affine_rescale_packings(relcp_ctx *ctx, const double *s);

/* Colony growth (Sec. 5.3, growing bacterial colony): the cylinder length
 * l of every spherocylinder grows by dl on the device (centres and axes
 * kept; mobility, bounding radii and the candidate list's displacement
 * bound follow at the next step).  A negative dl shrinks them (to undo a
 * growth whose step failed), never below 0.  *n_ready (host, may be NULL:
 * then no wait) = spherocylinders with l >= l_div afterwards.
 * RELCP_E_INVALID for a non-finite dl. */
RELCP_API int relcp_grow(relcp_ctx *ctx, double dl, double l_div, int32_t *n_ready);
/* Colony division (Sec. 5.3): every spherocylinder with cylinder length
 * l >= l_div becomes two cells that are the halves of its total length
 * l + 2r, tip to tip: cylinder length l / 2 - r each, centres
 * x +- (l + 2r) / 4 t (t = the cell's axis, body x); the first keeps the
 * parent's caller index, the second is appended (indices n, n + 1, ... in
 * the order of the parents' indices).  Each daughter is turned about the
 * world z axis by its own angle, jitter[2k] and jitter[2k + 1] for the
 * k-th dividing cell (radians; the caller draws them, e.g. N(0, 0.01^2)).
 * The context is re-sized (as relcp_set_state with new counts: warm-start
 * history and external wrenches cleared).  *n_divided (may be NULL) =
 * dividing cells.  One packing only; RELCP_E_INVALID if n_jitter <
 * 2 * dividing cells or a dividing cell has l < 2r (nothing changed then).
 * Waits for the stream. */
RELCP_API int relcp_divide(relcp_ctx *ctx, double l_div, const double *jitter, int32_t n_jitter,
                           int32_t *n_divided);

/* Rows of the last accepted step, i.e. the contact set A_n at acceptance
 * with the multipliers gamma_n (Alg. 1; Def. ReLCP), in caller buffers of
 * n_contacts_final entries (any may be NULL): body pair (caller's indices,
 * ia < ib), recursion at which the row was generated, multiplier gamma,
 * true Phi where generated, unit normal from ia towards ib (3 each).
 * Waits for the stream; RELCP_E_INVALID for a NULL context. */
RELCP_API int relcp_get_contacts(const relcp_ctx *ctx, int32_t *ia, int32_t *ib, int32_t *recursion_added, double *gamma,
                       double *phi_at_discovery, double *normal);

/* Execution of the LCP loop (not in the paper: how the projected gradient
 * of Eq. cqpp is launched; the same Jacobi-scaled iteration in every
 * mode).  mode 0 = automatic (resident when every packing has at most
 * 256 bodies, or at most 8192 in a context of at least 32 packings; else
 * row graph with one launch per pass), 1 = grid (two passes per iteration
 * over all rows and bodies, through the velocities K D gamma, launched in
 * chunks), 2 = resident (one workgroup per packing runs its whole solve in
 * one launch; block = workgroup size 256, 512 or 1024; lds = stage the
 * packing's velocities in LDS when they fit), 3 = row graph (A = dt D^T K D
 * assembled over rows once per recursion, one pass per iteration, the
 * passes replayed in chunks from an instantiated HIP graph that reads the
 * solve's parameters from device memory; one launch per pass where graphs
 * are unavailable), 4 = row graph with one launch per pass.  In mode 4, a
 * pass over at least RELCP_REDUCE_SPLIT_BLOCKS workgroups of 256 rows
 * (environment, read when a context is created; default 1024) has the last
 * pass's partial sums reduced by a separate one-workgroup launch instead of
 * by each of its workgroups (the same iterates either way). */
RELCP_API int relcp_set_lcp_config(relcp_ctx *ctx, int32_t mode, int32_t block, int32_t lds);

/* Autotuner (not in the paper: launch configuration only): times every LCP configuration (grid; resident x {256, 512,
 * 1024} x {global, LDS}; row graph; row graph per-pass launches) on the
 * rows of the last accepted step, each solve from gamma = 0 (the step's
 * own multipliers already solve that LCP), once untimed and then reps
 * times each; keeps the fastest for this context and writes it to
 * config[3] = {mode, block, lds} and the average milliseconds per
 * configuration to ms[9] in that order (either may be NULL; a
 * configuration that does not fit reports 0).  The multipliers of the last
 * step are restored. */
RELCP_API int relcp_autotune(relcp_ctx *ctx, double dt, double lcp_tol, int32_t reps, int32_t *config, double *ms);

/* Kernel timing with HIP events (not in the paper: measurement; off by
 * default; one event pair per
 * timed launch): each kernel of a class is launched with the pair as the
 * dispatch's own start and end timestamps, so a duration is the kernel's
 * execution alone; a graph launch of row-graph passes (LCP mode 3) is timed
 * by a pair recorded on the stream around it.  Classes: 0 = LCP scatter pass (D gamma -> K), 1 = LCP gather
 * pass (D^T V, projection, step-size reductions), 2 = SNSD narrowphase,
 * 3 = candidate pairs, 4 = trial integration, 5 = resident LCP solve,
 * 6 = warm-start features and MLP inference, 7 = row-graph LCP iteration
 * pass in FP32, 8 = row-graph assembly, 9 = row-graph passes launched after
 * the solve had finished (they return at once; LCP mode 4), 10 = row-graph
 * iteration pass in FP64, 11 = row-graph start pass (either precision).
 * relcp_get_timing fills count[12] (launches) and ms[12] (summed
 * durations) since the last reset, and resets when reset != 0. */
RELCP_API int relcp_set_timing(relcp_ctx *ctx, int32_t enable);
RELCP_API int relcp_get_timing(relcp_ctx *ctx, int32_t *count, double *ms, int32_t reset);

/* ---- learned warm start of the iteration-0 LCP ----
 *
 * The paper leaves the start of the LCP iteration open (the projected
 * gradient solve of Eq. cqpp converges from any nonnegative start); these
 * calls only change the start, never the converged multipliers, the
 * contact sets or the acceptance test.  Per row of A_0 (pairs with
 * Phi_0 <= skin) the library computes 8 features, oriented so that body a
 * has the smaller caller index:
 *   0 Phi_0 / abar (abar: mean of the two bodies' mean semi-extents),
 *   1 dt (D^T U_prev) / abar (previous-step velocity along the row),
 *   2 previous-step multiplier of the pair (the RELCP_WS_PREV start),
 *   3, 4 rows of A_0 at body a, at body b,
 *   5, 6 min / max semi-extent of a, of b,
 *   7 overlap load of the neighbourhood: the sum over the other rows of A_0
 *     at a and at b of max(0, -Phi_0) / abar.
 * Model: z = w3 . GELU(W2 GELU(W1 x + b1) + b2) + b3, GELU exact (erf,
 * evaluated to 5e-7), x = (feature - mean) / std; the start corrects the
 * previous-step multiplier: y0 = max(0, f_2 + scale z) in length units
 * (f_2 = raw feature 2), gamma0 = y0 abar / A_aa.  Weights are a flat fp32
 * vector of RELCP_MLP_NPARAM values in the order W1 (128 x 8, row = hidden
 * unit), b1 (128), W2 (128 x 128), b2 (128), w3 (128), b3 (1); norm holds
 * mean (8), std (8), scale (1).  The matrix products run on the matrix
 * cores with bf16 operands (x, W1, the first hidden layer, W2) and fp32
 * accumulation; the rest is fp32. */
#define RELCP_MLP_NPARAM 17793
#define RELCP_MLP_NORM 17

/* Select the warm start of the iteration-0 LCP (the paper leaves it open,
 * as above): RELCP_WS_COLD, _PREV or _LEARNED (_LEARNED needs an installed
 * model, else RELCP_E_INVALID). */
RELCP_API int relcp_set_warm_start(relcp_ctx *ctx, int32_t mode);
/* Install a model: params (RELCP_MLP_NPARAM host floats), norm (17 host
 * floats, std and scale > 0).  Copied; RELCP_E_INVALID on non-finite input. */
RELCP_API int relcp_set_warmstart_model(relcp_ctx *ctx, const float *params, const float *norm);
/* Record the rows of A_0 (Alg. 1 initialisation) of every accepted step
 * with their features and final multipliers: the training data of the
 * learned start (not in the paper).  Off by default. */
RELCP_API int relcp_enable_contact_log(relcp_ctx *ctx, int32_t on);
/* Copy out the log of the last accepted step into caller device buffers of
 * cap rows (any may be NULL): feat (cap x 8 floats, row-major), gamma (the
 * row's multiplier after the step's last recursion, in the features' length
 * units A_aa gamma / abar: the training target), ia < ib (caller indices).
 * *count = rows (0 when logging is off or the last step failed); returns
 * RELCP_E_CAPACITY, writing nothing, when *count > cap. */
RELCP_API int relcp_log_contacts(relcp_ctx *ctx, float *feat, float *gamma, int32_t *ia, int32_t *ib, int32_t cap,
                                 int32_t *count);

/* Training and inference on device arrays (stream = hipStream_t or NULL).
 * params: RELCP_MLP_NPARAM device floats, 16-byte aligned; feat: rows of 8
 * raw features; idx (may be NULL): row k of the batch is entry idx[k];
 * norm: host array as above.  Asynchronous on the stream. */
/* out[idx[k]] (or out[k]) = max(0, f_2 + scale z) (length units) for the n
 * rows. */
RELCP_API int relcp_mlp_forward(const float *params, const float *norm, int32_t n, const float *feat,
                                const int32_t *idx, float *out, void *stream);
/* Bytes of device workspace that relcp_mlp_grad needs for a batch of n. */
RELCP_API size_t relcp_mlp_workspace_bytes(int32_t n);
/* Gradient of the batch loss mean_k (z_k - (target_k - f_2k) / scale)^2
 * (targets in length units, as logged) into grad (RELCP_MLP_NPARAM device
 * floats) and the loss into *loss (one device float, may be NULL).
 * Deterministic: per-32-row partial gradients in the caller's workspace,
 * summed in a fixed order. */
RELCP_API int relcp_mlp_grad(const float *params, const float *norm, int32_t n, const float *feat, const float *target,
                             const int32_t *idx, float *grad, float *loss, void *work, size_t work_bytes,
                             void *stream);
/* One Adam update (beta1 0.9, beta2 0.999, eps 1e-8; step count t >= 1) of
 * params with moment buffers m, v (RELCP_MLP_NPARAM device floats each). */
RELCP_API int relcp_mlp_adam(float *params, const float *grad, float *m, float *v, int32_t t, float lr, void *stream);

/* ---- stand-alone operations on device arrays (parity tests, tools) ---- */

/* Shared-normal signed distance (Sec. 2.1.4; Lemma uniform interior tangent
 * ball) of m pairs, FP64.  Device SoA inputs for the bodies: x (3 arrays of
 * nb), q (4 arrays of nb), kind, p (3 arrays of nb); pairs pa, pb (m);
 * box[3] host.  Output out (10 arrays of m): Phi, n (3), r_a = p_a - x_a (3),
 * r_b = p_b - x_b (3).  Both bodies of a pair share one kind (ellipsoids,
 * spherocylinders, or tori: the centre-circle distance minus both minor
 * radii, Sec. 6).  Runs on `stream` (hipStream_t, NULL = default) and
 * synchronises before returning. */
RELCP_API int relcp_snsd_device(int32_t nb, const double *x, const double *q, const int32_t *kind, const double *p, int32_t m,
                      const int32_t *pa, const int32_t *pb, const double *box, int32_t planar, double *out,
                      void *stream);

/* Candidate pairs of one packing: all a < b with bounding-sphere gap <= skin
 * (the near-contacting pairs of Alg. 1), sorted by (a, b).  Device SoA x
 * (3 arrays of nb), kind, p (3 arrays).  Writes up to cap pairs to pa, pb
 * (device) and the total count to *m (host). */
RELCP_API int relcp_broadphase_device(int32_t nb, const double *x, const int32_t *kind, const double *p, const double *box,
                            double skin, int32_t cap, int32_t *pa, int32_t *pb, int32_t *m, void *stream);

/* The LCP of one recursion (Eq. relcp; Eq. cqpp), 0 <= g = qv + dt D^T K D
 * gamma _|_ gamma >= 0, solved by the library's Jacobi-scaled BB projected
 * gradient (precision 64 or 32) from the warm start in gamma.  Device arrays:
 * rows ia, ib (m), n, ta = r_a x n, tb = r_b x n (3 arrays of m each), qv (m),
 * body operator kt (nb), Kr (6 arrays of nb: xx, yy, zz, xy, xz, yz), gamma
 * (m, in/out).  mode: LCP execution as in relcp_set_lcp_config, 1 = grid,
 * 3 = row graph with graph-replayed passes, 4 = row graph with one launch
 * per pass (0 = 4).  *iters and *residual (FP64 residual) are host outputs. */
RELCP_API int relcp_lcp_solve_device(int32_t nb, int32_t m, const int32_t *ia, const int32_t *ib, const double *n,
                           const double *ta, const double *tb, const double *qv, const double *kt, const double *Kr,
                           double dt, int32_t planar, int32_t precision, int32_t mode, double tol, int32_t max_iters,
                           double *gamma, int32_t *iters, double *residual, void *stream);

/* ---- building blocks of the step (exposed for testing and reuse) ----
 *
 * Exclusive prefix sum of n device ints, out[i] = in[0] + ... + in[i-1]
 * (out may alias in); *total (a device int, or NULL) receives the sum of
 * all n.  The step uses it for the per-body offsets of the incidence lists,
 * the cell lists of the candidate search and the slice bases of the row
 * graph.  Runs on stream and returns after it has finished; RELCP_E_INVALID
 * for n < 0 or missing arrays. */
RELCP_API int relcp_exclusive_scan_device(const int32_t *in, int32_t *out, int32_t n, int32_t *total,
                                          void *stream);
/* The same prefix sum for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, hosts that forbid
 * hipMalloc): no allocation and no host wait.  Scratch (one int per tile of
 * 2048 items) lives in a file-scope device array of RELCP_NOALLOC_SCAN_MAX /
 * 2048 ints (16 KiB) per GPU, held until the process ends; its address is
 * looked up on a device's first call.  n up to RELCP_NOALLOC_SCAN_MAX
 * (RELCP_E_CAPACITY above it, nothing launched), RELCP_E_INVALID for n < 0
 * or missing arrays.  Asynchronous: the kernels are ordered on stream and
 * the call returns after launching them.  Every call on a GPU shares that
 * GPU's array, so calls that overlap on one GPU (other streams, other host
 * threads) race; calls ordered on one stream do not. */
#define RELCP_NOALLOC_SCAN_MAX 8388608
RELCP_API int relcp_exclusive_scan_device_noalloc(const int32_t *in, int32_t *out, int32_t n, int32_t *total,
                                                  void *stream);
/* Stream compaction: out[j] = index of the j-th nonzero flag among the n
 * device ints flags (increasing order), *count (a device int, or NULL) = the
 * number of them.  The step selects the pairs of A_0 (Phi_0 <= delta_c) and
 * the constraints added by an augmentation (Alg. 1) this way.  out holds up
 * to n ints and must not alias flags.  Runs on stream and returns after it
 * has finished; RELCP_E_INVALID for bad sizes or pointers. */
RELCP_API int relcp_compact_flags_device(const int32_t *flags, int32_t n, int32_t *out, int32_t *count,
                                         void *stream);

#ifdef __cplusplus
}
#endif

#endif /* RELCP_H */
