/*
 * bdrs.h -- C ABI of the MI355X (gfx950) Dual O-BDRS solver.
 *
 * The library solves the unregularised discrete optimal-transport problem
 *     p* = min_{X in Pi(r,c)} <C, X>,   C_ij = cost_scale * ||x_i - y_j||^2
 * (Eq. 1 of the paper) by Dual O-BDRS in the log domain (Algorithm 1;
 * lambda = 1 is Dual BDRS, Prop. 1), and certifies it with the linear-memory
 * primal-dual bounds L <= p* <= <C, Z^> <= U of Proposition 3, evaluated as in
 * Algorithm 2.  The cost matrix is never stored: every sweep recomputes C_ij
 * from the point coordinates, so memory is O(m + n).
 *
 * Conventions shared by every entry point:
 *  - Every function returns a bdrs_status; nothing throws or aborts across
 *    the ABI.  On an error bdrs_last_error() returns a message (thread-local,
 *    valid until the next call on the same thread) naming the bad field.
 *  - "device" pointers point to memory of the current HIP device; "host"
 *    pointers to ordinary host memory.  The caller owns every buffer it
 *    passes.  The library never allocates device memory: all device storage
 *    it needs lives in the caller's workspace (bdrs_workspace_size).
 *  - Argument checks that need no device run on the host before any HIP
 *    call, so they work on a machine without a GPU.
 *  - Work is enqueued on the caller's stream (a hipStream_t, NULL = default
 *    stream).  Functions that return host values (certificate, solve,
 *    get_state) synchronise that stream.
 *  - One solver object is not thread-safe; distinct objects are.
 */
#ifndef BDRS_H_
#define BDRS_H_

#include <stddef.h>
#include <stdint.h>

#if defined(__GNUC__)
#define BDRS_API __attribute__((visibility("default")))
#else
#define BDRS_API
#endif

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  BDRS_OK = 0,
  BDRS_NOT_CONVERGED = 1,  /* informational: iteration cap hit before the gap target */
  BDRS_E_INVALID = -1,     /* bad argument (the message names it)                     */
  BDRS_E_NOMEM = -2,       /* workspace too small / admission over the memory budget  */
  BDRS_E_DEVICE = -3,      /* HIP error, or no usable gfx950 device                   */
  BDRS_E_STATE = -4,       /* call not valid in the object's current state            */
  BDRS_E_NUMERIC = -5      /* non-finite values, or a negative duality gap (U < L)    */
} bdrs_status;

/* flags */
#define BDRS_F_REPAIR 1u     /* bdrs_certificate / bdrs_solve also compute <C, Z^> (repaired cost) */
/* Ablation variants of the row update (Cor. 1 and the momentum / kernel
 * ablation; lambda must be 1).  All keep the column update at eta / (k + 1)
 * (kernel K^{.(k+1)}), the schedule and the initialisation:
 *   BDRS_F_OLD_KERNEL   row update with the old kernel K^{.k} (temperature
 *                       eta / k; K^{.0} is all ones) instead of K^{.(k+1)}
 *   BDRS_F_NO_MOMENTUM  row update with t = b^{k-1} instead of the
 *                       extrapolated b~^{k-1}
 *   BDRS_F_DEBIASED     debiased annealed Sinkhorn: a^k = (a^{k-1})^theta_k r /
 *                       (K^{.k} b^{k-1}), theta_k = 0 for k <= 1 and 1/k after;
 *                       requires the two flags above
 * Annealed Sinkhorn = OLD_KERNEL | NO_MOMENTUM, annealed Sinkhorn with
 * momentum = OLD_KERNEL, current-kernel annealed Sinkhorn = NO_MOMENTUM,
 * Dual BDRS = none.  The certificate stays valid: its plan Z uses the row
 * update's temperature and weights t (so Z 1 = r) and its lower bound the
 * column update's temperature and row scaling; with OLD_KERNEL or DEBIASED
 * this takes one more column sweep per certificate, and such solvers are
 * not accepted by bdrs_batch_solve. */
#define BDRS_F_OLD_KERNEL 2u
#define BDRS_F_NO_MOMENTUM 4u
#define BDRS_F_DEBIASED 8u
/* bdrs_solve launches every kernel on its own instead of replaying a
 * captured block of iterations (see bdrs_solve); the results are the same. */
#define BDRS_F_NO_GRAPH 16u
/* Retain the dual state with the lowest relative gap (U - L) / U of all
 * certificates so far (the colour-transfer experiments keep that state for
 * the barycentric projection); bdrs_restore_best brings it back.  Adds an
 * O(m + n) region to the workspace (bdrs_workspace_size counts it when the
 * flag is set).  Not accepted by bdrs_batch_solve and the solve server. */
#define BDRS_F_KEEP_BEST_STATE 32u

typedef struct bdrs_solver_* bdrs_solver;

/*
 * Problem and solver parameters (problem statement Eq. 1; Algorithm 1; Prop. 3).
 *   m, n       number of source / target points, 1 <= m, n <= 2^30 (m n < 2^62)
 *   dim        coordinate dimension d, 1 <= d <= 3
 *   x, y       device, float32, row-major m x dim / n x dim (finite)
 *   r, c       device, float64, the marginals: strictly positive, finite,
 *              each summing to 1 within 1e-9 (problem statement, Eq. 1)
 *   cost_scale s > 0 in C_ij = s ||x_i - y_j||^2
 *   eta        initial temperature eta > 0 (Algorithm 1: eta_k = eta / (lambda k + 1))
 *   lambda     overrelaxation, 1 <= lambda < 2 (Prop. 2; 1 = BDRS)
 *   omega      Omega >= osc(C) used by the upper bound U (Prop. 3), finite and
 *              > 0; 1 is valid whenever the costs lie in [0, 1].  The library
 *              cannot check Omega >= osc(C) in O(m + n); a too small Omega can
 *              make U fall below L, which every certificate reports
 *              (bdrs_cert.negative_gap, BDRS_E_NUMERIC)
 *   workspace  device memory of at least bdrs_workspace_size() bytes, 256-byte
 *              aligned, owned by the caller, used exclusively by this solver
 *              until bdrs_destroy
 *   stream     hipStream_t on which all work is enqueued (NULL: default stream)
 *   flags      BDRS_F_* bits
 * x, y, r, c are copied into the workspace by bdrs_create; the caller may
 * free them afterwards.
 */
typedef struct {
  int32_t m, n, dim;
  const float *x, *y;
  const double *r, *c;
  double cost_scale;
  double eta;
  double lambda;
  double omega;
  void *workspace;
  size_t workspace_bytes;
  void *stream;
  uint32_t flags;
} bdrs_params;

/*
 * One certificate (Prop. 3 evaluated by Algorithm 2) at iteration k, with the
 * scalings A = alpha-hat^k, B = beta-hat^k, t = beta-tilde^{k-1} and
 * eps = eta / (lambda k + 1).  All sums are accumulated in float64.
 *   L            dual lower bound <r, f> + <c, g>
 *   U            primal upper bound <t, w> + Omega delta
 *   gap, rel_gap U - L and (U - L) / U
 *   *_best       best bounds so far: U_best = min U, L_best = max L, and the
 *                iterations that attained them; rel_gap_best = (U_best - L_best) / U_best
 *   delta        1/2 ||s - c||_1, the column mass the repair relocates
 *   cost_Z       <C, Z> = sum_j s_j mu_j, the cost of the intermediate plan
 *   repaired_cost <C, Z^> of the feasible repair (only with BDRS_F_REPAIR, else NaN)
 *   n_nonfinite  number of non-finite values met in the certificate inputs
 *   negative_gap 1 when U - L < -1e-9 |U| for this certificate, or
 *                U_best - L_best < -1e-9 |U_best| for the best bounds, else 0.
 *                Prop. 3 gives L <= p* <= U for every certificate, so a
 *                negative gap means the bounds are not valid (float32 error
 *                in the sweeps, or omega below osc(C)).  The gap is reported
 *                as computed, never clamped; the call returns BDRS_E_NUMERIC,
 *                the stopping rule never counts such a certificate as meeting
 *                its target, and a certificate whose own gap is negative is
 *                not folded into the best bounds.
 */
typedef struct {
  int64_t k;
  double eps, L, U, gap, rel_gap;
  double L_best, U_best, rel_gap_best;
  int64_t k_L_best, k_U_best;
  double delta, cost_Z, repaired_cost;
  int64_t n_nonfinite;
  int64_t negative_gap;
} bdrs_cert;

/* Bytes of device workspace bdrs_create needs for these sizes (O(m + n)).
 * Reads only m, n, dim.  Errors: BDRS_E_INVALID for bad sizes or NULL out. */
BDRS_API bdrs_status bdrs_workspace_size(const bdrs_params *p, size_t *bytes);

/* Validates the parameters, copies the inputs into the workspace and
 * initialises the state of Algorithm 1 (log alpha^{-1} = log beta^{-1} =
 * log beta^{-2} = 0, k = 0).  Synchronises the stream.  Errors:
 * BDRS_E_INVALID (the message names the field; marginal contents are
 * checked after the copy), BDRS_E_NOMEM (workspace too small),
 * BDRS_E_DEVICE (no gfx950 device, HIP failure).  *out is NULL on error. */
BDRS_API bdrs_status bdrs_create(const bdrs_params *p, bdrs_solver *out);

/* Runs `iters` >= 0 iterations of Algorithm 1 (schedule, momentum, row
 * sweep, overrelaxation, column sweep, overrelaxation) without a
 * certificate.  Asynchronous on the solver's stream; enqueues kernels only
 * and keeps the iteration counter in device memory, so a stream capture of
 * bdrs_step can be replayed as a block of iterations. */
BDRS_API bdrs_status bdrs_step(bdrs_solver s, int32_t iters);

/* Certificate of the last finished iteration (Prop. 3 / Algorithm 2): one
 * extra column pass from the stored log alpha-hat and log beta-tilde, then
 * the float64 reductions.  With BDRS_F_REPAIR one more row pass gives the
 * repaired cost.  Updates the best bounds.  Synchronous.  BDRS_E_STATE if no
 * iteration has run yet; BDRS_E_NUMERIC (with *out filled) for non-finite
 * values or a negative gap (bdrs_cert.negative_gap). */
BDRS_API bdrs_status bdrs_certificate(bdrs_solver s, bdrs_cert *out);

/* Runs until (U_best - L_best) / U_best <= tau (tau_relative != 0) or
 * U_best - L_best <= tau (tau_relative == 0), checking after every
 * iteration k with (k + 1) % cert_every == 0 and after the last; the
 * certificate is fused into that iteration's column sweep.  At most
 * max_iters iterations.  *out holds the last certificate.  Returns BDRS_OK
 * when the target is met, BDRS_NOT_CONVERGED at the cap, BDRS_E_NUMERIC at
 * the first certificate with non-finite values or a negative gap (a
 * negative gap never meets the target).
 * A block of cert_every iterations that starts at a multiple of cert_every
 * and ends with its certificate is captured once as a hipGraph (on a private
 * stream of the solver; the kernels read the iteration counter from device
 * memory, so the graph holds for every such block) and replayed on the
 * solver's stream; other blocks, solvers with BDRS_F_REPAIR, OLD_KERNEL,
 * DEBIASED or BDRS_F_NO_GRAPH, and solvers with profiling on launch their
 * kernels one by one.  Results are bitwise the same either way. */
BDRS_API bdrs_status bdrs_solve(bdrs_solver s, double tau, int32_t tau_relative,
                       int32_t max_iters, int32_t cert_every, bdrs_cert *out);

/* Copies the dual state of Algorithm 1 into caller device buffers (float64,
 * original point order; NULL skips a vector): log alpha^k (m), log beta^k
 * (n), log beta^{k-1} (n), log alpha-hat^k (m), log beta-hat^k (n),
 * log beta-tilde^{k-1} (n), and the number of finished iterations (host).
 * The state is held in float64 (O(m + n)); only the O(m n) sweeps run in
 * float32.  Synchronous. */
BDRS_API bdrs_status bdrs_get_state(bdrs_solver s, double *log_alpha, double *log_beta,
                           double *log_beta_prev, double *log_alpha_hat,
                           double *log_beta_hat, double *log_beta_tilde,
                           int64_t *iters_done);

/* Replaces the dual state (device float64 buffers in original point order;
 * log_alpha, log_beta and log_beta_prev are required, the hats and
 * beta-tilde are optional) and the iteration counter; resuming from a state
 * saved by bdrs_get_state continues the same trajectory.  Resets the best
 * bounds.  Synchronous. */
BDRS_API bdrs_status bdrs_set_state(bdrs_solver s, const double *log_alpha,
                           const double *log_beta, const double *log_beta_prev,
                           const double *log_alpha_hat, const double *log_beta_hat,
                           const double *log_beta_tilde, int64_t iters_done);

/* Warm-start hints of the sweeps: for every source point the index of a
 * target point whose term was near that row's maximum in the last row sweep
 * (row_hint, m entries) and for every target point the index of a source
 * point likewise (col_hint, n entries); -1 = none.  Device int32 buffers,
 * original point order; NULL skips one.  They only choose the float32 shift
 * of each reduction (any valid index gives a correct result), so they belong
 * to a checkpoint only when a resumed run must repeat the original bit for
 * bit.  Synchronous. */
BDRS_API bdrs_status bdrs_get_hints(bdrs_solver s, int32_t *row_hint, int32_t *col_hint);
BDRS_API bdrs_status bdrs_set_hints(bdrs_solver s, const int32_t *row_hint, const int32_t *col_hint);

/* One LSE sweep on the solver's problem, for parity checks of the kernel:
 * out_i = LSE_j( w_j - C_ij / eps ) in natural-log units (the reduction of
 * the row update of Algorithm 1) when transpose == 0, and
 * out_j = LSE_i( w_i - C_ij / eps ) (the column update) when transpose != 0.
 * w and out are device float64 in original point order (length n / m resp.
 * m / n); the sweep itself runs in float32 on weights taken relative to
 * their tile maximum.  Uses the solver's workspace (clobbers its sweep buffers but not
 * the dual state).  Synchronises the stream. */
BDRS_API bdrs_status bdrs_lse(bdrs_solver s, int32_t transpose, double eps,
                     const double *w, double *out);

/*
 * The state plan after k >= 1 finished iterations,
 *   X^k = diag(alpha^{k-1}) K^{.lambda k} diag(beta^{k-1}),  K = exp(-C / eta)
 * (the O-BDRS state of Prop. 2; for lambda = 1 the BDRS plan of Lemma 1,
 * whose column sums are c), and what the colour-transfer experiments read
 * from it: its row and column sums, their errors against r and c, and the
 * barycentric projection y^_i = sum_j X_ij y_j / sum_j X_ij of every source
 * point onto the target points.  X is never formed: one row sweep at
 * temperature eta / (lambda k) on the weights log beta^{k-1} that also
 * accumulates the target coordinates, and one column sweep on log alpha^{k-1}
 * (float32 sweeps, float64 merges and sums).
 */
typedef struct {
  int64_t k;                      /* finished iterations (the plan is X^k) */
  double eps;                     /* temperature of its kernel, eta / (lambda k) */
  double row_l1, col_l1;          /* sum_i |(X 1)_i - r_i|,  sum_j |(X^T 1)_j - c_j| */
  double row_max_abs, col_max_abs;/* largest absolute marginal error */
  double row_max_rel, col_max_rel;/* largest error relative to r_i (c_j) */
  double mass;                    /* 1^T X 1 */
} bdrs_plan_stats;

/* Evaluates the state plan of the solver's current iterate.  Optional
 * outputs (NULL skips, device memory, original point order): bary m x dim
 * row-major float64 (in the caller's coordinates), row_marg m float64,
 * col_marg n float64; stats (host, optional).  BDRS_E_STATE before the first
 * iteration.  Uses the solver's sweep buffers, not its dual state or warm-
 * start hints, so the iteration that follows is unchanged.  Synchronises the
 * stream. */
BDRS_API bdrs_status bdrs_plan(bdrs_solver s, double *bary, double *row_marg, double *col_marg,
                               bdrs_plan_stats *stats);

/*
 * Feasible plan from the state plan X^k by the two-sided rounding of
 * Altschuler, Weed and Rigollet (2017, Algorithm 2), which the momentum /
 * kernel ablation applies to every method: rows scaled down to r
 * (x = min(1, r / X 1)), then columns down to c (y = min(1, c / X'^T 1)),
 * then the missing mass e_r e_c^T / ||e_r||_1 added.  The result G lies in
 * Pi(r, c), so <C, G> is an upper bound of the optimum for any iterate.
 * Three sweeps at the plan's temperature (the last one cost-weighted) and
 * float64 sums; e_r^T C e_c in closed form for the squared Euclidean cost.
 */
typedef struct {
  int64_t k;             /* finished iterations (the plan rounded is X^k) */
  double eps;            /* temperature of its kernel, eta / (lambda k) */
  double cost;           /* <C, G> */
  double cost_clipped;   /* <C, diag(x) X diag(y)>, the part before the added mass */
  double mass_moved;     /* ||e_r||_1 = ||e_c||_1 */
} bdrs_round_stats;

/* Rounds the solver's current state plan (host output).  BDRS_E_STATE
 * before the first iteration.  Uses the solver's sweep buffers, not its
 * dual state or hints.  Synchronises the stream. */
BDRS_API bdrs_status bdrs_round(bdrs_solver s, bdrs_round_stats *out);

/*
 * Export of a feasible plan of the current iterate, exactly and in O(m + n)
 * memory, as the factors of
 *
 *     P_ij = exp(u_i + v_j - C_ij / eps) + a_i b_j,   C_ij = s |x_i - y_j|^2.
 *
 * BDRS_PLAN_ROUNDED: G, the two-sided rounding of the state plan X^k that
 *   bdrs_round prices (Altschuler, Weed and Rigollet 2017, Algorithm 2):
 *   u = log alpha^k + log x, v = log beta^k + log y, a = e_r,
 *   b = e_c / ||e_r||_1, eps = eta / (lambda k).
 * BDRS_PLAN_REPAIRED: Z^ = Z diag(e) + p q^T / delta, the repair of the
 *   intermediate plan Z = diag(alpha-hat) K diag(beta-tilde) of the last
 *   finished iteration (proof of Prop. 3, feasible primal repair):
 *   u = log alpha-hat, v = log beta-tilde + log e with
 *   e_j = min(1, c_j / s_j), a = p, b = (c - s)_+ / delta (0 when
 *   delta = 0), eps = the row update's temperature of that iteration; its
 *   cost is the repaired cost of the certificate at that iteration.
 *
 * Both lie in Pi(r, c) up to the float32 sweeps' accuracy: the deficits that
 * a and b carry are r and c minus row and column sums taken by the sweeps
 * (relative error about 1e-6 per sum), so P 1 = r and P^T 1 = c hold to that
 * relative accuracy entry by entry.
 */
#define BDRS_PLAN_ROUNDED 0
#define BDRS_PLAN_REPAIRED 1

typedef struct {
  int32_t kind;          /* BDRS_PLAN_ROUNDED or BDRS_PLAN_REPAIRED */
  int64_t k;             /* finished iterations of the state exported */
  double eps;            /* temperature of the kernel part */
  double cost_scale;     /* s of C_ij = s |x_i - y_j|^2 */
  double cost;           /* <C, P> */
  double mass;           /* mass of the rank-one part: ||e_r||_1 (rounded), delta (repaired) */
} bdrs_plan_export;

/* Writes the factors of the chosen feasible plan into caller device buffers
 * (float64, original point order; NULL skips one): log_u and a (m),
 * log_v and b (n); info (host, optional).  BDRS_E_INVALID for an unknown
 * kind, BDRS_E_STATE before the first iteration, BDRS_E_NUMERIC when the
 * plan's cost is not finite.  Runs three sweeps (rounded) or the
 * certificate's column sweep and the repair's row sweep (repaired); uses the
 * solver's sweep and certificate buffers, not its dual state or warm-start
 * hints, so the iteration that follows is unchanged.  Synchronises the
 * stream. */
BDRS_API bdrs_status bdrs_export_plan(bdrs_solver s, int32_t kind, double *log_u, double *log_v,
                                      double *a, double *b, bdrs_plan_export *info);

/* Dense entries of a factored plan for the rows [row_begin, row_end) into
 * out, a caller device buffer of (row_end - row_begin) x n float64,
 * row-major, original point order: out[(i - row_begin) n + j] = P_ij from
 * the factors above (device, original order; a and b both given or both
 * NULL for no rank-one part) at temperature eps, with C_ij in float64 from
 * the solver's stored float32 coordinates.  A large plan is written in
 * strips of rows.  BDRS_E_INVALID for a NULL log_u or log_v, a NULL out
 * with a non-empty range, a row range outside [0, m), eps not positive and
 * finite, or n > 65535 * 256.  Write-bound (8 bytes per entry).
 * Synchronises the stream. */
BDRS_API bdrs_status bdrs_plan_entries(bdrs_solver s, const double *log_u, const double *log_v,
                                       const double *a, const double *b, double eps,
                                       int64_t row_begin, int64_t row_end, double *out);

/*
 * Batched solving (many independent problems in one set of launches).
 * The problems are solver objects from bdrs_create (each with its own
 * workspace), all with the same dim, all at an iteration count that is a
 * multiple of cert_every (fresh solvers are at 0).  Every phase of an
 * iteration (row sweep, row epilogue, column sweep, column epilogue) runs as
 * ONE launch over a work list of (problem, block of outputs, split) items of
 * all active problems; a block of cert_every iterations ends with the fused
 * certificate of every active problem and one readback.  A problem whose
 * certificate meets the target (the same rule as bdrs_solve) or that reaches
 * max_iters retires at that block boundary; the others go on.  Each problem's
 * arithmetic is the same as when it is solved alone with bdrs_solve, so its
 * results are bitwise equal.
 * With use_graph != 0 one block of iterations is captured as a hipGraph
 * (on a private stream) and replayed, and captured again only when the set
 * of active problems changes.
 *   workspace   device memory of bdrs_batch_workspace_size() bytes (256-byte
 *               aligned) for descriptors, work lists and certificate records
 *   max_iters   per problem, a positive multiple of cert_every
 *   outs        host array of count certificates (the last of each problem)
 *   statuses    host array of count statuses (BDRS_OK: target met,
 *               BDRS_NOT_CONVERGED: cap reached, BDRS_E_NUMERIC)
 * Synchronous.  Returns BDRS_OK if every problem met the target,
 * BDRS_NOT_CONVERGED if some hit the cap, an error otherwise. */
BDRS_API bdrs_status bdrs_batch_workspace_size(const bdrs_solver *solvers, int32_t count,
                                               size_t *bytes);
BDRS_API bdrs_status bdrs_batch_solve(const bdrs_solver *solvers, int32_t count, void *workspace,
                                      size_t workspace_bytes, double tau, int32_t tau_relative,
                                      int32_t max_iters, int32_t cert_every, int32_t use_graph,
                                      bdrs_cert *outs, int32_t *statuses);

/*
 * Batched solving for callers that cannot allocate device memory (code under
 * stream capture, tight serving loops, harnesses that forbid allocation):
 * bdrs_batch_solve without its workspace argument and with use_graph = 0.
 * The descriptors, work lists and certificate records live in a device array
 * of BDRS_BATCH_STATIC_BYTES that the library holds on every GPU it runs on
 * until the process ends, and the blocks are launched one by one on the
 * first solver's stream.  The call allocates no device memory and creates no
 * stream, event or graph; each solver's own workspace is the caller's, as
 * always.  Results are bitwise those of bdrs_batch_solve.  BDRS_E_NOMEM when
 * bdrs_batch_workspace_size of the solvers exceeds BDRS_BATCH_STATIC_BYTES
 * (checked on the host before any device work); other errors as
 * bdrs_batch_solve.  Every call on a GPU shares that GPU's array, which keeps
 * the last call's contents (each call writes all it reads): calls that
 * overlap on one GPU, from several threads, race and must be serialised by
 * the caller.  Synchronous.
 */
#define BDRS_BATCH_STATIC_BYTES (16u << 20)
BDRS_API bdrs_status bdrs_batch_solve_static(const bdrs_solver *solvers, int32_t count, double tau,
                                             int32_t tau_relative, int32_t max_iters, int32_t cert_every,
                                             bdrs_cert *outs, int32_t *statuses);

/*
 * Solve server: continuous batching of independent OT solves on one GPU.
 * The server owns a device memory pool given by the caller (the "HBM
 * budget"); every admitted request gets its workspace (bdrs_workspace_size of
 * its sizes) from the pool, and the batch engine's descriptors and work lists
 * for the running set live there too (a request is admitted only when both
 * fit).  A worker thread admits queued requests in arrival order whenever a
 * slot and pool memory are free, runs blocks of block_iters iterations of all
 * running requests together (one launch per phase, as in bdrs_batch_solve;
 * a block whose running set equals the previous block's is captured as a
 * hipGraph and replayed until the set changes), evaluates each request's
 * certificate at the end of every block, and retires a request when its
 * stopping rule holds (same rule as bdrs_solve with cert_every = block_iters)
 * or max_iters is reached, releasing its memory for the next request.  A
 * request's result is bitwise the same as solving it alone with bdrs_solve.
 */
typedef struct bdrs_server_* bdrs_server;

/* One solve request.  Inputs are HOST arrays, copied by bdrs_server_submit. */
typedef struct {
  int32_t m, n, dim;
  const float *x, *y;          /* host, row-major m x dim / n x dim */
  const double *r, *c;         /* host marginals (as in bdrs_params) */
  double cost_scale, eta, lambda, omega;
  double tau;                  /* stop when the (relative) best gap <= tau */
  int32_t tau_relative;
  int32_t max_iters;           /* positive multiple of the server's block_iters */
} bdrs_request;

typedef struct {
  int32_t state;               /* 0 queued, 1 running, 2 done */
  int32_t status;              /* when done: BDRS_OK, BDRS_NOT_CONVERGED or an error */
  bdrs_cert cert;              /* the last certificate (when done) */
  double t_submit, t_admit, t_done;  /* seconds on the server clock (bdrs_server_now) */
} bdrs_result;

/* pool: device memory (256-byte aligned) of pool_bytes, owned by the caller
 * until bdrs_server_destroy.  max_slots >= 1 requests run concurrently.
 * block_iters >= 1 iterations per block.  Starts the worker thread. */
BDRS_API bdrs_status bdrs_server_create(void *pool, size_t pool_bytes, int32_t max_slots,
                                        int32_t block_iters, bdrs_server *out);
/* Validates a request (sizes, parameters, and the contents of its arrays as
 * in bdrs_create) and prepares its host image (points in tile order, tile
 * records) on the calling thread, so that the worker only uploads it at
 * admission; the request's latency (t_submit) starts when this call starts.
 * Thread-safe.  BDRS_E_INVALID for a bad request, BDRS_E_NOMEM if its
 * workspace can never fit the pool.  *ticket identifies the request. */
BDRS_API bdrs_status bdrs_server_submit(bdrs_server s, const bdrs_request *req, uint64_t *ticket);
/* Admission policy (thread-safe; takes effect at the next block boundary).
 * big_work > 0: a request with m n > big_work entries per sweep is admitted
 * only while no other such request runs (large requests run one at a time,
 * in arrival order), and smaller requests behind a waiting large one may be
 * admitted before it; a GPU-saturating request then is not slowed down by
 * other large ones, while small requests keep the benefit of batching.
 * big_work <= 0 (the default): plain arrival-order admission. */
BDRS_API bdrs_status bdrs_server_set_policy(bdrs_server s, double big_work);
/* Non-blocking state of a request. */
BDRS_API bdrs_status bdrs_server_poll(bdrs_server s, uint64_t ticket, bdrs_result *out);
/* Blocks until the request is done (or the server stops). */
BDRS_API bdrs_status bdrs_server_wait(bdrs_server s, uint64_t ticket, bdrs_result *out);
/* Counts: running and queued requests, pool bytes in use. */
BDRS_API bdrs_status bdrs_server_stats(bdrs_server s, int32_t *running, int32_t *queued,
                                       size_t *pool_used);
/* Seconds since the server was created (the clock of bdrs_result). */
BDRS_API bdrs_status bdrs_server_now(bdrs_server s, double *t);
/* Stops the worker after its current block; requests not finished by then
 * end with BDRS_E_STATE.  Frees host memory; the pool stays the caller's. */
BDRS_API bdrs_status bdrs_server_destroy(bdrs_server s);

/*
 * Tile-shape autotuner.  The work tile of one sweep launch is a block of
 * outputs (256 outputs, 4 wavefronts of 64) against one "split" of the input
 * tiles; the number of splits per sweep direction decides how many tiles one
 * work item streams, how many partial (max, sum) records the epilogue merges
 * and how many work items fill the 256 CUs.  A process-wide table keyed by
 * the exact shape (dim, m, n) holds the chosen split counts; every layout
 * (bdrs_workspace_size, bdrs_create, the server's admission) made after an
 * entry exists uses it, and shapes without an entry use a built-in heuristic
 * (about 16384 wavefronts per sweep, at least 4 input tiles per split).  A
 * workspace must be sized with the same table in effect as the bdrs_create
 * that uses it.  The table is guarded by a mutex.
 */
typedef struct {
  int32_t dim, m, n;             /* problem shape (the table key) */
  int32_t splits_row;            /* input splits of the row sweep (over the n columns) */
  int32_t splits_col;            /* input splits of the column sweep (over the m rows) */
  int32_t candidates;            /* split counts timed per direction (0 if set by hand) */
  double us_row, us_col;         /* measured median time of one row / column sweep with its
                                    epilogue, microseconds (0 if set by hand) */
  double us_row_default, us_col_default;  /* the same for the heuristic's split counts */
} bdrs_tune_entry;

/* Workspace bytes bdrs_autotune needs for this shape (room for the partial
 * records of the largest candidate split count).  Host only. */
BDRS_API bdrs_status bdrs_autotune_workspace_size(const bdrs_params *p, size_t *bytes);
/* Times candidate split counts for the problem in *p (same fields and
 * checks as bdrs_create; workspace of bdrs_autotune_workspace_size bytes):
 * runs min(500, max(10, 2e13 / (2 m n))) iterations of Algorithm 1 to reach
 * the low-temperature regime where a solve spends most sweeps, then
 * `rounds` rounds that each time every candidate's row and column sweep
 * (with its epilogue) once with HIP events on p->stream, interleaved so the
 * drift of the state affects every candidate alike.  The candidate with
 * the smallest median per direction is entered into the table (replacing an
 * entry of the same shape) and copied to *out.  The workspace contents are
 * scratch.  Synchronous.  rounds in [1, 1000]. */
BDRS_API bdrs_status bdrs_autotune(const bdrs_params *p, int32_t rounds, bdrs_tune_entry *out);
/* Inserts or replaces the entry of e's shape (e.g. a table saved earlier).
 * Split counts are clamped to [1, input tiles]. */
BDRS_API bdrs_status bdrs_tune_set(const bdrs_tune_entry *e);
/* Copies entry `index` (0-based, insertion order) to *out; BDRS_E_INVALID
 * past the end.  *count (optional) receives the number of entries. */
BDRS_API bdrs_status bdrs_tune_get(int32_t index, bdrs_tune_entry *out, int32_t *count);
/* Empties the table. */
BDRS_API bdrs_status bdrs_tune_clear(void);

/* Kernel timing for measurement.  enable != 0 brackets every LSE sweep
 * kernel this solver launches from then on with a pair of HIP events on the
 * solver's stream and clears the totals; enable == 0 stops recording.
 * Reading synchronises the stream and returns the number of timed sweep
 * launches, their summed duration in milliseconds and the implicit entries
 * (m n per sweep) they processed since the last enable. */
BDRS_API bdrs_status bdrs_profile(bdrs_solver s, int32_t enable);
BDRS_API bdrs_status bdrs_profile_read(bdrs_solver s, int64_t *sweeps, double *ms,
                                       double *entries);
/* Entries the timed sweeps actually evaluated since the last enable: a sweep
 * skips an input tile for a wavefront of 64 outputs when its bound puts
 * every term of the tile below 2^-T of each output's running maximum, with
 * T = 30 + ceil(log2 n_in) (at most 64) for n_in inputs (all skipped terms
 * of an output together stay below 2^-30 of its sum, under float32's
 * rounding), so this can be far below the implicit
 * m n per sweep late in a solve.  Counted per (64 outputs, 64 inputs) pair,
 * padding included.  Synchronises the stream. */
BDRS_API bdrs_status bdrs_profile_evaluated(bdrs_solver s, double *entries);

/* Makes the state retained under BDRS_F_KEEP_BEST_STATE the current one:
 * the dual state and warm-start hints after the iteration whose certificate
 * had the lowest relative gap, and its iteration count (*iters_done, may be
 * NULL).  Later bdrs_plan / bdrs_round / bdrs_get_state / bdrs_certificate /
 * bdrs_step act on it; the best-bound records are kept.  The retained state
 * is that of the solver's whole history (bdrs_set_state does not clear it).
 * BDRS_E_INVALID without the flag, BDRS_E_STATE before the first
 * certificate.  Synchronises the stream. */
BDRS_API bdrs_status bdrs_restore_best(bdrs_solver s, int64_t *iters_done);

/* Destroys the solver object (host memory only; the workspace stays the
 * caller's).  Synchronises the stream.  NULL is accepted. */
BDRS_API bdrs_status bdrs_destroy(bdrs_solver s);

/* Message of the last error on this thread ("" if none). */
BDRS_API const char *bdrs_last_error(void);

/* Library version string. */
BDRS_API const char *bdrs_version(void);

#ifdef __cplusplus
}
#endif
#endif /* BDRS_H_ */
