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
  BDRS_E_NUMERIC = -5      /* non-finite values in the dual state or the certificate  */
} bdrs_status;

/* flags */
#define BDRS_F_REPAIR 1u     /* bdrs_certificate / bdrs_solve also compute <C, Z^> (repaired cost) */

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
 *   omega      Omega >= osc(C) used by the upper bound U (Prop. 3); 1 is valid
 *              whenever the costs lie in [0, 1]
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
 */
typedef struct {
  int64_t k;
  double eps, L, U, gap, rel_gap;
  double L_best, U_best, rel_gap_best;
  int64_t k_L_best, k_U_best;
  double delta, cost_Z, repaired_cost;
  int64_t n_nonfinite;
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
 * iteration has run yet. */
BDRS_API bdrs_status bdrs_certificate(bdrs_solver s, bdrs_cert *out);

/* Runs until (U_best - L_best) / U_best <= tau (tau_relative != 0) or
 * U_best - L_best <= tau (tau_relative == 0), checking after every
 * iteration k with (k + 1) % cert_every == 0 and after the last; the
 * certificate is fused into that iteration's column sweep.  At most
 * max_iters iterations.  *out holds the last certificate.  Returns BDRS_OK
 * when the target is met, BDRS_NOT_CONVERGED at the cap. */
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

/* Kernel timing for measurement.  enable != 0 brackets every LSE sweep
 * kernel this solver launches from then on with a pair of HIP events on the
 * solver's stream and clears the totals; enable == 0 stops recording.
 * Reading synchronises the stream and returns the number of timed sweep
 * launches, their summed duration in milliseconds and the implicit entries
 * (m n per sweep) they processed since the last enable. */
BDRS_API bdrs_status bdrs_profile(bdrs_solver s, int32_t enable);
BDRS_API bdrs_status bdrs_profile_read(bdrs_solver s, int64_t *sweeps, double *ms,
                                       double *entries);

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
