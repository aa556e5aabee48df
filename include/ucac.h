/*
 * ucac.h -- C-ABI of the MI355X (gfx950) library that runs the inner iteration of
 * the two-level component-based ADMM for unit commitment with AC optimal power
 * flow (UC-ACOPF) of Zhang, Kim & Kim, "On Solving Unit Commitment with
 * Alternating Current Optimal Power Flow on GPU".
 *
 * One inner iteration (Sec. III-A, steps step:uc .. step:y, in that order) is:
 *   1. one dynamic program per generator for the commitments (Sec. III-B,
 *      Alg. dp_algo);
 *   2. one closed-form update per (generator, period) and one trust-region
 *      Newton solve per (line, period) for the ACOPF variables (step:opf);
 *   3. the relaxed commitment duplicates in [0,1] (step:uc_bar) and one
 *      balance-constrained projection per (bus, period) (step:opf_bar),
 *      a Jacobi pair (both read the other's previous value);
 *   4. the artificial variable z and the multiplier y of every coupling row
 *      (step:z, step:y), the residuals, and the outer update of lambda and
 *      beta (step:outer, tau = 6, theta = 0.8) when the inner loop ends.
 *
 * Every function returns UCAC_OK (0) or a status below.  A negative status
 * leaves the handle's iterate as it was before the call.  All pointers to
 * arrays are HOST pointers unless stated; the library copies what it needs and
 * never keeps a caller pointer.  A handle is not thread-safe; different handles
 * are independent.  Floating point is IEEE FP64 throughout.
 */
#ifndef UCAC_H
#define UCAC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  UCAC_OK = 0,
  UCAC_NOT_CONVERGED = 1,  /* ucac_solve hit max_iters before the tolerance */
  UCAC_E_INVAL = -1,       /* bad argument or network data (see ucac_last_error) */
  UCAC_E_NOMEM = -2,       /* device or host allocation failed */
  UCAC_E_DEVICE = -3,      /* a HIP runtime call failed */
  UCAC_E_STATE = -4,       /* state buffer of the wrong size or content */
  UCAC_E_NUMERIC = -5      /* a NaN/Inf appeared in the iterate */
};

typedef struct ucac_handle ucac_handle;

/* Network and unit data of one instance (Sec. II: eq:uc-acopf, eq:acopf, set:UC,
 * eq:coupling).  Per-unit quantities on base_mva.  Arrays indexed [t][k] are
 * row-major with T rows.  All indices are 0-based.  Read only during create. */
typedef struct {
  int32_t n_bus, n_line, n_gen, T, ref_bus;
  double base_mva;
  const int32_t *line_from, *line_to;        /* [n_line] end buses, from != to */
  const double *line_r, *line_x, *line_b;    /* [n_line] series r, x and total charging b (pi model) */
  const double *line_rate;                   /* [n_line] MVA limit r-bar at both ends (uc_acopf_ij/ji_limit) */
  const double *bus_gs, *bus_bs;             /* [n_bus] shunt G^s, B^s (balance equations) */
  const double *bus_vmin, *bus_vmax;         /* [n_bus] voltage magnitude bounds (uc_acopf_w_bound) */
  const double *load_p, *load_q;             /* [T][n_bus] demand P_{t,i}, Q_{t,i} */
  const int32_t *gen_bus;                    /* [n_gen] */
  const double *gen_pmin, *gen_pmax;         /* P-lo, P-bar of eq:coupling; ACOPF box is [0, P-bar] */
  const double *gen_qmin, *gen_qmax;         /* Q-lo, Q-bar; ACOPF box is [min(0,Q-lo), max(0,Q-bar)] */
  const double *gen_c2, *gen_c1;             /* generation cost c2 p^2 + c1 p in $/MW^2h, $/MWh */
  const double *gen_cnl, *gen_csu, *gen_csd; /* no-load ($/h), start-up ($), shut-down ($) costs */
  const double *gen_ru, *gen_rd;             /* ramp-up / ramp-down limits R^U, R^D (p.u. per period) */
  const double *gen_su, *gen_sd;             /* start-up / shut-down ramps S^U, S^D */
  const int32_t *gen_min_up, *gen_min_dn;    /* T^U, T^D >= 1 (uc_minup, uc_mindn) */
  const int32_t *gen_u0;                     /* u^on_{0,g} in {0,1} */
  const int32_t *gen_init_on, *gen_init_off; /* L_g, F_g (uc_initial_on/off) */
  const double *gen_p0;                      /* p_{0,g} */
} ucac_network;

/* Algorithm parameters.  ucac_params_default fills the defaults in brackets. */
typedef struct {
  double rho_pq;      /* [5e3] penalty of power rows (line flows, generator p, q) */
  double rho_va;      /* [1e4] penalty of voltage-square and angle rows */
  double rho_uc;      /* [1e5] penalty of commitment duplicate rows */
  double rho_cpl;     /* [5e3] penalty of the six bound/ramp coupling rows */
  double beta0;       /* [1e5] initial outer penalty beta */
  double tau, theta;  /* [6, 0.8] beta grows by tau if ||z^k|| > theta ||z^{k-1}|| */
  double lambda_max;  /* [1e12] box of the outer multiplier lambda */
  double beta_max;    /* [1e24] cap of beta */
  double mu_line;     /* [5e3] penalty of the PHR line-limit term */
  int32_t newton_max_iter; /* [50] trust-region Newton iterations per line solve */
  double newton_gtol; /* [1e-12] projected-gradient tolerance, times max(1, rho_pq, rho_va) */
  int32_t max_inner;  /* [1000] inner iterations before a forced outer update */
  double eps_in0;     /* [1e-2] inner tolerance of outer iteration k: max(tol/2, eps_in0 2^-k) */
  double tol;         /* [1e-4] primal/dual residual tolerance used by the inner rule */
  int32_t warm_start; /* [0] line Newton start: 0 flat (mid voltages, zero angles),
                         1 previous iterate, 2 learned (needs ucac_set_warmstart) */
  int32_t device;     /* [0] HIP device ordinal */
  /* Residual balancing of the four penalty classes (power rows: line flows and
   * generator consensus; voltage/angle rows; bound/ramp coupling rows; commitment
   * rows), the remedy Sec. V names for the method's sensitivity to the penalties.
   * After every adapt_every-th inner iteration (0: fixed penalties), per class:
   * r = max |a_r + z_r| over its rows, s = rho max |change of the duplicates in its
   * rows| / max |y_r| over its rows; rho times adapt_tau if r > adapt_mu s, divided
   * by adapt_tau if s > adapt_mu r, within [rho / adapt_span, rho * adapt_span] of the
   * configured value, at most adapt_max times per class, not for a class whose
   * multipliers are all zero nor for one whose r and s are both at most 1e-9
   * (rounding noise).  The penalties in force are part of the iterate
   * (ucac_get_state); the multipliers are stored unscaled, so they stay valid.  With
   * it on, every iteration runs its control step as a kernel of its own. */
  int32_t adapt_every; /* [0]; 20 suits the benchmark meshes */
  double adapt_mu;     /* [3] */
  double adapt_tau;    /* [1.5] */
  int32_t adapt_max;   /* [20] */
  double adapt_span;   /* [100] */
} ucac_params;

/* Fill p with the defaults above. */
void ucac_params_default(ucac_params* p);

/* Validate and copy an instance to the device, cold-start the iterate (flat
 * voltages, mid-range generation, every unit committed, zero multipliers) and
 * build the iteration graph.  *out receives a handle the caller frees with
 * ucac_destroy.  UCAC_E_INVAL: NaN/Inf data, index out of range, a line with
 * from == to or r = x = 0, pmin > pmax, qmin > qmax, vmin > vmax or vmin <= 0,
 * min up/down < 1, u0 not in {0,1}, a bus with neither a line nor a generator,
 * or a bad parameter.  UCAC_E_NOMEM / UCAC_E_DEVICE on allocation / HIP errors. */
int ucac_create(const ucac_network* net, const ucac_params* params, ucac_handle** out);

/* Run all later work of the handle on this HIP stream (a hipStream_t, e.g. the
 * current torch stream).  NULL selects the handle's own stream. */
int ucac_set_stream(ucac_handle* h, void* hip_stream);

/* Exactly n_iters inner iterations, each followed by the inner/outer control
 * (outer update when the inner loop ends).  Does not stop at the tolerance.
 * Synchronous: returns when the work is done. */
int ucac_step(ucac_handle* h, int32_t n_iters);

/* Iterate until r_p <= tol and r_d <= tol (UCAC_OK) or until max_iters inner
 * iterations (UCAC_NOT_CONVERGED).  The stopping iteration is decided on the
 * device, so the result does not depend on how often the host polls: the call runs
 * chunks of 64 iterations from a snapshot, and a chunk that reaches the tolerance is
 * replayed from its snapshot to stop exactly there (state, multipliers, milestones
 * and work counters as if the iterations after it never ran).  Allocates the
 * snapshot (the state's size) on its first call.
 * *iters_done (may be NULL) receives the iterations run by this call. */
int ucac_solve(ucac_handle* h, double tol, int32_t max_iters, int32_t* iters_done);

/* UC warm start (Sec. IV-A: the commitments come from a multiperiod ACOPF solved
 * first, each unit on or off by its generation level there).  Replaces the iterate:
 * from the cold start, the same iteration with every commitment held at its
 * cold-start value (all units on), no dynamic program, no commitment rows and no
 * minimum-generation row -- the multiperiod ACOPF, generation anywhere in
 * [0, P-bar] -- is solved to r_p, r_d <= tol or max_iters iterations (as
 * ucac_solve); then a unit is committed in a period when its generation there is
 * at least half its minimum output P-lo, and the iterate becomes the cold start
 * with those commitments (start-ups and shut-downs from their changes, relaxed
 * commitments equal to them, slacks feasible for them, multipliers zero, beta0).
 * Returns the relaxed solve's status (UCAC_OK or UCAC_NOT_CONVERGED; the
 * commitments are set either way) or a negative error; *iters_done (may be NULL)
 * receives its iterations.  The parameters, the Newton start and a learned start
 * stay as they were. */
int ucac_uc_warmstart(ucac_handle* h, double tol, int32_t max_iters, int32_t* iters_done);

/* Residuals of the current iterate: r_primal = max |A x + B xbar| over all
 * coupling rows (the paper's primal infeasibility), r_dual = max |xbar^{l+1} -
 * xbar^l|, z_inf = max |z|, objective = generation plus commitment cost.
 * Any output pointer may be NULL. */
int ucac_residuals(const ucac_handle* h, double* r_primal, double* r_dual, double* z_inf, double* objective);

/* Copy the solution into caller-allocated host arrays (any may be NULL):
 * p, q, u_on, u_su, u_sd [T][n_gen]; vm, va [T][n_bus] (vm = sqrt(wbar),
 * va = thetabar, the bus-side duplicates). */
int ucac_get_solution(const ucac_handle* h, double* p, double* q, int8_t* u_on, int8_t* u_su,
                      int8_t* u_sd, double* vm, double* va);

/* Full iterate as a flat FP64 array (line x-side, generator x-side, duplicates,
 * z/y/lambda of every row, then beta, ||z^{k-1}||, k, l, iteration count,
 * r_p, r_in, r_d, ||z||, converged flag, the penalties in force rho_pq, rho_va,
 * rho_cpl, rho_uc and their residual-balancing change counts).  With buf == NULL only *bytes is set.
 * UCAC_E_STATE if *bytes is too small. */
int ucac_get_state(const ucac_handle* h, void* buf, size_t* bytes);

/* Replace the iterate (resume or inject).  UCAC_E_STATE if bytes differs from
 * the state size, the buffer holds NaN/Inf, or a penalty in force is not positive. */
int ucac_set_state(ucac_handle* h, const void* buf, size_t bytes);

/* Newton iterations of the last line solve, per (t, line): [T][n_line]. */
int ucac_get_branch_iters(const ucac_handle* h, int32_t* iters);

/* Start points of the last iteration that ran the learned start (ucac_set_warmstart),
 * as the network predicted them, before any fallback: x0 [4][T][n_line] (host, FP32)
 * holds v_i, v_j, theta_i, theta_j of every line solve (network outputs decoded:
 * v = 1 + y0, 1 + y1; theta = angle target + y2 / 10, + y3 / 10).  Contents are
 * unspecified if no iteration has run the learned start. */
int ucac_get_line_starts(const ucac_handle* h, float* x0);

/* Number of kernels in one inner iteration, in the order ucac_kernel_times
 * reports them: the unit side (per generator: the generator update, the UC
 * dynamic program and the relaxed commitments), lines (trust-region Newton; with
 * the learned start this slot also times the network; the line kernel also stores
 * the line-end sums of the bus QP), bus QP (bus solve with the
 * generator-consensus multipliers), the line-end duplicates with the line
 * multipliers together with the coupling/commitment multipliers (one launch),
 * control (residuals and inner/outer decision).
 * The step:outer multiplier update has no kernel of its own in an iteration: the
 * kernels that own the rows apply it in the next iteration, and a call that ends
 * with it pending applies it before returning. */
#define UCAC_N_KERNELS 5

/* Profiling: run n_iters inner iterations (exactly as ucac_step, same results)
 * with every kernel launched on its own and a HIP event recorded on the handle's
 * stream before and after it; avg_ms[k] (n_slots >= UCAC_N_KERNELS) receives the
 * mean device time of kernel k per iteration.  Those event pairs also count the
 * latency between an event record and the next dispatch.  With n_slots >
 * UCAC_N_KERNELS, avg_ms[UCAC_N_KERNELS + k] (for UCAC_N_KERNELS + k < n_slots)
 * also receives kernel k's mean duration taken from its own dispatch's begin and
 * end timestamps (the figure a kernel trace reports; the line kernel's does not
 * include the learned start's network kernel; 0 for a kernel without work).
 * Synchronous. */
int ucac_kernel_times(ucac_handle* h, int32_t n_iters, double* avg_ms, int32_t n_slots);

/* Running totals of the line kernel's work since create or the last reset:
 * out[0] evaluations of value, gradient and Hessian (one at the start of each
 * solve and one at every trial point; after a rejected trial the gradient and
 * Hessian of the current point are reused, not formed again), out[1]
 * rejected trial steps, out[2] CG iterations, out[3] Newton iterations, out[4]
 * learned starts that fell back to the flat start, out[5] Newton steps taken
 * from the direct 4x4 factorization instead of CG (the free-subspace Hessian
 * positive definite and the step inside the trust region, where CG returns the
 * same step), out[6] projected searches (a step that left the box and whose
 * projection failed the model's sufficient-decrease test, stopped instead at the
 * first bound its ray reaches); out has 7 slots.  reset != 0 zeroes them after
 * reading. */
int ucac_branch_counters(ucac_handle* h, uint64_t* out, int32_t reset);

/* After ucac_solve (or ucac_step): first_iter[m] (m = 0, 1, 2) receives the first
 * iteration of that call at which both r_primal and r_dual were <= 1e-2, 1e-3,
 * 1e-4 respectively, or -1 if never.  Recorded on the device every iteration. */
int ucac_solve_milestones(const ucac_handle* h, int32_t* first_iter);

/* ---- the UC dynamic program on its own (Sec. III-B, Alg. dp_algo) -----------
 * G independent unit-commitment DPs over T periods, one per unit, on tables the
 * caller supplies: tab[g][t][s'][s] (FP64, row-major) is the cost of period t
 * when the unit was in state s' before and is in state s (0 off, 1 on) in t.
 * min_up, min_dn (T^U, T^D; values below 1 act as 1), u0 (initial state 0/1),
 * hold_on, hold_off (L_g, F_g: periods the initial state must still be held)
 * are int32 [G].  Outputs: u_on[g][t] (int8 0/1) and cost[g], the optimal total
 * (the stay/switch recursion with "stay" on ties).  Every pointer is DEVICE
 * memory owned by the caller; the call only enqueues the work on `stream` (a
 * hipStream_t, or NULL for the default stream) and returns: synchronize before
 * reading the outputs.  lanes_per_unit: 64 (one wavefront per unit) or 16 (four
 * units per wavefront).  UCAC_E_INVAL if the horizon's LDS exceeds 64 KiB per
 * block (T above about 1200 with 64 lanes, about 300 with 16).  Errors are read
 * with ucac_last_error(NULL). */
int ucac_dp_batch(int32_t G, int32_t T, const double* tab, const int32_t* min_up, const int32_t* min_dn,
                  const int32_t* u0, const int32_t* hold_on, const int32_t* hold_off, int8_t* u_on, double* cost,
                  int32_t lanes_per_unit, void* stream);

/* ---- learned warm start of the line Newton solves --------------------------
 * A 20 -> 64 -> 64 -> 4 perceptron with SiLU activations, BF16 weights and FP32
 * accumulation on the matrix cores, predicts each line subproblem's solution
 * from its local data; Newton starts there, and a lane that does not reach the
 * Newton tolerance restarts from the flat start (the plain method stays the
 * fallback and judge; the tolerance is unchanged).  Parameters are one FP32
 * vector of UCAC_MLP_PARAMS values: W1 [64][20], b1 [64], W2 [64][64], b2 [64],
 * W3 [4][64], b3 [4] (row-major).  Inputs per line and period (20): 0.1 G_ii,
 * 0.05 B_ij, 10 (B_ii + B_ij), rating/3, the four flow targets, the two
 * voltage-square targets minus 1, 5 (angle target difference), the two
 * line-limit multipliers / mu, the four voltage bounds minus 1, log10(rho_pq) - 4,
 * log10(rho_va) - 4, (target P^2 + Q^2 - rating^2) / rating^2 at the from end.
 * Outputs (4): v_i - 1, v_j - 1, 10 (th_i - angle target i), 10 (th_j - target j). */
#define UCAC_MLP_PARAMS 5764

/* Load trained weights into the handle and use the learned start from the next
 * iteration on (the warm_start mode becomes 2).  weights == NULL returns to the
 * start of ucac_params.warm_start.  UCAC_E_INVAL for a wrong count or NaN/Inf. */
int ucac_set_warmstart(ucac_handle* h, const float* weights, size_t n);

/* Training data from the method itself: run n_iters inner iterations (as
 * ucac_step) and, in iteration i, log every stride-th line solve starting at
 * offset i % stride: its 20 inputs and its converged solution in the 4-output
 * encoding, into caller arrays feats [cap][20] and targets [cap][4] (host).
 * *n_logged receives the number of pairs kept (at most cap). */
int ucac_log_pairs(ucac_handle* h, int32_t n_iters, int32_t stride, float* feats, float* targets, int64_t cap,
                   int64_t* n_logged);

typedef struct ucac_mlp ucac_mlp;

/* A network on device `device`, weights drawn from U(-1/sqrt(fan_in), +) with
 * this seed, zero biases. */
int ucac_mlp_create(int32_t device, uint64_t seed, ucac_mlp** out);
int ucac_mlp_set_weights(ucac_mlp* m, const float* weights, size_t n);   /* n == UCAC_MLP_PARAMS; resets Adam */
int ucac_mlp_get_weights(const ucac_mlp* m, float* weights, size_t n);
/* y [n][4] = network(x [n][20]) (host arrays). */
int ucac_mlp_forward(ucac_mlp* m, const float* x, int64_t n, float* y);
/* Gradient of the mean squared error over the n samples and 4 outputs
 * (grad [UCAC_MLP_PARAMS], may be NULL) and the loss; weights unchanged. */
int ucac_mlp_grad(ucac_mlp* m, const float* x, const float* t, int64_t n, float* grad, double* loss);
/* ucac_mlp_grad for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving or training loops, harnesses that forbid hipMalloc): the
 * same kernels and the same result as ucac_mlp_grad, with no allocation of any kind.
 * x [n][20], t [n][4] (FP32), grad [UCAC_MLP_PARAMS] (FP32) and loss (one FP64) are
 * DEVICE pointers owned by the caller; loss receives the sum of squared errors over
 * the n samples and 4 outputs (ucac_mlp_grad's loss times 4n).  The call only
 * enqueues the work on `stream` (a hipStream_t, NULL for the network's own stream)
 * and returns: synchronize before reading the outputs.  The sample indices and the
 * per-wavefront gradient partials live in one fixed device array per GPU (6.0 MB,
 * held until the process ends), so n must lie in 1..UCAC_MLP_NOALLOC_MAX
 * (UCAC_E_INVAL otherwise, with the limit in ucac_mlp_last_error).  Every call on a
 * GPU uses that GPU's one array: calls that overlap on one GPU (on different streams,
 * or from different threads) race and must be serialized by the caller.  The array
 * keeps the last call's contents; each call writes every entry it reads first. */
#define UCAC_MLP_NOALLOC_MAX 16384
int ucac_mlp_grad_noalloc(ucac_mlp* m, const float* x, const float* t, int64_t n, float* grad, double* loss,
                          void* stream);
/* Adam (beta1 0.9, beta2 0.999, eps 1e-8) on shuffled mini-batches for `epochs`
 * passes over the n pairs; *last_loss = mean squared error of the last pass. */
int ucac_mlp_train(ucac_mlp* m, const float* x, const float* t, int64_t n, int32_t epochs, int32_t batch, double lr,
                   uint64_t seed, double* last_loss);
const char* ucac_mlp_last_error(const ucac_mlp* m);
void ucac_mlp_destroy(ucac_mlp* m);

/* ---- batches: many independent instances in one launch per kernel -----------
 * Every member is an ordinary instance (its own arena and state), created from
 * its network with the shared params.  One captured graph per iteration launches
 * each kernel once for all members: the grid is the concatenation of the
 * members' own grids and each block finds its member from small device tables.
 * Each member keeps its own control (residuals, beta, lambda, convergence); in
 * ucac_batch_solve a converged member stops (its blocks return at entry) while
 * the others continue.  Members' iterates are bit-identical to what the same
 * member would compute alone.  Not thread-safe; calls are serialized on the
 * batch's stream. */
typedef struct ucac_batch ucac_batch;

/* Mapping choices (results do not depend on them):
 *   dp_lanes      lanes per generator of the UC dynamic program: 64 (one
 *                 wavefront per unit) or 16 (four units per wavefront);
 *   branch_block  block size of the line kernel: 256 or 64;
 *   order         0: members in the given order; 1: largest line work first. */
typedef struct {
  int32_t dp_lanes, branch_block, order;
} ucac_batch_config;

/* nets[n] (host, read during the call); params->warm_start must be 0 or 1.
 * Errors of member k are reported as "member k: ..." by ucac_last_error(NULL). */
int ucac_batch_create(const ucac_network* nets, int32_t n, const ucac_params* params, ucac_batch** out);
int32_t ucac_batch_size(const ucac_batch* b);
/* The member's handle, owned by the batch (do not destroy it): use it with
 * ucac_residuals, ucac_get_solution, ucac_get_state, ucac_set_state. */
int ucac_batch_member(ucac_batch* b, int32_t k, ucac_handle** member);
/* n_iters inner iterations of every member. */
int ucac_batch_step(ucac_batch* b, int32_t n_iters);
/* Until every member has r_p, r_d <= tol or max_iters iterations; iters_done[n]
 * and converged[n] (host, may be NULL) per member.  UCAC_OK when all converged,
 * else UCAC_NOT_CONVERGED. */
int ucac_batch_solve(ucac_batch* b, double tol, int32_t max_iters, int32_t* iters_done, int32_t* converged);
/* Time every mapping candidate over `iters` iterations (plus 2 warm-up) from the
 * current iterate, keep the fastest, and restore the iterate.  ms_per_iter
 * receives up to n_slots per-candidate times (candidate order: dp_lanes
 * {64,16} fastest-varying, then branch_block {256,64}, then order {0,1}). */
int ucac_batch_autotune(ucac_batch* b, int32_t iters, ucac_batch_config* chosen, double* ms_per_iter, int32_t n_slots);
int ucac_batch_set_config(ucac_batch* b, const ucac_batch_config* c);
int ucac_batch_get_config(const ucac_batch* b, ucac_batch_config* c);
const char* ucac_batch_last_error(const ucac_batch* b);
void ucac_batch_destroy(ucac_batch* b);

/* Replace the parameters of a live handle (penalties, outer-loop and Newton
 * settings, tol, warm_start 0/1, residual balancing) from the next iteration on;
 * the iterate, multipliers and beta are kept (the multipliers are stored unscaled,
 * so a changed penalty leaves them valid); the penalties in force become the new
 * ones and their residual-balancing counts restart.  A learned start loaded with
 * ucac_set_warmstart stays in use.  device cannot change.  UCAC_E_INVAL for
 * invalid values (the handle is unchanged). */
int ucac_set_params(ucac_handle* h, const ucac_params* params);

/* Message of the last error on this handle (or of the last failed create when
 * h is NULL).  Valid until the next call on the handle. */
const char* ucac_last_error(const ucac_handle* h);

/* Free the handle and its device memory.  NULL is ignored. */
void ucac_destroy(ucac_handle* h);

#ifdef __cplusplus
}
#endif

#endif /* UCAC_H */
