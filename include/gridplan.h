/*
 * gridplan.h - C ABI of libgridplan, the MI355X (gfx950) hot path of
 * implicit-gradient expansion planning (Degleris, El Gamal, Rajagopal,
 * "Scalable and Interactive Electricity Grid Expansion Planning").
 *
 * Problem (Section 2.1, eq. (1) and eq. (2)):
 *   minimise over eta in [eta_min, eta_max]
 *       gamma' eta + (1/S) sum_s w_s h_s(x*_s(eta)),
 *   x*_s(eta) = argmin_x c_s(x) s.t. A_s(eta) x <= b_s(eta)   (dispatch map)
 * Gradient and update (Section 2.2):
 *   Delta = gamma + (1/S) sum_s (d x*_s/d eta)' grad h_s(x*_s),
 *   eta <- proj_[eta_min, eta_max](eta - alpha * Delta).
 *
 * Dispatch model of one scenario (hours t = 0..T-1, 1 h each):
 *   p[g,t] in [0, avail[g,t] * eta_g]     generator output
 *   f[l,t] in [-eta_l, eta_l]             line flow from -> to (AC line or
 *                                         HVDC link, Section 3.1)
 *   th[n,t] free                          bus angle
 *   ch[k,t], dis[k,t] in [0, eta_k]       battery charge / discharge
 *   soc[k,t] in [0, hours * eta_k]        battery state of charge
 *   u[n,t] >= 0                           unserved load
 *   balance: sum_{g@n} p + sum_{k@n}(dis - ch) + u + sum_{l:to=n} f
 *            - sum_{l:from=n} f = load[n,t]             (dual: price pi)
 *   flow:    f - beta_l (th[from] - th[to]) = 0         (dual: mu; AC
 *            lines only: an HVDC link's flow enters its two balance rows
 *            and is otherwise free within its capacity; beta_l may scale
 *            with eta_l, see gp_network.beta_scales)
 *   soc:     soc[t] - soc[t-1] - eff ch[t] + dis[t] = 0, cyclic (dual: nu)
 *   ramp:    p[g,t] - p[g,t-1] - s[r,t] = 0, cyclic, for the R units with a
 *            ramp limit, s[r,t] in [-rho_g eta_g, rho_g eta_g]  (dual: kappa)
 *   c_s(x) = sum cost_g p + lambda_u sum u + (r/2) ||x||^2
 *   h_s(x) = c_s(x) + omega * sum emis_g p   (emissions-aware planning),
 *            + lmp * sum pi D when a price weight is set (plan_set_price_weight)
 *
 * Canonical per-scenario vector orders (used by the accessors):
 *   x = [p (G*T) | f (L*T) | th (N*T) | ch (B*T) | dis (B*T) | soc (B*T) | u (N*T) | s (R*T)]
 *   y = [pi (N*T) | mu (L_ac*T) | nu (B*T) | kappa (R*T)], every block
 *   [device][hour], with L_ac = n_lines - n_hvdc (the AC lines come first)
 *   and the ramp blocks in generator order.
 * Capacity vector per network: eta = [generators | lines | batteries];
 * across networks the vectors are concatenated in network order (K total).
 *
 * Conventions:
 *   - All pointers in the descriptors and call arguments are HOST pointers
 *     unless stated otherwise; the library copies what it keeps.  Callers
 *     own every buffer they pass; nothing is retained after a call returns.
 *   - Every call validates its arguments on the host before touching the
 *     GPU; a negative return is an error and leaves the plan unchanged
 *     (plan_last_error() then describes it).  GP_ENOTCONVERGED (> 0) means
 *     results were written but some scenario missed the tolerance.
 *   - All device work runs on the HIP stream given to plan_init.  Calls on
 *     one plan are not thread-safe.
 */
#ifndef GRIDPLAN_H
#define GRIDPLAN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GP_OK 0
#define GP_ENOTCONVERGED 1
#define GP_EINVAL (-1)
#define GP_ENOMEM (-2)
#define GP_EHIP (-3)
#define GP_ESTATE (-4)

typedef struct gp_plan gp_plan;

/* One transmission network and its plannable devices (Section 2.1: eta
 * holds generator, line and storage capacities). */
typedef struct {
  int32_t n_nodes, n_lines, n_gens, n_batt;
  const int32_t* line_from;  /* [n_lines] node index in [0, n_nodes) */
  const int32_t* line_to;    /* [n_lines] node index, != line_from */
  const double* line_beta;   /* [n_lines] susceptance, > 0 (AC lines) */
  const int32_t* gen_node;   /* [n_gens] */
  const double* gen_cost;    /* [n_gens] marginal cost, $/MWh, >= 0 */
  const double* gen_emis;    /* [n_gens] emission rate, t/MWh, >= 0 */
  const int32_t* batt_node;  /* [n_batt] */
  const double* eta_min;     /* [n_gens + n_lines + n_batt], >= 0; battery
                                entries > 0 (dispatch_grad) */
  const double* eta_max;     /* [n_gens + n_lines + n_batt], >= eta_min */
  int32_t n_hvdc;            /* in [0, n_lines]: the last n_hvdc lines are HVDC
                                links (no power-flow row, no angle coupling;
                                their line_beta is not read) */
  int32_t beta_scales;       /* 0, or 1: the constraint matrix depends on the
                                capacities (Section 2.1's A_s(eta)): an AC
                                line's susceptance is line_beta[l] * eta_l /
                                eta_min_l (an expanded corridor of parallel
                                circuits), so AC lines need eta_min > 0; the
                                gradient then includes the matrix terms */
  const double* gen_ramp;    /* [n_gens] or NULL: share of its capacity a unit
                                can move between consecutive hours (>= 0, 0 =
                                no limit): rows p[g,t] - p[g,t-1] - s[g,t] = 0
                                (cyclic) with |s| <= gen_ramp[g] * eta_g */
} gp_network;

/* One operating scenario (Section 2.1: each scenario s has its own cost and
 * constraints; Section 3 uses independent days). */
typedef struct {
  int32_t network;     /* index into gp_case_desc.networks */
  int32_t T;           /* hours, 1 <= T <= 8784 */
  const float* avail;  /* [n_gens * T], availability in [0, 1], [g][t] */
  const float* load;   /* [n_nodes * T], MW, >= 0, [n][t] */
  double weight;       /* w_s, scales h_s in the planner objective */
} gp_scenario;

typedef struct {
  int32_t n_networks;
  const gp_network* networks;
  int32_t n_scenarios;
  const gp_scenario* scenarios;
  double r;         /* quadratic regulariser, $/MW^2 h, > 0 */
  double lambda_u;  /* unserved-load penalty, $/MWh, > 0 */
  double eff;       /* charging efficiency in (0, 1] */
  double hours;     /* battery duration, h, > 0 */
} gp_case_desc;

/* Solver options.  Zero-initialise and set what you need; zero fields take
 * the defaults given in brackets. */
typedef struct {
  double tol;            /* relative KKT residual target [1e-4]; at 1e-4
                            and above the dispatch solve restarts and
                            re-weights more often than below it, where the
                            frequent schedule stalled tight solves */
  int32_t max_iter;      /* per solve [400000] */
  int32_t check_every;   /* iterations per graph replay and convergence
                            check; 0 = chosen by the autotuner from
                            {32, 64, 128} [0] */
  int32_t block;         /* threads per block (64/128/256/512); 0 = tuned */
  int32_t no_graph;      /* 1 = launch eagerly instead of hipGraph replay */
  double rho0;           /* initial primal weight [10] */
  int32_t verbose;       /* 1 = progress lines on stderr, 2 = also a line
                            per convergence check of the first batch entry */
  int32_t variant;       /* sweep form: 0 tuned, 1 one block per tile,
                            2 persistent work queue */
  int32_t accept_warm;   /* 1 = take every warm start as given: no
                            dual screen, no stall limit [0] */
  int32_t stall_pct;     /* stall limit of a warm start, in percent of the
                            iterations of the network's last converged
                            cold solve; 0 = 100 [0] */
  int32_t reserved[4];
} gp_options;

/* Per-scenario solve statistics. */
typedef struct {
  int32_t iters;     /* iterations used */
  int32_t restarts;  /* restarts taken */
  int32_t status;    /* 0 converged, 1 iteration limit */
  int32_t start;     /* 0 cold, 1 warm, 2 warm start screened out (its
                        dual point scored below zero on the exact dual
                        function), 3 warm start abandoned for a cold
                        start after the stall limit */
  double r_pri, r_dual, r_gap, kkt;  /* relative KKT residual parts (FP64) */
  double cost;       /* c_s(x) at the returned point */
  double emis;       /* sum emis_g p at the returned point, t */
  double primal_weight;  /* final primal weight */
} gp_solve_stats;

/* Build a plan: copies the case to device memory in the library's own
 * layout.  hip_stream may be NULL: the plan then works on a private
 * non-blocking stream of its own (every call synchronises it before
 * returning).  On success *out owns
 * device memory until plan_free.  Errors: GP_EINVAL (bad shapes, indices,
 * NaN/Inf, negative costs or capacities), GP_ENOMEM, GP_EHIP. */
int plan_init(gp_plan** out, const gp_case_desc* cs, const gp_options* opt, void* hip_stream);

/* Solve the dispatch map x*_s(eta) (eq. (2)) for the listed scenarios at the
 * capacities eta (host FP64, [K], inside [eta_min, eta_max]) to the
 * relative KKT residual opt.tol:
 *   max(r_pri, r_dual, r_gap) with
 *   r_pri = ||E x - e||_inf / (1 + ||e||_inf),
 *   r_dual = ||(E'y - q - r x)_free||_inf / (1 + ||q||_inf),
 *   r_gap = |P(x) - D(y)| / (1 + max(|P(x)|, |D(y)|)), D the exact dual
 *   function, all in FP64.
 * scen: [nb] distinct scenario indices.  warm_mode: 0 cold start (x = 0,
 * y = 0), 1 start from each scenario's stored point: its last solution, or
 * the point plan_start_from_prediction seeded; scenarios without a stored
 * point start cold.  Per scenario, a warm start whose dual point has a
 * lower exact dual function value than y = 0 is replaced by the cold start
 * (stats.start = 2), and one that has not converged within the
 * iterations of the last converged cold solve on the same network (times
 * opt.stall_pct / 100) restarts cold (stats.start = 3; iters counts both
 * parts).
 * cost_out: [nb] c_s(x) (nullable).
 * stats_out: [nb] (nullable).  Returns GP_OK, GP_ENOTCONVERGED or an error. */
int dispatch_solve_batch(gp_plan* p, const double* eta, const int32_t* scen, int32_t nb,
                         int32_t warm_mode, double* cost_out, gp_solve_stats* stats_out);

/* Implicit gradient (Section 2.2) of the weighted mean planner objective
 *   (1/nb) sum_s w_s h_s(x*_s(eta)),  h_s = c_s + omega * emissions,
 * with respect to eta, for the scenarios of the last dispatch_solve_batch
 * call (scen must equal that list).  The gamma term is not included.
 * eta: nullable host [K]; when given it must equal (bitwise) the eta of that
 * solve, so a caller holding capacities from an earlier solve gets
 * GP_ESTATE instead of the gradient at other capacities.
 * At a zero generator or line capacity the value is the derivative for
 * increasing capacity: -sum_t avail * max(z, 0) for a generator and
 * -sum_t |z| for a line, z the bound's multiplier E'y - q - r x.
 * For omega > 0 the emission part solves an adjoint QP with the same
 * iteration and stopping triple, the gap measured relative to
 * 1 + max(|P|, |D|, |D(0)|) (its optimum can sit near zero); returns
 * GP_ENOTCONVERGED (gradient written) if it misses opt.tol.
 * grad_out: [K] host FP64.  h_out: nullable, receives the weighted mean
 * planner objective.  Errors: GP_ESTATE when no matching solve exists. */
int dispatch_grad(gp_plan* p, const double* eta, const int32_t* scen, int32_t nb, double omega,
                  double* grad_out, double* h_out);

/* The weighted mean planner objective (1/nb) sum_s w_s (c_s + omega * e_s)
 * of the last dispatch_solve_batch (eq. (1) without gamma'eta; c_s and the
 * emissions e_s at each scenario's returned point, FP64), for the same
 * scenario list and, when eta is given (nullable host [K]), the same
 * capacities.  h_out: host scalar.  Errors: GP_ESTATE, GP_EINVAL. */
int dispatch_objective(gp_plan* p, const double* eta, const int32_t* scen, int32_t nb, double omega,
                       double* h_out);

/* One projected gradient step (Section 2.2):
 *   Delta = gamma + dispatch_grad(...),  eta <- clip(eta - alpha*Delta).
 * Solves the listed scenarios (a stochastic batch when nb < S) at eta_inout,
 * warm-started from their previous solutions when warm_mode = 1.
 * gamma: [K] $/MW-yr.  eta_inout: [K] updated in place.  phi_out: nullable,
 * receives gamma'eta + (1/nb) sum w_s h_s at the input eta.
 * delta_out: nullable [K], receives Delta.  GP_ENOTCONVERGED: a solve or
 * the adjoint missed opt.tol; eta_inout still took the step (with the
 * gradient of the unconverged point), so a caller that wants to discard
 * such steps keeps a copy of eta. */
int plan_step(gp_plan* p, double alpha, const int32_t* scen, int32_t nb, const double* gamma,
              double omega, int32_t warm_mode, double* eta_inout, double* phi_out,
              double* delta_out);

/* Weight lmp of a planner objective on the prices (Section 2.1 lets h_s
 * depend on the LMPs): from this call on, dispatch_grad, dispatch_objective
 * and plan_step use h_s = c_s + omega * emissions + lmp * sum_{n,t}
 * pi[n,t] load[n,t] (what consumers pay at the LMPs; lmp may be negative).
 * Its gradient needs the prices' sensitivity: the adjoint solve then
 * carries lmp * load on its balance rows (the adjoint runs whenever omega >
 * 0 or lmp != 0).  Prices that the dispatch does not determine (a node all
 * of whose terminals are held at bounds) leave that adjoint infeasible and
 * the call reports GP_ENOTCONVERGED.  0 by default.  Errors: GP_EINVAL (not
 * finite; at dispatch_grad, a network with beta_scales in the batch). */
int plan_set_price_weight(gp_plan* p, double lmp);

/* Copy scenario s's last solution (canonical orders above) to host buffers:
 * x_out [n_x] FP32 and y_out [n_y] FP64 (either nullable).  n_x and n_y are
 * returned through the nullable size pointers. */
int dispatch_get_solution(gp_plan* p, int32_t s, float* x_out, double* y_out, int64_t* n_x,
                          int64_t* n_y);

/* Replace scenario s's starting point for the next warm_mode = 1 solve
 * (canonical orders; host x FP32 [n_x], y FP64 [n_y]; y may be NULL to keep
 * the stored dual, or zeros when there is none). */
int dispatch_set_start(gp_plan* p, int32_t s, const float* x, const double* y);

/* Measurement aid: continue the last solve of the listed scenarios (scen
 * must equal that call's list) for `iters` iterations launched eagerly and
 * return the mean duration, in ms from HIP events on the plan's stream, of
 * one launch of the row (dual) sweep and of the variable (primal) sweep.
 * Leaves the stored solutions untouched. */
int plan_time_sweeps(gp_plan* p, const int32_t* scen, int32_t nb, int32_t iters, double* ms_dual,
                     double* ms_primal);

/* The sweep configuration in use (set by the autotuner on the first solve
 * of a scenario list unless fixed by the options): threads per block, form
 * (1 one block per tile, 2 persistent work queue), iterations per graph
 * replay, and (nullable) the tuner's measured ms per iteration,
 * [form][block 128, 256, 512], 0 where not measured. */
int plan_tuning(const gp_plan* p, int32_t* block, int32_t* variant, int32_t* check_every,
                double* ms_table);

/* ---- learned warm start (predicted prices and angles seed the solver) ----
 * Rows are one per (listed scenario, node), scenarios in list order, nodes in
 * network order; all listed scenarios must share T.  Matrices are row-major
 * FP32 in DEVICE memory owned by the caller. */

/* Number of rows and the common horizon T of a scenario list. */
int plan_nn_rows(gp_plan* p, const int32_t* scen, int32_t nb, int64_t* rows, int32_t* T);

/* Features at capacities eta: X_dev [rows x (5T + 3)] = per hour the node's
 * load, available renewable (zero-cost) capacity, available thermal
 * capacity, neighbours' load and neighbours' available renewable capacity
 * (MW/100), then the node's battery capacity, incident line capacity and
 * thermal nameplate (MW/100). */
int plan_features(gp_plan* p, const double* eta, const int32_t* scen, int32_t nb, float* X_dev);

/* Targets from the stored solutions: Y_dev [rows x 2T] = asinh(price/100)
 * per hour, then angle/10 per hour. */
int plan_targets(gp_plan* p, const int32_t* scen, int32_t nb, float* Y_dev);

/* Seed the listed scenarios' next warm_mode = 1 solve from a prediction
 * P_dev [rows x 2T] in the target encoding: prices, clipped to
 * [0, lambda_u], become the balance duals,
 * angles the bus angles, flows the clipped DC flows of those angles,
 * generators their best response to the price, unserved load its best
 * response capped at the node's load; flow duals, batteries and SOC duals
 * zero. */
int plan_start_from_prediction(gp_plan* p, const double* eta, const int32_t* scen, int32_t nb,
                               const float* P_dev);

/* ---- the warm-start network: an MLP with BF16 MFMA GEMMs (FP32 accumulate),
 * FP32 master weights and Adam.  Layers n_in -> width (x hidden_layers) ->
 * n_out, ReLU between; parameters flat: all weight matrices ([in x out]
 * row-major, layer order) then all biases. */
typedef struct gp_mlp gp_mlp;
int mlp_init(gp_mlp** out, int32_t n_in, int32_t width, int32_t hidden_layers, int32_t n_out, uint64_t seed,
             void* hip_stream);
int mlp_num_params(const gp_mlp* m, int64_t* n);
int mlp_get_params(gp_mlp* m, float* w_out);       /* host [n] */
int mlp_set_params(gp_mlp* m, const float* w_in);  /* host [n] */
/* Y [rows x n_out] = net(X [rows x n_in]); on_device selects device (1) or
 * host (0) pointers for X and Y. */
int mlp_forward(gp_mlp* m, const float* X, int64_t rows, int32_t on_device, float* Y);
/* mlp_forward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels, with the layer activations in a file-scope device
 * array of 64 MiB (one per GPU, held until the process ends; its device
 * address is taken once per device by mlp_init) instead of buffers the
 * library allocates.  Allocates nothing and does not synchronise: the work
 * is enqueued on the network's stream and Y_dev is ready when the stream
 * reaches it.  X_dev [rows x n_in] and Y_dev [rows x n_out] are row-major
 * FP32 DEVICE buffers owned by the caller.  rows may not exceed what the
 * array holds for this network (2 * rows * max(n_in rounded up to 32, width)
 * BF16 entries): *max_rows (nullable) receives that limit, and larger rows
 * fail with GP_EINVAL (split the call).  Every call on a GPU uses that GPU's
 * one array: calls that overlap on one GPU (several streams, or several
 * networks) race and must be ordered by the caller.  Nothing in the array
 * needs to start at zero (each call writes what it reads). */
int mlp_forward_noalloc(gp_mlp* m, const float* X_dev, int64_t rows, float* Y_dev, int64_t* max_rows);
/* Mean squared error over all outputs and its parameter gradient (host
 * [n], nullable). */
int mlp_loss_grad(gp_mlp* m, const float* X, const float* T, int64_t rows, int32_t on_device, double* loss,
                  float* grad_out);
/* One Adam step (beta 0.9 / 0.999, eps 1e-8) on the mean squared error. */
int mlp_adam_step(gp_mlp* m, const float* X, const float* T, int64_t rows, int32_t on_device, double lr,
                  double* loss);
/* Standardisation of inputs and targets: column means and standard
 * deviations (FP64 sums; a column without spread keeps sd 1) of X [rows x
 * n_in] and T [rows x n_out].  From then on the network sees (x - mu)/sd,
 * is trained on (y - mu)/sd (the loss is in those units) and mlp_forward
 * returns predictions in target units. */
int mlp_fit_scaling(gp_mlp* m, const float* X, const float* T, int64_t rows, int32_t on_device);
/* Read (host arrays, each nullable) or set (host arrays, sd > 0) the
 * scaling.  GP_ESTATE from the getter when none is set. */
int mlp_get_scaling(gp_mlp* m, float* x_mu, float* x_sd, float* y_mu, float* y_sd);
int mlp_set_scaling(gp_mlp* m, const float* x_mu, const float* x_sd, const float* y_mu, const float* y_sd);
/* Mean HIP-event time (ms) of one forward pass (the layer GEMMs with their
 * bias/ReLU epilogues) over the first `rows` rows of the input loaded by the
 * last forward / loss / Adam call, `iters` passes back to back on the
 * network's stream; a measurement aid.  GP_ESTATE when fewer rows are
 * loaded. */
int mlp_time_forward(gp_mlp* m, int64_t rows, int32_t iters, double* ms_out);
/* C [M x N] = op(A) op(B) through the same BF16 MFMA kernel (host FP32 in,
 * rounded to BF16; op = transpose when ta / tb).  A is [M x K] or [K x M],
 * B [K x N] or [N x K]. */
int mlp_gemm_test(const float* A, const float* B, float* C, int32_t M, int32_t N, int32_t K, int32_t ta,
                  int32_t tb);
void mlp_free(gp_mlp* m);
const char* mlp_last_error(const gp_mlp* m);

/* Number of capacities K and scenarios S of a plan. */
int plan_sizes(const gp_plan* p, int64_t* K, int32_t* S);

/* Free the plan and its device memory (NULL is ignored). */
void plan_free(gp_plan* p);

/* Message for the last error on this plan (or of the last failed plan_init
 * when p is NULL); never NULL. */
const char* plan_last_error(const gp_plan* p);

#ifdef __cplusplus
}
#endif

#endif /* GRIDPLAN_H */
