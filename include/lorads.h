/*
 * lorads.h -- C ABI of the MI355X (gfx950) LoRADS hot-path library.
 *
 * Problem (the linear SDP of Section 1 of "A Low-Rank ADMM Splitting Approach
 * for Semidefinite Programming"):
 *
 *     min <C, X>   s.t.   <A_i, X> = b_i  (i < m),   X PSD of order n.
 *
 * The library solves it by the two-phase method of Algorithm 2: a
 * Burer-Monteiro augmented Lagrangian warm start with dynamic rank (Sections
 * 4.1-4.3) followed by the ADMM of Algorithm 1 on the split problem, whose U-
 * and V-subproblems (eqs. linU/linV) are solved by warm-started CG
 * (Section 4.4).
 *
 * Conventions shared by every entry point
 *  - Symmetric sparse matrices (C and each A_i) arrive as upper-triangle COO
 *    triplets (row <= col); an off-diagonal triplet (j, k, v) stands for both
 *    (j, k) and (k, j).  Duplicate triplets are summed.
 *  - Factor matrices (U, V, W, P, R, X) are dense, row-major, n rows, r
 *    columns, leading dimension ld >= r (elements between rows are ignored
 *    and never written).
 *  - Pointers named "device" are HIP device pointers owned by the caller
 *    (e.g. torch tensor data_ptr()); pointers named "host" are host memory
 *    owned by the caller.  The library never frees caller memory.
 *  - Constraint-indexed vectors (b, z, w, lambda) use the caller's constraint
 *    numbering (the a_con ids of the problem).
 *  - dtype selects the element type of every floating-point device array of
 *    the call: LORADS_F64 (double) or LORADS_F32 (float).  Arithmetic inside
 *    a call is done in that type, with FP64 accumulation of reductions.
 *  - stream is a hipStream_t (NULL = the default stream).  Calls enqueue work
 *    on it and return without waiting, unless stated otherwise.
 *  - Errors are returned as lorads_status, never thrown across the ABI.  On an
 *    error the outputs are unspecified; lorads_last_error() gives a message.
 *  - A context is not thread-safe; distinct contexts are independent.
 */
#ifndef LORADS_H
#define LORADS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lorads_ctx lorads_ctx;

typedef enum {
  LORADS_OK = 0,
  LORADS_MAXITER = 1,    /* iteration cap reached before the tolerance */
  LORADS_TIMELIMIT = 2,  /* time limit reached before the tolerance */
  LORADS_EINVAL = -1,    /* invalid argument or malformed problem */
  LORADS_ENOMEM = -2,    /* device allocation failed */
  LORADS_EDEVICE = -3,   /* HIP runtime error */
  LORADS_ENUMERIC = -4,  /* non-finite value met during a solve */
  LORADS_ESTATE = -5     /* call out of order (e.g. solution before solve) */
} lorads_status;

typedef enum { LORADS_F64 = 0, LORADS_F32 = 1 } lorads_dtype;
/* the third solver precision (lorads_options.precision) */
#define LORADS_MIXED 2

/* Constraint structure detected by lorads_setup. */
typedef enum {
  LORADS_STRUCT_GENERIC = 0, /* any sparse symmetric A_i */
  LORADS_STRUCT_DIAG = 1,    /* every A_i = a_i e_j e_j^T (MaxCut: diag(X) = 1) */
  LORADS_STRUCT_PAIR = 2,    /* every A_i = a_i (e_j e_k^T + e_k e_j^T), j < k
                                (matrix completion) */
  LORADS_STRUCT_RANK1 = 3    /* every A_i = c_i a_i a_i^T with a sparse a_i
                                (sensor network localization, Section 3; the
                                balance constraint <1 1^T, X> = 0 of graph
                                bisection), when not DIAG */
} lorads_structure;

/* One SDP instance, host memory, caller-owned; lorads_setup copies it. */
typedef struct {
  int32_t n;                 /* order of X, >= 1 */
  int32_t m;                 /* number of constraints, >= 1 */
  int64_t c_nnz;             /* C triplets (may be 0: C = 0) */
  const int32_t *c_row;      /* [c_nnz], 0 <= row <= col < n */
  const int32_t *c_col;      /* [c_nnz] */
  const double *c_val;       /* [c_nnz], finite */
  int64_t a_nnz;             /* triplets of all A_i together, >= 1 */
  const int32_t *a_con;      /* [a_nnz], constraint id in [0, m) */
  const int32_t *a_row;      /* [a_nnz], 0 <= row <= col < n */
  const int32_t *a_col;      /* [a_nnz] */
  const double *a_val;       /* [a_nnz], finite */
  const double *b;           /* [m], finite */
  double mu;                 /* objective f(X) = <C, X> + (mu / 2) ||X||_F^2
                                (Section 1's convex f; mu = 0: the linear SDP);
                                finite and >= 0 (EINVAL otherwise); the
                                batched solve takes mu = 0 only */
} lorads_problem;

/* Solver parameters.  lorads_default_options() fills the documented defaults;
 * fields marked (paper) are fixed by Section 5.1/5.2, the others are the
 * library's rules where the paper is silent. */
typedef struct {
  int32_t precision;       /* LORADS_F64: plain FP64 method.  LORADS_F32: CG
                              iterations in FP32 on FP32 copies of the fixed
                              factor; U, V, lambda, right-hand sides, dual
                              updates, decisions and residuals stay FP64.
                              LORADS_MIXED (2): as LORADS_F32, and the two
                              maps of Phase I's exact line search,
                              A(U D^T + D U^T) and A(D D^T), read FP32 copies
                              of U and the direction D (FP32 inner products;
                              the quartic's sums, the gradient, z, lambda and
                              every decision stay FP64).  Applies to
                              symmetric-pair structures with one coefficient
                              and r >= 9; elsewhere it runs as LORADS_F32 */
  double eps;              /* final tolerance on eq. (stop), default 1e-6 */
  double switch_tol;       /* phase-I exit on primal infeasibility, default 1e-3
                              (Section 5.1: 1e-3 for most instances; its 1e-2
                              for MaxCut goes with a stop on primal
                              infeasibility alone, not with eq. (stop)) */
  double h;                /* rho factor at the phase switch (paper) */
  double rho_growth;       /* 1.2 (paper) */
  int32_t rho_every;       /* 5 (paper) */
  double rho_max;          /* 5000 (paper) */
  int32_t max_admm_iter;   /* 5000 (paper) */
  double time_limit;       /* seconds; <= 0: none */
  double gamma_fixed;      /* > 0: fixed gamma; 0: the library's gamma rule */
  double gamma_scale;      /* gamma rule: gamma = gamma_scale * (1 + scale), scale
                              as gamma_rule selects */
  double cg_tol_max;       /* CG relative tolerance tau = min(cg_tol_max, */
  double cg_tol_floor;     /*   max(cg_tol_floor, cg_tol_kkt * KKT_prev))  */
  double cg_tol_kkt;
  int32_t cg_maxit;        /* cap min(n r, cg_maxit) */
  int32_t lbfgs_mem;       /* L-BFGS memory, default 4 */
  int32_t alm_inner_max;   /* inner iteration cap at the rank cap, 2000 */
  int32_t rank_grow_iters; /* an inner solve reaching this count grows the rank, 1000 */
  double rank_factor;      /* 1.5 (paper) */
  int32_t r0;              /* initial rank (> 0 required unless init_U given) */
  int32_t r_max;           /* rank cap: min(r_max, n, 256), or with r_max = 0
                              min(floor(sqrt(2m)), n, 256) (floor(sqrt(2m)) is
                              the Barvinok-Pataki bound of Section 2; 256 is the
                              largest rank the operator kernels take).  The
                              batched launch caps ranks at 32 as well (its lane
                              group holds one factor row); a solve never raises
                              the rank above its cap */
  double alm_inner_rel;    /* inner stop ||grad||/(1+||C||_F) <= max(rel v, floor) */
  double alm_inner_floor;
  double alm_eta;          /* multiplier update when v <= eta * v_at_last_update */
  double alm_rho_factor;   /* otherwise rho *= factor */
  int32_t alm_outer_max;
  double rho0;             /* phase-I initial rho; 0: 1/max(1, ||b||_inf) */
  uint64_t seed;           /* SplitMix64 stream for rank-growth columns */
  int32_t phase1;          /* 1: run the warm start; 0: start ADMM at init_U */
  int32_t verbose;         /* 0 silent, 1 per-phase summary, 2 per iteration */
  int32_t profile;         /* 1: time the operator launches with HIP events
                              (fields prof_* of the result); 2: time only the
                              fused CG operator (class 0), whose launches carry
                              their own start / stop events, so the other
                              launches run without event records between them;
                              other values: EINVAL */
  int32_t batch_mode;      /* 0: batched persistent launch when the context holds
                              >= 2 problems, all with diagonal constraints
                              (MaxCut), else one problem after the other;
                              1: require the batched launch (EINVAL otherwise);
                              2: always one problem after the other */
  int32_t batch_block;     /* workgroup size of the batched launch (multiple of
                              64 up to 256); 0: the context's tuned value
                              (lorads_batch_autotune), default 256 */
  /* per-problem starting points, host, caller-owned, arrays of nprob pointers
     (NULL or a NULL entry: not given).  init_U[p] is n x r0 row-major; without
     it the problem cannot be solved (the random start is an input).
     init_lambda[p] has m entries in the caller's constraint order. */
  const double *const *init_U;
  const double *const *init_lambda;
  const int32_t *init_rank;  /* per-problem initial rank (nprob entries, NULL:
                                r0 for every problem); init_U[p] is n x init_rank[p] */
  int32_t warm_check;      /* 1: a problem started from a given init_lambda falls
                              back to the cold start (lambda = 0, the given U) when
                              the first Phase-I outer iteration does not lower the
                              primal infeasibility; such problems are solved one
                              after the other (batch_mode 1: EINVAL).  Default 0 */
  int32_t gamma_rule;      /* scale of the gamma rule (gamma_fixed = 0):
                              0: gamma = gamma_scale (1 + ||C||_F / sqrt(n)), the
                              cost's per-row scale (default);
                              1: gamma = gamma_scale (1 + ||C||_2), the cost's
                              operator norm, estimated once per problem by the
                              power method on C (relative change < 1e-12, at most
                              1000 products) -- for costs whose norm sits in few
                              directions, such as -J of the Lovasz theta SDP.
                              The batched launch takes rule 0 only */
} lorads_options;

typedef struct {
  int32_t status;          /* lorads_status of this problem */
  int32_t rank;            /* final rank r */
  int32_t alm_outer, alm_inner, rank_growths;
  int32_t admm_iters;
  int64_t cg_iters;        /* total CG iterations of phase II */
  double obj;              /* f(X) at X = U_hat U_hat^T, U_hat = (U + V)/2:
                              <C, X> (+ (mu/2) ||X||_F^2) */
  double dual_obj;         /* b^T y with y = -lambda */
  double pinf;             /* ||A(X) - b||_2 / (1 + ||b||_1)      (App. B) */
  double dinf;             /* |min(0, lambda_min(C - A*(y)))| / (1 + ||vec C||_1);
                              with mu != 0, C + mu X in place of C */
  double gap;              /* (<C,X> - b^T y) / (1 + |<C,X>| + |b^T y|); with
                              mu != 0, <C + mu X, X> in place of <C, X> */
  double lambda_min;       /* smallest eigenvalue of the dual slack */
  double kkt;              /* final value of eq. (stop) */
  double pinf_stop;        /* ||A(UV^T) - b||_2 / (1 + ||b||_inf) at exit */
  double dres_stop;        /* gamma ||V+ - V||_F / (1 + ||V||_F) at exit */
  double rho, gamma;       /* final penalties */
  double t_phase1, t_phase2, t_metrics, t_total;   /* seconds */
  double op_bytes;         /* algorithmic bytes of every A(.) / A*(.)V / CG
                              operator application of the solve */
  /* with options.profile: per kernel class (0 fused CG operator, 1 forward map,
     2 adjoint product, 3 the warm start's line-search pair of maps) the summed
     launch time in ms measured by HIP events on the solver's stream, the number
     of launches and their algorithmic bytes */
  double prof_ms[4];
  double prof_bytes[4];
  int64_t prof_launches[4];
  int32_t warm_fallback;   /* 1 when options.warm_check restarted Phase I cold */
} lorads_result;

/* Fill *opt with the defaults above (precision F64, eps 1e-6, switch 1e-3,
 * h 1, ...). */
void lorads_default_options(lorads_options *opt);

/* Validate and ingest nprob problems onto the current HIP device.
 * Checks: n, m >= 1; indices in range; row <= col; finite values; every
 * constraint has at least one triplet.  Detects the structure class of each
 * problem, builds the device layouts and reorders constraints internally.
 * nprob > 1 enables the batched solve.  Returns EINVAL before touching the
 * device when the input is malformed.  *out receives the new context. */
lorads_status lorads_setup(const lorads_problem *probs, int32_t nprob, lorads_ctx **out);

/* Structure class, n and m of problem `prob`. */
lorads_status lorads_problem_info(const lorads_ctx *ctx, int32_t prob, int32_t *structure,
                                  int32_t *n, int32_t *m);

/* Layout flags of problem `prob` (*flags, a bit set):
 * LORADS_FLAG_DENSE_C: C has at least n^2 / 4 entries and n >= 256, so it is
 * also kept dense (n x ldc, FP64 and FP32) and every product with C runs on
 * the matrix cores (MFMA), for r <= 64; otherwise its sparse rows are used. */
#define LORADS_FLAG_DENSE_C 1
lorads_status lorads_problem_flags(const lorads_ctx *ctx, int32_t prob, int32_t *flags);

/* z = A(U V^T), z_i = <A_i, U V^T> (definition of the linear map, Section 1).
 * U, V: device, n x r (ld); z: device, m.  Enqueued on stream. */
lorads_status lorads_apply_A(lorads_ctx *ctx, int32_t prob, const void *U, const void *V,
                             int32_t r, int32_t ld, void *z, int32_t dtype, void *stream);

/* out = (c_scale C + A*(w)) V with A*(w) = sum_i w_i A_i: the products in the
 * subproblem optimality conditions (optU)/(optV) and the right-hand sides of
 * (linU)/(linV).  w: device, m; V, out: device, n x r (ld). */
lorads_status lorads_apply_AT_V(lorads_ctx *ctx, int32_t prob, const void *w, double c_scale,
                                const void *V, int32_t r, int32_t ld, void *out,
                                int32_t dtype, void *stream);

/* Solve the subproblem system of (linU)/(linV),
 *     gamma X + rho A*(A(X W^T)) W = R,
 * by unpreconditioned CG (Section 4.4) on the n x r matrix space with the
 * Frobenius inner product, starting from the content of X (device, in: x0,
 * out: solution).  Stops when ||R - M X||_F <= tol ||R - M x0||_F or after
 * maxit iterations.  W, R, X: device n x r (ld).  Blocks the host until done;
 * *iters and *relres (host, may be NULL) receive the iteration count and the
 * final relative residual.  Returns MAXITER if the tolerance was not met.
 * This is the linear objective's operator: a problem's mu is not applied
 * here (solves add mu X (W^T W) themselves). */
lorads_status lorads_cg_solve(lorads_ctx *ctx, int32_t prob, const void *W, double rho,
                              double gamma, const void *R, void *X, int32_t r, int32_t ld,
                              double tol, int32_t maxit, int32_t dtype, int32_t *iters,
                              double *relres, void *stream);

/* lorads_cg_solve for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same CG, kernels and results, with the work buffers (the CG-layout copies
 * of W, R and X, the direction and the operator output; for general
 * constraints also one m-vector; for completion factors whose interleaved rows
 * exceed 4 MiB also 8 n ld_cg partial sums) placed in a static device workspace of
 * 64 MiB that the library holds on each GPU it runs on until the process ends,
 * instead of allocated.  The call allocates nothing; lorads_setup records the
 * workspace of the current device and creates every buffer the call touches.
 * Arguments, layout, ownership and blocking as lorads_cg_solve.  Errors:
 * EINVAL when one call needs more than 64 MiB of workspace (about
 * (6 n ld_cg) elements, ld_cg = r rounded up to 64 bytes for completion
 * problems, r otherwise) or for rank-one constraint problems
 * (LORADS_STRUCT_RANK1, whose work vectors grow with the rank), ESTATE when
 * the context was set up on another device.  Every call on a GPU uses that GPU's one workspace, which keeps the
 * last call's contents (the call clears what must start at zero): calls that
 * overlap on one GPU (other threads, other streams, other contexts) race. */
lorads_status lorads_cg_solve_noalloc(lorads_ctx *ctx, int32_t prob, const void *W, double rho,
                                      double gamma, const void *R, void *X, int32_t r, int32_t ld,
                                      double tol, int32_t maxit, int32_t dtype, int32_t *iters,
                                      double *relres, void *stream);

/* Full two-phase solve (Algorithm 2) of every problem of the context; with
 * nprob > 1 all problems advance together in batched launches.  res: host
 * array of nprob results.  Blocks the host until done.  Returns the worst
 * per-problem status. */
lorads_status lorads_admm_solve(lorads_ctx *ctx, const lorads_options *opt, lorads_result *res);

/* Autotuner of the batched launch: runs the batched solve once per candidate
 * workgroup size (host array cand[ncand], multiples of 64 up to 256) with the
 * given options (callers pass a short iteration budget), times each run with
 * HIP events, keeps the fastest in the context for later solves with
 * batch_block = 0 and returns it in *best (times_ms, host, may be NULL:
 * ncand timings).  Overwrites the problems' last solutions.  EINVAL unless the
 * context is eligible for the batched launch. */
lorads_status lorads_batch_autotune(lorads_ctx *ctx, const lorads_options *opt, const int32_t *cand,
                                    int32_t ncand, int32_t *best, double *times_ms);

/* Copy the last solution of problem `prob` to host buffers (any may be NULL):
 * U, V: n x rank row-major; lambda: m (caller order).  ESTATE before a solve. */
lorads_status lorads_get_solution(const lorads_ctx *ctx, int32_t prob, double *U, double *V,
                                  double *lambda);

/* G = A^T B for tall-skinny A (n x ra, lda) and B (n x rb, ldb), FP64, with
 * gfx950 FP64 MFMA tiles; G: device ra x rb row-major.  The r x r Gram
 * products used for ||X||_F and the completion recovery error. */
lorads_status lorads_gram(const void *A, const void *B, int64_t n, int32_t ra, int32_t rb,
                          int32_t lda, int32_t ldb, void *G, void *stream);

/* Smallest eigenvalue of the dual slack C + A*(lambda) (= C - A*(y), y = -lambda)
 * by Lanczos with full reorthogonalisation (Appendix B's dual infeasibility).
 * lambda: device, m, FP64, caller order.  Blocks the host.  With mu != 0 the
 * solver's own measures use grad f(X) = C + mu X in place of C; this call
 * takes C alone. */
lorads_status lorads_dual_lambda_min(lorads_ctx *ctx, int32_t prob, const void *lambda,
                                     int32_t max_steps, double *out);

void lorads_destroy(lorads_ctx *ctx);

/* Message for the last non-OK status of ctx (or, when ctx is NULL, of the last
 * failed setup or lorads_gnn_* call on this thread).  Valid until the next call on the same context. */
const char *lorads_last_error(const lorads_ctx *ctx);

/* Library version string. */
const char *lorads_version(void);

/* ------------------------------------------------------------------------
 * Learned warm start for Phase I.  The paper names better warm starts as
 * future work (Section 6); this network is an addition.  A message-passing
 * network over a weighted graph (for MaxCut, the graph itself) predicts a
 * dual multiplier per node, used as lambda0 = -yhat, and a graph-level rank
 * factor.  FP32 throughout; hidden width 64.
 *
 *   x_j  = [deg_j, sum_k w_jk, sum_k |w_jk|, sum_k w_jk^2, ln n_g] / 10
 *   A_jk = w_jk / (1 + sum_k |w_jk|)
 *   H0 = relu(x W_in^T + b_in);  H_l = relu(H_{l-1} W_s^T + (A H_{l-1}) W_n^T + b_l)
 *   yhat_j = <H_L[j], v_y> + c_y;   rhat_g = <mean_{j in g} H_L[j], v_r> + c_r
 *   loss = mean_j (yhat_j - y_j)^2 + omega mean_g (rhat_g - r_g)^2
 *
 * Parameters form one flat FP32 vector: W_in (64 x 5), b_in (64), per layer
 * W_s (64 x 64), W_n (64 x 64), b (64), then v_y (64), c_y, v_r (64), c_r;
 * matrices row-major (out x in).  lorads_gnn_param_count gives its length.
 * All buffers in these calls are host memory unless stated; every call blocks
 * the host until its device work is done.
 * ------------------------------------------------------------------------ */
typedef struct lorads_gnn lorads_gnn;

/* Number of parameters for `layers` message-passing layers (hidden 64). */
int64_t lorads_gnn_param_count(int32_t layers);

/* Create a network on the current HIP device with zero parameters and zero
 * Adam state.  layers in [1, 8].  EINVAL otherwise. */
lorads_status lorads_gnn_create(int32_t layers, lorads_gnn **out);

/* Copy count (= lorads_gnn_param_count) parameters from / to host FP32.
 * set_params also clears the Adam moments and step counter. */
lorads_status lorads_gnn_set_params(lorads_gnn *g, const float *theta, int64_t count);
lorads_status lorads_gnn_get_params(const lorads_gnn *g, float *theta, int64_t count);

/* Replace the resident graph set.  Graph q owns nodes [node_off[q],
 * node_off[q+1]) (node_off: n_graphs + 1 ascending entries, node_off[0] = 0).
 * Edges are nnz directed COO triplets (row[e], col[e], w[e]) over global node
 * ids; an undirected edge is listed in both directions, both ends in the same
 * graph; no self loops; weights finite.  The library builds the adjacency rows,
 * the features and the normalised weights on the device and keeps activations
 * for every node resident.  EINVAL on any violation. */
lorads_status lorads_gnn_load_graphs(lorads_gnn *g, int32_t n_graphs, const int64_t *node_off,
                                     int64_t nnz, const int32_t *row, const int32_t *col,
                                     const float *w);

/* Training targets for the whole graph set: y (one per node) and r (one per
 * graph), host FP32. */
lorads_status lorads_gnn_set_targets(lorads_gnn *g, const float *y, const float *r);

/* Forward pass over graphs [g0, g1): yhat for their nodes (node_off[g1] -
 * node_off[g0] entries) and rhat (g1 - g0 entries); either may be NULL. */
lorads_status lorads_gnn_forward(lorads_gnn *g, int32_t g0, int32_t g1, float *yhat, float *rhat);

/* Forward and backward pass over graphs [g0, g1) against the targets: *loss
 * (may be NULL) and the gradient, which stays on the device for
 * lorads_gnn_adam_step and is also copied to grad (count entries, may be
 * NULL).  ESTATE before set_targets. */
lorads_status lorads_gnn_loss_grad(lorads_gnn *g, int32_t g0, int32_t g1, float omega,
                                   double *loss, float *grad, int64_t count);

/* One Adam update (bias-corrected moments) with the last gradient.  ESTATE
 * before a loss_grad call. */
lorads_status lorads_gnn_adam_step(lorads_gnn *g, float lr, float beta1, float beta2, float eps);

/* Summed HIP-event time (ms) and launch count of the dense layer kernels
 * (message aggregation + the MFMA products) since the last call; the counters
 * are reset by the call.  Either pointer may be NULL. */
lorads_status lorads_gnn_layer_time(lorads_gnn *g, double *ms, int64_t *launches, double *flops);

void lorads_gnn_destroy(lorads_gnn *g);

#ifdef __cplusplus
}
#endif

#endif /* LORADS_H */
