/*
 * certglm: safe dual bounds for branch-and-bound nodes of the k-sparse, box-constrained,
 * ridge-regularised GLM, computed on one AMD Instinct MI355X (gfx950).
 *
 * Method: Liu et al., "Scalable First-order Method for Certifying Optimal k-Sparse GLMs"
 * (arXiv 2502.09502). The problem is problem (1) of Sec. 1,
 *
 *     min_beta f(X beta, y) + lambda2 ||beta||_2^2   s.t.  ||beta||_inf <= M,  ||beta||_0 <= k,
 *
 * with f the least-squares loss ||u - y||^2, the logistic loss sum log(1 + exp(-y_i u_i)) or the
 * squared hinge loss sum max(0, 1 - y_i u_i)^2, or the Poisson and Gamma losses (App. D.1).
 * A node fixes z_j = 0 on a set Z0 and z_j = 1 on a set Z1 in the perspective relaxation
 * P_conv of Sec. 2; this library solves that relaxation by restarted FISTA (Alg. 3) with the
 * exact prox of Alg. 1 (via the Moreau identity of Sec. 3.3) and the value of g from Alg. 2,
 * and certifies every answer with the weak-duality bound of Sec. 3.4, evaluated in FP64.
 *
 * Conventions (every entry point):
 *   - returns an int status, CGL_OK (0) on success; no C++ exception or abort crosses the ABI;
 *     cgl_status_str() names a status, cgl_last_error() gives the detail of the last failure
 *     on the calling thread;
 *   - pointers are host pointers unless an argument says otherwise;
 *   - the caller owns every buffer it passes; the library copies what it keeps;
 *   - indices are 0-based; matrices are row-major with a leading dimension;
 *   - a context and the objects created from it are used by one thread at a time.
 */
#ifndef CERTGLM_H
#define CERTGLM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CGL_ABI_VERSION 1

/* ------------------------------------------------------------------ statuses and enums */

enum cgl_status {
  CGL_OK = 0,
  CGL_E_INVAL = 1,    /* an argument is invalid (detail in cgl_last_error) */
  CGL_E_NOMEM = 2,    /* device or host allocation failed */
  CGL_E_DEVICE = 3,   /* a HIP runtime call failed */
  CGL_E_BUSY = 4,     /* server queue full */
  CGL_E_NOTFOUND = 5, /* unknown ticket */
  CGL_E_INTERNAL = 6
};

enum cgl_dtype { CGL_F64 = 0, CGL_F32 = 1, CGL_BF16 = 2 };
enum cgl_mem { CGL_MEM_HOST = 0, CGL_MEM_DEVICE = 1 };
enum cgl_loss {
  CGL_LOSS_LS = 0,
  CGL_LOSS_LOGISTIC = 1,
  CGL_LOSS_SQHINGE = 2,
  CGL_LOSS_POISSON = 3, /* sum exp(u_i) - y_i u_i, y_i >= 0; needs an explicit L */
  CGL_LOSS_GAMMA = 4    /* sum y_i exp(-u_i) + u_i, y_i > 0; needs an explicit L */
};

/* Arithmetic of the iteration. Every bound is certified in FP64 either way.
 *   CGL_PREC_F64:   FP64 iterates and FP64 products with X in its stored precision
 *                   (the plain per-node path);
 *   CGL_PREC_MIXED: BF16 operands on MFMA with FP32 accumulation for the correction products
 *                   around an FP64 base point that is re-centred in FP64 when progress stalls. */
enum cgl_precision { CGL_PREC_F64 = 0, CGL_PREC_MIXED = 1 };

/* Per-node result status. */
enum cgl_node_status {
  CGL_CONVERGED = 0,     /* FP64-certified relative gap <= tol */
  CGL_NOT_CONVERGED = 1, /* max_iter reached; lower_bound is still a valid bound */
  CGL_INFEASIBLE = 2,    /* |Z1| > k: no feasible z; lower_bound = +inf */
  CGL_NUMERIC = 3,       /* a non-finite value appeared; lower_bound is the best valid one */
  CGL_CANCELLED = 4,     /* server request cancelled before completion */
  CGL_PRUNED = 5,        /* certified lower bound > incumbent: the node can be pruned */
  CGL_BELOW_INCUMBENT = 6 /* primal value < incumbent: stop and branch (Sec. 4.3 rules) */
};

typedef struct cgl_ctx cgl_ctx;
typedef struct cgl_problem cgl_problem;
typedef struct cgl_server cgl_server;

/* ------------------------------------------------------------------ node and result */

/* One branch-and-bound node. fixed_zero = Z0 (beta_j = 0), fixed_in = Z1 (z_j = 1: the
 * coordinate pays lambda2 beta_j^2 and |beta_j| <= M but not the cardinality budget beyond its
 * own unit). Indices must be distinct, in [0, p) and Z0, Z1 disjoint, else CGL_E_INVAL.
 * |Z1| > k is not an error: the result is CGL_INFEASIBLE with lower_bound = +inf.
 * The relative gap is (P_best - D_best) / max(|P_best|, 1). */
typedef struct cgl_node {
  const int32_t* fixed_zero;
  int32_t n_zero;
  const int32_t* fixed_in;
  int32_t n_in;
  double tol;           /* relative-gap tolerance, e.g. 1e-6 */
  int32_t max_iter;     /* iteration cap (>= 1) */
  int32_t check_every;  /* dual monitor period in iterations (>= 1). On the FP64 path the
                           monitor is the certified bound; on the batched engine it is a
                           working-precision estimate that only decides when the node asks
                           for its FP64 certificate, and a period of 2 is the faster choice
                           on a 256-node batch */
  int32_t precision;    /* enum cgl_precision */
  const double* warm_start; /* NULL, or p host doubles: the first iterate (fixed-zero entries
                                are set to 0); with CGL_PREC_MIXED the FP64 base point is
                                computed there before the first iteration */
  double incumbent;     /* +inf for none; else the early-termination rules of Sec. 4.3 apply */
} cgl_node;

typedef struct cgl_result {
  double lower_bound; /* FP64 weak-duality bound D(zeta); valid whatever the status */
  double primal;      /* FP64 objective of the returned beta (an upper bound on P_conv) */
  double gap_abs;     /* primal - lower_bound */
  double gap_rel;     /* gap_abs / max(|primal|, 1) */
  int32_t iters;      /* FISTA iterations run */
  int32_t restarts;   /* momentum restarts (phi reset to 1) */
  int32_t status;     /* enum cgl_node_status */
  int32_t recentres;  /* FP64 re-centrings (mixed precision only) */
  double err_vs_fp64_est; /* |working-precision objective - FP64 objective| / max(|P|, 1) at the
                             returned beta: the error of the fast arithmetic against FP64 */
} cgl_result;

/* Fill a node with defaults: no fixed sets, tol 1e-6, max_iter 100000, check_every 1,
 * CGL_PREC_F64, no warm start, incumbent +inf. */
void cgl_node_init(cgl_node* node);

int cgl_version(void);
const char* cgl_status_str(int status);
const char* cgl_last_error(void);

/* ------------------------------------------------------------------ context */

/* device: HIP device ordinal. hip_stream: a hipStream_t to run on, or NULL for a stream the
 * context creates (default priority). CGL_E_DEVICE on HIP failures. */
int cgl_ctx_create(int device, void* hip_stream, cgl_ctx** out);
int cgl_ctx_destroy(cgl_ctx* ctx);

/* Kernel timing (measurement support). While on (on = 1 or 2), solves on this context time
 * every launch of the listed kernels with HIP events on the context's stream (both paths then
 * launch without graph capture; the batched products are launched with their start and stop
 * events attached, the other kernels are bracketed) and accumulate the elapsed time of launches
 * that did work. The batched X pass (which = 3) is timed only at on = 2: a timed launch starts
 * a few microseconds later. on = 3 records only the host wall time of the batched engine's
 * phases (which = 5, 6, 7 below) and leaves the launches as they run unprofiled (graph-captured
 * chunks). CGL_E_INVAL for another value of on.
 * which: 0 = X^T pass of the plain path (k_xt), 1 = X pass of the plain path (k_xb),
 *        2 = batched BF16 MFMA X^T pass, 3 = batched BF16 MFMA X pass, 4 = batched FP64 pass;
 *        and host wall time of the batched engine's phases (launch to completion):
 *        5 = iteration chunks, 6 = certification rounds, 7 = admission and retirement;
 *        8 = the prox kernel of cgl_prox_node_batch (one launch per call);
 *        9 = the batched X pass's operand extent: total_ms holds the sum over passes of the
 *            fraction of the padded columns read (not a time), launches the passes;
 *        10, 11 (on = 3 only) = GPU time of the batched engine's graph-captured chunks and of
 *            its certification rounds (HIP events around each on the stream);
 *        12 = rewrites of the batched engine's support-first column order (launches = count,
 *            total_ms = 0); 13 = nodes admitted into the batched engine's slots (launches =
 *            count, total_ms = 0);
 *        14 = the tilings of the products of the last batched engine set up on this context,
 *            whatever the profiling level (total_ms = the X pass's code, launches = the X^T
 *            pass's; code = split-K, plus 100 for the 128-row tile or 200 for the 64-row tile,
 *            else 256 rows; 0 before any engine); reset does not apply to it.
 * cgl_ctx_kernel_stats returns the totals since the last reset (reset = 1 clears them). */
int cgl_ctx_set_profiling(cgl_ctx* ctx, int32_t on);
int cgl_ctx_kernel_stats(cgl_ctx* ctx, int32_t which, int32_t reset, double* total_ms,
                         int64_t* launches);

/* ------------------------------------------------------------------ problem */

/* Create the problem data of problem (1) on the device.
 *   X      : n x p row-major, leading dimension ldx >= p, element type x_dtype (F64, F32, or
 *            BF16 as raw 16-bit patterns); x_mem says whether X is a host or a device pointer.
 *            The values given ARE the problem (a BF16 X is not an approximation of anything).
 *   y      : n host doubles (logistic and squared hinge: each -1 or +1; Poisson >= 0; Gamma > 0).
 *   loss   : enum cgl_loss.  lambda2 > 0, M > 0, k >= 1.
 *   L      : Lipschitz constant of grad F (Alg. 3); L <= 0 asks the library to compute it
 *            (power iteration on X^T X in FP64, times 2 for least squares and squared hinge,
 *            / 4 for logistic, then enlarged by a safety factor of 1.002); Poisson and Gamma
 *            have no global constant and need L > 0.
 * The library copies X (in its stored precision, plus a transposed BF16 copy for the mixed
 * path) and y into device memory it owns. The values of the arguments (host X and y included)
 * are checked before ctx, so that a NULL ctx with a bad argument reports the argument. Errors: CGL_E_INVAL (n, p < 1; p > 32768; ldx < p;
 * lambda2 <= 0; M <= 0; k < 1; a non-finite entry of X (NaN or infinity in any dtype, checked
 * on the device copy whether X was given in host or in device memory); non-finite y; y outside
 * the loss's range; L <= 0 for Poisson or Gamma), CGL_E_NOMEM. */
int cgl_problem_create(cgl_ctx* ctx, const void* X, int32_t x_dtype, int32_t x_mem, int64_t n,
                       int64_t p, int64_t ldx, const double* y, int32_t loss, double lambda2,
                       double M, int32_t k, double L, cgl_problem** out);
/* Destroying an owner of a shared design (below) leaves its sharers standalone; destroying a
 * sharer drops it from its owner's engine. Neither may have nodes on a server then. */
int cgl_problem_destroy(cgl_problem* prob);
/* Two problems on the same design X (problem (1) with other labels, loss or constants, e.g. a
 * least-squares and a logistic relaxation of one dataset): from now on the owner's batched
 * engine also serves the sharer's mixed-precision nodes, so that one pass over the BF16 design
 * per iteration advances the nodes of both (cgl_solve_batch and the server route the sharer's
 * nodes there; its FP64-path solves are its own). Each node keeps its own problem's labels,
 * loss, lambda2, M, k, L and eigen shift. Call before the first mixed-precision solve of either
 * problem. Errors: CGL_E_INVAL (NULL argument; the same problem twice; different contexts; n, p
 * or the stored precision differ; the stored designs differ in any bit, compared on the device;
 * either already shares a design as a sharer, or the sharer has sharers; an engine of either
 * exists; more than 4 problems on one design). */
int cgl_problem_share_design(cgl_problem* owner, cgl_problem* sharer);
/* The Lipschitz constant in use. */
int cgl_problem_lipschitz(const cgl_problem* prob, double* L);
/* Eigen-perspective relaxation for least squares (App. D.2): with Q = X^T X - shift I and
 * lambda_eig = lambda2 + shift, later FP64-path solves minimise
 *   ||X beta - y||^2 - shift ||beta||^2 + 2 lambda_eig g_node(beta)
 * (between the perspective relaxation, shift = 0, and the k-sparse optimum) and certify it with
 *   ||y||^2 - beta^T Q beta - 2 lambda_eig g_node*((X^T y - Q beta) / lambda_eig)
 * evaluated at the iteration's momentum point. The bound is valid for 0 <= shift <=
 * lambda_min(X^T X), and the library accepts a shift only when it proves that: an FP64 Cholesky
 * factorisation of G - (shift + delta) I, G = X^T X formed in FP64 from the stored X, runs to
 * completion on the device (delta = 4 (n + p + 2) 2^-53 trace(G) covers the rounding of G and of
 * the factorisation; cgl_problem_eigen_shift finds the largest such shift). With n < p only
 * shift 0 is valid. L becomes 2 (1.002 lambda_max(X^T X) - shift).
 * Both paths solve the shifted problem: the FP64 path, and the batched engine (CGL_PREC_MIXED,
 * also through a server), whose FP64 certificate and bound witness (cgl_solve_batch_dual) then
 * follow the bound above at the certified iterate. cgl_certify rejects a shifted problem;
 * shift = 0 restores the perspective one.
 * Errors: CGL_E_INVAL for another loss, shift < 0, shift >= lambda_max, a shift the
 * factorisation does not prove, or while a server runs nodes of the problem. */
int cgl_problem_set_eigen(cgl_problem* prob, double shift);

/* The largest shift that the Cholesky test of cgl_problem_set_eigen proves, found by bisection
 * on [0, lambda_max] to a width of 1e-7 of the proved shift (one FP64 factorisation of the
 * p x p Gram matrix per step; 0 when n < p). Least squares only (CGL_E_INVAL otherwise). */
int cgl_problem_eigen_shift(cgl_problem* prob, double* shift);

/* Check a node against a problem's p and k on the host (no device work): the rules of
 * cgl_node above, tol >= 0, max_iter >= 1, check_every >= 1, a known precision, a finite warm
 * start (p doubles) and a non-NaN incumbent. CGL_OK or CGL_E_INVAL with the reason;
 * *infeasible (nullable) receives 1 when |Z1| > k (a valid node whose bound is +inf). */
int cgl_node_validate(const cgl_node* node, int64_t p, int32_t k, int32_t* infeasible);

/* ------------------------------------------------------------------ solves */

/* Solve one node relaxation (blocking). beta_out: NULL or p host doubles (the best-primal
 * iterate). res: one result. */
int cgl_solve_node(cgl_problem* prob, const cgl_node* node, double* beta_out, cgl_result* res);

/* Solve count nodes of one problem together (blocking). Nodes with precision CGL_PREC_MIXED
 * share batched MFMA products over X; nodes with CGL_PREC_F64 are solved one after another on
 * the plain path. beta_out: NULL or count x p host doubles. res: count results. Each result
 * equals the cgl_solve_node result of the same node within the tolerances. */
int cgl_solve_batch(cgl_problem* prob, const cgl_node* nodes, int32_t count, double* beta_out,
                    cgl_result* res);

/* cgl_solve_batch that also returns each bound's witness. For a node with CGL_PREC_MIXED, row i
 * of dual_beta_out (count x p host doubles, required) receives the iterate beta_D whose dual
 * point zeta = -grad f(X beta_D) gave res[i].lower_bound = D(zeta) (Sec. 3.4, evaluated in
 * FP64), so that a caller can re-evaluate the bound on its own. The rows of other nodes are set
 * to NaN: the F64 path takes its bound at the momentum point of Alg. 3, and infeasible nodes
 * have none. */
int cgl_solve_batch_dual(cgl_problem* prob, const cgl_node* nodes, int32_t count,
                         double* beta_out, cgl_result* res, double* dual_beta_out);

/* ------------------------------------------------------------------ certification utilities */

/* FP64 objective and weak-duality bound at a given beta (host, p doubles): primal = f(X beta) +
 * 2 lambda2 g_node(beta) (+inf outside the domain) and dual = D(zeta) with
 * zeta = -grad f(X beta) (Sec. 3.4). */
int cgl_certify(cgl_problem* prob, const cgl_node* node, const double* beta, double* primal,
                double* dual);

/* FP64 products with the problem's X on the device: trans = 0: out (n) = X v (v: p doubles);
 * trans = 1: out (p) = X^T v (v: n doubles). Host pointers. */
int cgl_problem_matvec(cgl_problem* prob, int32_t trans, const double* v, double* out);

/* The node prox on the device (Alg. 1 via the Moreau identity, node form): for each of count
 * rows w_i (host, count x p doubles), beta_i = prox_{g_node/rho}(w_i) with k' = k - |Z1_i|, and
 * gval_i = g_node(beta_i) (Alg. 2). nodes may be NULL (no fixed sets, only k used). beta_out:
 * count x p doubles; gval_out: NULL or count doubles. p <= 1048576 (above 16384 each vector is
 * streamed from device memory by its workgroup instead of held per thread; the standalone
 * workload of Sec. 4.1 runs to p = 102400). Errors (CGL_E_INVAL): NULL ctx, W or beta_out;
 * count < 0; p < 1 or p > 1048576; rho <= 0, M <= 0 or k < 0; an invalid node; 256 < k' < |F|. */
int cgl_prox_node_batch(cgl_ctx* ctx, double rho, double M, int32_t k, const cgl_node* nodes,
                        const double* W, int32_t count, int64_t p, double* beta_out,
                        double* gval_out);

/* cgl_prox_node_batch for callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same prox kernel for nodes
 * without fixed sets (k' = k, every coordinate free), with device buffers in and out and no
 * allocation, host copy or synchronisation inside the call.
 *   W: count x p device doubles (row-major); beta_out: count x p device doubles; gval_out: NULL
 *   or count device doubles (g(beta_i), Alg. 2).
 * The work is enqueued on the context's stream and the call returns without waiting: the
 * outputs are ready once that stream has been synchronised (or a later call on it ordered after
 * them). The per-vector states live in a fixed device array of 992 KiB per GPU (reserved
 * for the life of the process), shared by every call on that GPU and rewritten by each: calls
 * that overlap on one GPU (other streams or other contexts) race and must be serialised by the
 * caller.
 * Errors (CGL_E_INVAL, nothing enqueued): NULL ctx, W or beta_out; count < 0 or count > 4096;
 * p < 1 or p > 32768; rho <= 0, M <= 0 or k < 0; 256 < k < p. */
int cgl_prox_batch_noalloc(cgl_ctx* ctx, double rho, double M, int32_t k, const double* W,
                           int32_t count, int64_t p, double* beta_out, double* gval_out);

/* ------------------------------------------------------------------ serving */

/* A request loop over resident problems: submitted node relaxations are admitted into device
 * slots while slots and the HBM budget allow, advanced together (continuous batching: finished
 * slots are refilled between iteration chunks), and returned through poll.
 *   hbm_budget_bytes: upper bound on the device memory the server's slot state may use
 *                     (0 = no limit beyond max_slots); max_slots: slots per problem.
 * Each resident problem's engine runs on a HIP stream of its own. The HIP runtime maps a
 * process's streams onto GPU_MAX_HW_QUEUES hardware queues (4 by default), and kernels that
 * share a queue run in order: with more resident problems than that, set the variable to at
 * least the number of resident problems plus two before the process's first HIP call. */
int cgl_server_create(cgl_ctx* ctx, size_t hbm_budget_bytes, int32_t max_slots,
                      cgl_server** out);
/* Queue a node of prob (copied; never blocks). ticket receives its id. CGL_E_BUSY when the
 * queue is full. */
int cgl_server_submit(cgl_server* srv, cgl_problem* prob, const cgl_node* node,
                      uint64_t* ticket);
/* Advance the device work: resident engines (each on a stream of its own) and queued FP64-path
 * nodes that are idle start their next chunk of iterations (after retiring finished slots and
 * admitting queued nodes), then every engine or node whose chunk has completed is served; the
 * call waits for the first completion when none has happened yet. Then it returns up to max
 * finished results in completion order: tickets[i], res[i],
 * and, if betas is not NULL, the p_i doubles of result i's solution at betas + i * betas_stride
 * (the rest of that row is left as it was). A result whose p exceeds betas_stride stays queued:
 * the call returns the results before it (CGL_E_INVAL, with nothing taken, when it is the first
 * one). got receives the count. latency_s (nullable) receives submit-to-completion wall seconds
 * per result. */
int cgl_server_poll(cgl_server* srv, int32_t max, uint64_t* tickets, cgl_result* res,
                    double* betas, int64_t betas_stride, double* latency_s, int32_t* got);
/* Cancel a queued or running request; it is returned by poll with status CGL_CANCELLED. */
int cgl_server_cancel(cgl_server* srv, uint64_t ticket);
/* Counts: queued, running, finished-but-not-polled. */
int cgl_server_stats(cgl_server* srv, int32_t* queued, int32_t* running, int32_t* done);
int cgl_server_destroy(cgl_server* srv);

#ifdef __cplusplus
}
#endif

#endif /* CERTGLM_H */
