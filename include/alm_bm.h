/*
 * alm_bm.h -- C ABI of the MI355X (gfx950) ALM-BM library (libalmbm.so).
 *
 * The library computes the data-parallel hot path of the augmented Lagrangian
 * Burer-Monteiro method (ALM-BM) of arxiv 2505.15775 for semidefinite programs
 *
 *     (P)   minimise <C, X>  subject to  A(X) = b,  X PSD          (Sec. 1.2)
 *
 * on a factor R (n x r), X = R R^T, with the augmented Lagrangian
 *
 *     Lbar_sigma(R, y) = <C, RR^T> + <y, b - A(RR^T)> + sigma/2 ||A(RR^T) - b||^2
 *
 * (eq. AL-BM; the paper writes rho for sigma and F for R).
 *
 * Problem structure accepted
 *   cost        C = S + Diag(d) - j_coef * J, with S a sparse symmetric matrix
 *               holding only off-diagonal entries (both triangles), d a dense
 *               diagonal and J the all-ones matrix.  MaxCut (Sec. 6.1) uses
 *               C = -L/4: S_ij = w_ij/4, d_i = -sum_k w_ik/4, j_coef = 0.
 *   constraints ALM_BM_CONS_DIAG:  A_i = e_i e_i^T, m = n (X_ii = b_i).
 *               ALM_BM_CONS_TRACE_EDGES: A_0 = trace_coef * I and, for each
 *               edge e = {i, j} (i < j), A_{1+e} = (e_i e_j^T + e_j e_i^T)/2,
 *               so <A_{1+e}, X> = X_ij; m = n_edges + 1.  This is the entry
 *               constraint of the examples of Sec. 3.3 and Sec. 4.3 and the
 *               constraint set of the Lovasz-theta SDP.  The matrix completion
 *               SDP of Sec. 6 is this family with trace_coef = 0 (b_0 = 0),
 *               C = I/2 (d = 1/2, no S) on n = n1 + n2 rows and one edge
 *               (i, n1 + j) with b = M_ij per observed entry.
 *
 * Conventions (all entry points)
 *   - Every call returns alm_bm_status.  Nothing throws or aborts across the
 *     ABI.  Argument checks return ALM_BM_ERR_INVALID_ARG before any launch.
 *     alm_bm_last_error() gives a message for the last failing call on the
 *     calling thread.
 *   - Pointers named "device" are device memory owned by the caller; they must
 *     stay valid while the handle uses them (the problem arrays for the life of
 *     the handle).  Pointers named "host" are host memory.
 *   - R and G are row-major n x r arrays with row stride r, in the handle's
 *     storage precision (double, float or bfloat16).  y, b, Av and every scalar
 *     are double in every precision mode.
 *   - Indices are 0-based int32.
 *   - All work is enqueued on the given stream.  Calls that return host
 *     results synchronise it: alm_bm_solve, alm_bm_inner_solve,
 *     alm_bm_lanczos_min_eig and alm_bm_lanczos_block (their small
 *     eigensolves run on the host), alm_bm_kkt, alm_bm_autotune, alm_bm_batch_autotune and
 *     alm_bm_batch_solve;
 *     alm_bm_set_hub_threshold synchronises the device.
 *   - A handle is not thread-safe.  Calls that overlap on one handle race.
 *   - The handle owns its workspace, allocated in alm_bm_create and sized by the
 *     descriptor (r_max, lanczos_kmax, rank_block_max, lbfgs_memory_max,
 *     hub_min_degree; BF16 handles also reserve the float factor of the
 *     precision ladder).  No other call allocates device memory, except that
 *     alm_bm_solve, alm_bm_inner_solve and alm_bm_batch_solve instantiate HIP
 *     graphs of their inner loops (runtime-owned).
 */
#ifndef ALM_BM_H
#define ALM_BM_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  ALM_BM_OK = 0,
  ALM_BM_NOT_CONVERGED = 1,        /* solve: outputs valid, tolerance not met     */
  ALM_BM_ERR_INVALID_ARG = -1,     /* null pointer, bad size, r > r_max, ...      */
  ALM_BM_ERR_INVALID_PATTERN = -2, /* CSR / edge list malformed (validate = 1)    */
  ALM_BM_ERR_HIP = -3,             /* a HIP runtime call failed                   */
  ALM_BM_ERR_OOM = -4,             /* workspace allocation failed                 */
  ALM_BM_ERR_NUMERIC = -5,         /* NaN or Inf in a scalar the solve depends on */
  ALM_BM_ERR_UNSUPPORTED = -6      /* combination of options not implemented      */
} alm_bm_status;

typedef enum {
  ALM_BM_F64 = 0,  /* R, G stored and computed in double                       */
  ALM_BM_F32 = 1,  /* R, G and the sparse values in float, float accumulation   */
  ALM_BM_BF16 = 2  /* R, G stored as bfloat16 (round to nearest even), float
                      arithmetic and accumulation, float sparse values          */
} alm_bm_precision;

typedef enum {
  ALM_BM_CONS_DIAG = 0,
  ALM_BM_CONS_TRACE_EDGES = 1
} alm_bm_cons_kind;

typedef struct {
  int64_t n;                 /* matrix order                                         */
  /* cost C = S + Diag(diag) - j_coef * J                                              */
  int64_t nnz;               /* stored off-diagonal entries of S (both triangles)    */
  const int32_t* row_ptr;    /* device, n+1 (CSR); NULL when ell_width > 0 or nnz = 0 */
  const int32_t* col_idx;    /* device, nnz; within a row sorted ascending (CSR)     */
  const double* val;         /* device, nnz                                          */
  int32_t ell_width;         /* > 0: ELL layout, row i holds entries
                                [i*ell_width, (i+1)*ell_width) of col_idx/val; pad
                                with col = i and val = 0; nnz must be n*ell_width   */
  const double* diag;        /* device, n; NULL means d = 0                          */
  double j_coef;             /* coefficient of -J (0 for MaxCut, 1 for Lovasz theta) */
  /* constraints                                                                       */
  alm_bm_cons_kind cons_kind;
  int64_t m;                 /* n (DIAG) or n_edges + 1 (TRACE_EDGES)                */
  const double* b;           /* device, m                                            */
  double trace_coef;         /* TRACE_EDGES: A_0 = trace_coef * I                    */
  int64_t n_edges;           /* TRACE_EDGES                                          */
  const int32_t* edge_i;     /* device, n_edges; edges sorted by (i, j), i < j,      */
  const int32_t* edge_j;     /*   no duplicates; y[1+e] belongs to edge e            */
  /* storage                                                                           */
  alm_bm_precision precision;
  int32_t r_max;             /* largest rank any call will use (1..128)              */
  int32_t lanczos_kmax;      /* largest Lanczos basis (0 disables Lanczos; <= 512)   */
  int32_t validate;          /* 1: check CSR/ELL and edge list on create (D2H copy)  */
  /* workspace reserved by alm_bm_create for optional solve features (no later
     call allocates):                                                                  */
  int32_t rank_block_max;    /* largest alm_bm_options.rank_block (0 or 1: one-vector
                                rank steps only; up to 8: n x rank_block_max doubles) */
  int32_t lbfgs_memory_max;  /* largest alm_bm_options.lbfgs_memory (0: no L-BFGS;
                                1..8: DIAG family only, two rings of memory + 1
                                n x r_max vectors, float-sized for BF16 handles)     */
  int32_t hub_min_degree;    /* DIAG CSR costs: rows with more stored entries are hub
                                rows (0: twice the average row length, at least 32;
                                < 0: none).  alm_bm_set_hub_threshold can later
                                only choose thresholds with at most this many hubs */
} alm_bm_problem_desc;

typedef struct alm_bm_problem alm_bm_problem;

typedef enum { ALM_BM_STEP_EXACT = 0, ALM_BM_STEP_FIXED = 1 } alm_bm_step_rule;
typedef enum { ALM_BM_INNER_GD = 0, ALM_BM_INNER_LBFGS = 1 } alm_bm_inner_solver;
typedef enum { ALM_BM_RANK_ADAPT = 0, ALM_BM_RANK_FIXED = 1 } alm_bm_rank_policy;

/* Options of alm_bm_solve.  alm_bm_default_options() fills the defaults given
 * after each field; readings of points the paper leaves open are stated there. */
typedef struct {
  double eps_kkt;            /* 1e-6   stop when the relative KKT measure <= eps      */
  double sigma;              /* 1.0    penalty (fixed, as the input rho of Alg. 1)    */
  int32_t max_outer;         /* 1000                                                   */
  int32_t max_inner;         /* 500    gradient steps per subproblem                  */
  alm_bm_step_rule step_rule;/* EXACT  exact minimiser of the quartic Lbar(R - tG)    */
  double eta_fixed;          /* 1e-3   step for ALM_BM_STEP_FIXED                     */
  alm_bm_rank_policy rank_policy; /* ADAPT p = 1 rank step of Alg. 1                 */
  int32_t r_cap;             /* 0 -> min(r_max, floor((sqrt(8m+1)-1)/2))              */
  double tau_rank;           /* <= 0 -> eps_kkt (1 + ||C||_F)                        */
  int32_t expand_needs_inner;/* 0      1: expand only after an inner solve converged  */
  double inner_tol_scale;    /* 0.1    tol_k = max(eps/10, min(0.1, pinf, kappa tol)) */
  double inner_tol_decay;    /* 0.7    kappa                                           */
  int32_t lanczos_kmax;      /* 0 -> the handle's lanczos_kmax                        */
  double lanczos_tol_rel;    /* 0.1    Ritz residual <= 0.1 eps (1 + ||C||_F)         */
  uint64_t seed;             /* 1      Lanczos start vector                            */
  int32_t graph_unroll;      /* 8      inner iterations per captured HIP graph; 0 = no graph */
  int32_t verbose;           /* 0      1: one line per outer iteration on stderr      */
  double time_limit_s;       /* 0      > 0: stop (NOT_CONVERGED) after this wall time  */
  int32_t bf16_promote;      /* 1      BF16 handle: ladder to float storage when stalled */
  int32_t refresh_every;     /* 0 -> 32 (F64), 16 (F32), 8 (BF16): inner steps between
                                full sparse evaluations of C R; in between, C R is
                                carried as C R - t C G (1 = always recompute)      */
  int32_t lanczos_restarts;  /* 3      restarts from the Ritz vector while the Ritz
                                residual exceeds its tolerance                    */
  double sigma_edges;        /* 0      TRACE_EDGES: penalty of the edge rows (the trace
                                row keeps sigma); 0 -> sigma.  With tr X fixed the
                                entries are O(1/n) and the edge rows need a penalty
                                ~ n sigma to move their multipliers              */
  double sigma_growth;       /* 1      penalty schedule (off at 1): after an outer
                                iteration whose primal infeasibility did not fall
                                below pinf_reduction x the previous one, sigma (and
                                sigma_edges with it) is multiplied by sigma_growth,
                                up to sigma_max.  The rule of the SDPLR solver that
                                Sec. 2 cites; Alg. 1 keeps rho fixed               */
  double sigma_max;          /* 1e6    cap of the schedule                             */
  double pinf_reduction;     /* 0.25   required decrease of pinf per outer iteration  */
  int32_t rank_block;        /* 1      rank step directions (Alg. 1's negative-curvature
                                step): 1 = the closed-form one-vector step; 2..8
                                = the smallest Ritz vectors below
                                -tau_rank of a full Lanczos pass, S of the small PSD
                                subproblem, and the columns of V S^(1/2); at most the
                                handle's rank_block_max                            */
  int32_t resume_outer;      /* 0      resume a stopped solve: the outer iteration to
                                continue from (the stopped solve's result.outer),
                                with R, r and y as it returned them                */
  double resume_inner_tol;   /* 0      with resume_outer: the stopped solve's
                                result.inner_tol (<= 0: none)                      */
  double resume_pinf;        /* 0      with resume_outer: its result.pinf (<= 0: none);
                                with the three, an FP64 solve stopped by max_outer
                                and resumed repeats the uninterrupted one bitwise   */
  alm_bm_inner_solver inner_solver; /* GD  subproblem solver: gradient descent (eq. GD)
                                or L-BFGS (the solver of the SDPLR code Sec. 2 names;
                                DIAG family, needs lbfgs_memory_max >= lbfgs_memory),
                                both with the exact quartic line search           */
  int32_t lbfgs_memory;      /* 3      L-BFGS pairs kept (1..8)                       */
} alm_bm_options;

typedef struct {
  int32_t outer;             /* outer iterations run                                  */
  int64_t inner_total;       /* gradient steps over all outer iterations              */
  int32_t rank;              /* final rank                                            */
  int32_t expansions;        /* rank expansions taken                                 */
  double pobj;               /* <C, RR^T>                                             */
  double dobj;               /* b^T y                                                 */
  double pinf, dinf, gap, kkt; /* relative KKT terms (Sec. 6) at (RR^T, y)            */
  double lam_min;            /* lambda_min(C - A* y) estimate: the smaller of the Ritz
                                value and the Rayleigh quotient of RR^T, both upper
                                bounds; dinf is computed from it                    */
  double time_s;             /* wall time of the solve                                */
  double time_lanczos_s;     /* of which in Lanczos                                   */
  int32_t promoted_at_outer; /* BF16 ladder switch point (-1 = none)                  */
  double time_promoted_s;    /* wall time spent after the switch                       */
  double sigma_final;        /* penalty at the end (differs from sigma only with the
                                schedule)                                              */
  int32_t sigma_increases;   /* schedule steps taken                                   */
  double inner_tol;          /* tolerance of the last subproblem (for resume_inner_tol) */
  double lanczos_resid;      /* Ritz residual ||Z v - theta v|| of the Lanczos run
                                behind lam_min.  A solve returns ALM_BM_OK only when
                                the low end of the Ritz interval is dual feasible to
                                the tolerance, resid - theta <= eps_kkt (1 + ||C||_F),
                                and theta did not exceed the Rayleigh quotient
                                <Z, RR^T>/||R||_F^2 by more than the Lanczos
                                tolerance (else the Ritz value is not the bottom of
                                the spectrum and dinf is not certified)           */
} alm_bm_result;

/* --------------------------------------------------------------------------- */

/* Create a handle for one problem.  Validates sizes, allocates the workspace,
 * converts the sparse values to float in the F32/BF16 modes and, for
 * TRACE_EDGES, builds the symmetric adjacency with edge ids (host round trip).
 * stream: where set-up copies and kernels run; synchronised before return.     */
alm_bm_status alm_bm_create(const alm_bm_problem_desc* desc, hipStream_t stream,
                            alm_bm_problem** out);
alm_bm_status alm_bm_destroy(alm_bm_problem* prob);

/* Objective and gradient of eq. (AL-BM) at (R, y):
 *   f  = Lbar_sigma(R, y)                         (device, 1 double)
 *   G  = 2 (C - A*(w)) R,  w = y - sigma (A(RR^T) - b)   (device n x r, nullable)
 *   Av = A(RR^T)                                  (device m doubles, nullable)
 * The factor 2 is that of grad h(F) = 2 grad f(X) F (Sec. 4.2).
 * r: 1..r_max.  R device n x r.  y device m.                                    */
alm_bm_status alm_bm_objective_grad(alm_bm_problem* prob, int32_t r, const void* R,
                                    const double* y, double sigma, double* f, void* G,
                                    double* Av, hipStream_t stream);

/* alm_bm_objective_grad without a handle and without any device allocation,
 * for callers that cannot allocate: code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc.  desc (host) describes a DIAG
 * family problem in ALM_BM_F64 storage with j_coef = 0; only n, nnz, row_ptr,
 * col_idx, val, ell_width, diag, m and b are read (no validation of the
 * pattern, no hub rows).  r: 1..128.  R, y, f, G (nullable), Av (nullable):
 * device doubles, as for alm_bm_objective_grad.  The per-block partial sums
 * live in a static device array of the library, one per GPU (4096 x 15 doubles
 * plus one scalar block, about 0.5 MB, held until the process ends), whose
 * address is resolved on the first call on each device (the runtime then loads
 * the array's code object, a one-time set-up: make that first call outside
 * graph capture and before memory is budgeted); every call on one GPU
 * shares it, so calls that overlap on one GPU (other streams or threads) race,
 * while calls in order on one stream do not.  The stream must belong to the
 * current device.  Results equal those of alm_bm_objective_grad on a handle
 * with default tiles.  Errors: ALM_BM_ERR_INVALID_ARG (null pointer, n or r out
 * of range, inconsistent sizes), ALM_BM_ERR_UNSUPPORTED (TRACE_EDGES, F32 or
 * BF16, j_coef != 0).                                                          */
alm_bm_status alm_bm_objective_grad_noalloc(const alm_bm_problem_desc* desc, int32_t r, const double* R,
                                            const double* y, double sigma, double* f, double* G, double* Av,
                                            hipStream_t stream);

/* Cost product P = C X with C = S + Diag(d) (the sparse product that dominates
 * the gradient evaluation and the exact line search, Sec. 6): X device n x r in
 * the storage precision, P device n x r in the arithmetic precision (double for
 * F64, float for F32 and BF16), row-major, caller-owned; X and P must not
 * overlap.  xpx (device, 1 double, nullable) receives <X, C X>.  Requires
 * j_coef = 0 (ALM_BM_ERR_UNSUPPORTED otherwise).                                */
alm_bm_status alm_bm_cost_apply(alm_bm_problem* prob, int32_t r, const void* X, void* P,
                                double* xpx, hipStream_t stream);

/* Coefficients k[0..4] of phi(t) = Lbar_sigma(R - t G, y) = sum_k k[k] t^k
 * (device, 5 doubles) and the exact minimiser t* over t >= 0 (device, 1 double,
 * nullable; ties to the smallest t; 0 when phi is unbounded below).  G is any
 * direction of the same shape as R (the solve uses the gradient).               */
alm_bm_status alm_bm_line_search(alm_bm_problem* prob, int32_t r, const void* R,
                                 const void* G, const double* y, double sigma,
                                 double* coeffs, double* t_star, hipStream_t stream);

/* One gradient-descent step of eq. (GD) (Sec. 4.2) with the exact line search:
 * G = grad Lbar_sigma(R, y), t* = argmin_{t >= 0} Lbar_sigma(R - t G, y), then
 * R <- R - t* G in place.  f (device, 1 double, nullable) receives the objective
 * before the step, t (device, 1 double, nullable) the step, G (device n x r,
 * nullable: the handle's workspace is used) the gradient.  This is the body of
 * the inner loop of alm_bm_solve.                                              */
alm_bm_status alm_bm_gd_step(alm_bm_problem* prob, int32_t r, void* R, const double* y,
                             double sigma, double* f, double* t, void* G, hipStream_t stream);

/* Dual update of eq. (ALM): y <- y + sigma (b - Av) in place (device, m);
 * pinf = ||Av - b|| / (1 + ||b||) (device, 1 double, nullable), Sec. 6.           */
alm_bm_status alm_bm_dual_update(alm_bm_problem* prob, const double* Av, double sigma,
                                 double* y, double* pinf, hipStream_t stream);

/* Smallest eigenvalue of the dual slack Z(y) = C - A*(y) (Sec. 1.2) by Lanczos
 * with full FP64 reorthogonalisation (two classical Gram-Schmidt passes),
 * start vector drawn from `seed` by a counter-based generator.  Stops when the
 * Ritz residual ||Z v - theta v|| <= tol or after max_iter (<= lanczos_kmax)
 * steps; then restarts from the Ritz vector (up to 3 times) while the residual
 * exceeds tol.
 * theta, resid: device 1 double each; iters: device 1 int32, Lanczos steps summed
 * over restarts (all nullable except theta); v: device n doubles, unit Ritz
 * vector (nullable).  Synchronises stream.
 * theta is a Ritz value, hence an upper bound on lambda_min.                    */
alm_bm_status alm_bm_lanczos_min_eig(alm_bm_problem* prob, const double* y, int32_t max_iter,
                                     double tol, uint64_t seed, double* theta, double* v,
                                     double* resid, int32_t* iters, hipStream_t stream);

/* The q smallest eigenpairs of Z(y) (Sec. 5: the rank step of Alg. 1 uses the
 * negative ones) by block Lanczos: a block Krylov space span{V0, Z V0, ...} of
 * min(max_iter + 1, n) columns from q counter-based random start vectors (seed),
 * each new column orthogonalised against all earlier ones (two classical
 * Gram-Schmidt passes, FP64), then Rayleigh-Ritz on the projected matrix on the
 * host.  A block of q vectors captures an eigenvalue of multiplicity up to q,
 * which a single Krylov vector cannot.  q in 1..8; max_iter in 1..lanczos_kmax
 * and the basis must exceed q.
 * theta: host q doubles, ascending Ritz values (upper bounds on the q smallest
 * eigenvalues; NaN past the basis size); V: device n x q column-major, the unit
 * Ritz vectors (nullable when the handle's rank_block_max >= q); resid: host q
 * doubles ||Z v - theta v|| (nullable; one more product each); basis: host 1
 * int32, the basis size used (nullable).  Synchronises stream.                */
alm_bm_status alm_bm_lanczos_block(alm_bm_problem* prob, const double* y, int32_t q, int32_t max_iter,
                                   uint64_t seed, double* theta, double* V, double* resid, int32_t* basis,
                                   hipStream_t stream);

/* The inner loop of alm_bm_solve on its own: gradient descent with exact line
 * search on eq. (AL-BM) at fixed y from R (in place, device n x r), until
 * ||G||_F ||R||_F <= tol (1 + |<C, RR^T>|) or max_steps steps.  opts (host,
 * nullable): sigma, step_rule, eta_fixed, graph_unroll, refresh_every are used.
 * steps_done, stop_flag (1 tolerance met, 2 step limit), f_last (objective at
 * the final R): host, nullable.  Synchronous.                                  */
alm_bm_status alm_bm_inner_solve(alm_bm_problem* prob, const alm_bm_options* opts, int32_t r, void* R,
                                 const double* y, double tol, int32_t max_steps, int32_t* steps_done,
                                 int32_t* stop_flag, double* f_last, hipStream_t stream);

/* Full ALM-BM solve (Alg. 1, ALORA, with p = 1 rank adaptation).
 * R: device buffer of n x r_max elements; its first n*(*r) elements hold the
 * starting factor (row stride *r) and on return the final factor (row stride
 * the returned *r).  r: host in/out.  y: device m, in/out (start and final dual).
 * opts: host, NULL = defaults.  out: host, nullable.  Synchronous.
 * Returns ALM_BM_OK when the KKT measure met eps_kkt, ALM_BM_NOT_CONVERGED when
 * max_outer or the time limit ran out (outputs still valid).
 * A BF16 handle whose solve switched to float storage (bf16_promote,
 * out->promoted_at_outer >= 0) measured and certified its float factor; R
 * receives that factor rounded to BF16, whose row norms are off by up to about
 * 2^-8 relative, so A(RR^T) - b there can exceed the tolerance.  The float
 * factor itself is available from alm_bm_ladder_factor.                       */
alm_bm_status alm_bm_solve(alm_bm_problem* prob, const alm_bm_options* opts, void* R,
                           int32_t* r, double* y, alm_bm_result* out, hipStream_t stream);

/* Kernel tiling of this handle's row kernels.  variant picks an alternative
 * (lanes per row, columns per lane) tile for the same rank, 0..2 (0 = default);
 * row_blocks is the grid of the row kernels, a multiple of 8 in
 * [8, max_row_blocks] (0 = default).  Results stay deterministic for a fixed
 * choice; different choices sum in different orders.                          */
alm_bm_status alm_bm_set_tiles(alm_bm_problem* prob, int32_t variant, int32_t row_blocks);

/* Hub rows of a MaxCut-type (DIAG family) CSR cost, for skewed degree
 * distributions (power-law graphs, Sec. 6.1's MaxCut on general sparse C).  A
 * row with more than min_degree stored entries is a hub: before each sparse
 * product C X a kernel with one workgroup per hub sums that row's neighbour
 * rows with all of the workgroup's lanes, and the row kernels read the sum
 * instead of walking the row with one lane group.  min_degree: 0 = the
 * default (twice the average row length rounded up, at least 32), > 0 = that
 * threshold, < 0 = no hubs.  alm_bm_create applies desc.hub_min_degree and
 * reserves the hub list and sums (2 x hubs x r_max values per precision kept)
 * for exactly the hubs of that threshold; this call rewrites them in place
 * after a device synchronisation, allocates nothing, and returns
 * ALM_BM_ERR_INVALID_ARG for a threshold with more hubs than reserved (a
 * larger threshold never has more).  Not concurrently with other calls on
 * the handle.  hubs: host int32 out, nullable: the number of hub rows.  No
 * effect (0 hubs) for the TRACE_EDGES family or an ELL cost; rejected on a
 * batch.  Results differ from the hub-free pass only in summation order.     */
alm_bm_status alm_bm_set_hub_threshold(alm_bm_problem* prob, int32_t min_degree, int32_t* hubs);

/* The small PSD subproblem of the block rank step (Alg. 1, Sec. 5), host
 * only: minimise over S PSD (q x q, 1 <= q <= 8)
 *   sum_a theta_a S_aa + sigma/2 sum_{abcd} S_ab S_cd M4[pair(a,b), pair(c,d)]
 * where pair(a,b) numbers the pairs a <= b row-major (np = q(q+1)/2 of them)
 * and M4 (host, np x np row-major, symmetric) holds the penalty's quadratic
 * form of A(V S V^T) for orthonormal Ritz directions V of the slack with
 * Ritz values theta (host, q).  S: host out, q x q row-major.  This is the
 * solver alm_bm_solve uses with rank_block > 1; it needs no device.         */
alm_bm_status alm_bm_psd_step(int32_t q, const double* theta, const double* M4, double sigma, double* S);

/* The penalty's quadratic form of the block rank step (Alg. 1, Sec. 5): for q
 * orthonormal directions V (device, n x q column-major doubles, 1 <= q <=
 * the handle's rank_block_max), M4 (host out, np x np row-major, np =
 * q(q+1)/2, pairs a <= b numbered row-major) with
 *   M4[pair(a,b), pair(c,d)] = sum_i w_i A_i(v_a v_b^T) A_i(v_c v_d^T),
 * w_i = edge_weight on the edge rows of the TRACE_EDGES family (the ratio
 * sigma_edges / sigma inside a solve) and 1 on every other row; the trace row
 * contributes trace_coef^2 [a = b][c = d] (exact for orthonormal V).  This is
 * the M4 that alm_bm_psd_step takes.  Synchronises stream.                  */
alm_bm_status alm_bm_block_moments(alm_bm_problem* prob, int32_t q, const double* V, double edge_weight, double* M4,
                                   hipStream_t stream);

/* Autotuner: times reps objective/gradient passes at rank r for every
 * (variant, row_blocks) candidate with HIP events on `stream`, keeps the
 * fastest in the handle and returns it (host int32 each, nullable).  Uses the
 * handle's workspace as input (values do not affect the timing).              */
alm_bm_status alm_bm_autotune(alm_bm_problem* prob, int32_t r, int32_t reps, int32_t* variant,
                              int32_t* row_blocks, hipStream_t stream);

/* ---- batched solves ----------------------------------------------------------
 * Many independent problems (DIAG family, one storage precision) solved
 * together: the instances are concatenated block-diagonally on the device and
 * each launch of the method covers every instance still running (per-instance
 * step sizes, tolerances, stop flags, duals, Lanczos recurrences and ranks; the
 * inner loop of all instances is one captured HIP graph per chunk of steps).
 * At the interface the factors share one row width, rank_stride: instance q's
 * rows sit at rows [off_q, off_q + n_q) of one (sum n) x rank_stride array, its
 * first r_q columns used and the rest zero (zero columns stay exactly zero
 * under the gradient step, so the padded problem is the rank-r_q problem).
 * Inside a solve each instance is kept at its own padded width (the next tile
 * width at or above r_q) in its region of that array and is laid out back on
 * return.  Rank expansion fills the next zero column, up to rank_stride.       */
typedef struct alm_bm_batch alm_bm_batch;

/* descs: host array of count descriptors (device arrays as for alm_bm_create,
 * copied into the batch, so they may be freed afterwards).  1 <= count <= 4096.
 * DIAG family, one precision.  The largest lbfgs_memory_max among the
 * descriptors reserves the L-BFGS rings of the batch ((sum n) x rank_stride
 * elements per slot) and one L-BFGS state per instance; rank_block_max and
 * hub_min_degree do not apply to batches.                                     */
alm_bm_status alm_bm_batch_create(int32_t count, const alm_bm_problem_desc* descs, int32_t rank_stride,
                                  hipStream_t stream, alm_bm_batch** out);
alm_bm_status alm_bm_batch_destroy(alm_bm_batch* batch);
/* offsets: host count+1 int64 (row offsets of the instances; offsets[count] = sum n). */
alm_bm_status alm_bm_batch_offsets(const alm_bm_batch* batch, int64_t* offsets);
/* R: device (sum n) x rank_stride in the storage precision (in/out); r: host
 * count ranks (in/out); y: device sum n doubles (in/out); results, status: host
 * count each (nullable).  opts as for alm_bm_solve (graph_unroll must be >= 1;
 * inner_solver L-BFGS needs lbfgs_memory <= the reserved memory; the penalty
 * schedule, rank_block > 1 and resume are for single solves: UNSUPPORTED).
 * Returns ALM_BM_OK when every instance met eps_kkt, else NOT_CONVERGED.        */
alm_bm_status alm_bm_batch_solve(alm_bm_batch* batch, const alm_bm_options* opts, void* R, int32_t* r,
                                 double* y, alm_bm_result* results, int32_t* status, hipStream_t stream);
/* Tile choice of a batch, the batched counterpart of alm_bm_autotune: for every
 * width a batched solve can give an instance (4, 8, 16, ... up to rank_stride),
 * times reps objective/gradient passes over all instances at that width with
 * each tile variant and keeps the fastest (another variant must beat variant 0
 * by 3 %, so that timing noise does not flip the choice); later alm_bm_batch_solve calls
 * launch that variant for that width (untuned widths use variant 0).  The
 * variants sum each row in a different order, so two handles tuned apart may
 * round differently; solves on one handle stay deterministic.  widths, variants:
 * host arrays of ALM_BM_BATCH_TUNE_MAX (nullable), receiving the table in
 * increasing width; n_out: its length (nullable).  reps >= 1.  Overwrites the
 * handle's scratch and its last objective pass; synchronises stream.          */
#define ALM_BM_BATCH_TUNE_MAX 16
alm_bm_status alm_bm_batch_autotune(alm_bm_batch* batch, int32_t reps, int32_t* widths, int32_t* variants,
                                    int32_t* n_out, hipStream_t stream);

/* The float factor of the last alm_bm_solve on this BF16 handle that switched to
 * float storage (the point its KKT measure and status refer to).  r: the rank
 * that solve returned; R: device n x r floats, row-major (caller-owned).  Valid
 * until the next alm_bm_solve on the handle; INVALID_ARG when the last solve did
 * not switch or r differs.  Enqueued on stream.                               */
alm_bm_status alm_bm_ladder_factor(alm_bm_problem* prob, int32_t r, float* R, hipStream_t stream);

/* Relative KKT measure of Sec. 6 at (RR^T, y) with lambda_min supplied by the
 * caller (host double); kkt_out: host array of 6 doubles
 * {pinf, dinf, gap, kkt, pobj, dobj}.  Synchronises stream.                      */
alm_bm_status alm_bm_kkt(alm_bm_problem* prob, int32_t r, const void* R, const double* y,
                         double lam_min, double* kkt_out, hipStream_t stream);

/* ---- learned warm start (MaxCut-type problems, DIAG family) -----------------
 * A per-vertex model proposes the initial dual y0 and a pooled-feature ridge
 * model the initial rank r0 (Alg. 1 starts from y = 0; the warm start is an
 * addition).  Features of vertex i, from the cost C = S + Diag(d):
 *   0 log(1 + deg_i)   1 sum_j |S_ij|   2 sum_j S_ij   3 d_i
 *   4 d_i - sum_j |S_ij| (Gershgorin bound of a dual-feasible y_i)
 *   5 mean and 6 max of log(1 + deg_j) over the neighbours j, 7 mean of their
 *   feature 1.
 * MLP: n_in -> h -> h -> 1, ReLU, FP32, inputs standardised inside the
 * kernels as (x - mu) * inv_sd; parameters flattened as W1[n_in][h], b1[h],
 * W2[h][h], b2[h], W3[h], b3 (alm_bm_ws_param_count floats).  h in {16,32,64},
 * n_in <= 8.                                                                    */
#define ALM_BM_WS_NFEAT 8
/* feats: device n x 8 float (row-major); scratch: device n floats.  Handle must
 * be DIAG family.                                                               */
alm_bm_status alm_bm_ws_features(alm_bm_problem* prob, float* feats, float* scratch, hipStream_t stream);
/* out[k] = mean over rows of feats[:, k] (device 8 doubles); n rows; work:
 * device 512 doubles.                                                           */
alm_bm_status alm_bm_ws_pool(const float* feats, int64_t n, double* out, double* work, hipStream_t stream);
int64_t alm_bm_ws_param_count(int32_t n_in, int32_t h);
/* Floats of workspace alm_bm_ws_loss_grad needs for `nblocks` blocks.          */
int64_t alm_bm_ws_work_size(int32_t n_in, int32_t h, int32_t nblocks);
/* out (device n doubles) = MLP(X) for X device n x n_in float.                 */
alm_bm_status alm_bm_ws_forward(const float* params, int32_t n_in, int32_t h, const float* mu,
                                const float* inv_sd, int64_t n, const float* X, double* out,
                                hipStream_t stream);
/* Mean squared error (1/n) sum (MLP(x_v) - t_v)^2 into *loss (device double)
 * and its gradient into grad (device, param_count floats), deterministic for a
 * fixed nblocks (1..4096).  work: device, alm_bm_ws_work_size floats.          */
alm_bm_status alm_bm_ws_loss_grad(const float* params, int32_t n_in, int32_t h, const float* mu,
                                  const float* inv_sd, int64_t n, const float* X, const float* target,
                                  float* grad, double* loss, float* work, int32_t nblocks,
                                  hipStream_t stream);
/* Adam (Kingma & Ba 2015) on count parameters, bias corrections for `step` >= 1.
 * params, grad, m, v: device floats.                                             */
alm_bm_status alm_bm_ws_adam(float* params, const float* grad, float* m, float* v, int32_t count,
                             float lr, float beta1, float beta2, float eps, int32_t step,
                             hipStream_t stream);
/* Ridge regression on the host: coef (p+1 doubles, last = intercept) minimising
 * sum_k (x_k . coef[0:p] + coef[p] - t_k)^2 + lambda ||coef[0:p]||^2 for the
 * rows x_k of X (host k x p, row-major), by the normal equations.              */
alm_bm_status alm_bm_ws_ridge_fit(const double* X, const double* t, int32_t k, int32_t p, double lambda,
                                  double* coef);

/* ---- measurement ------------------------------------------------------------
 * Random-row gather probe, the access pattern that bounds the sparse cost
 * product (each stored entry of C gathers one row of the factor): reads rows
 * idx[0..count) (each row_bytes = 8, 16, 32, 64, 128 or 256 bytes) of table
 * (device, rows x row_bytes bytes, 8-byte aligned) and writes per-thread sums
 * to out (device, alm_bm_gather_probe_out_size() floats) so no load is dead.
 * idx: device int32, each in [0, rows) (not checked).  Enqueued on stream;
 * time it with events to get the chip's gathered rows per second.           */
int64_t alm_bm_gather_probe_out_size(void);
alm_bm_status alm_bm_gather_probe(const void* table, int64_t rows, int32_t row_bytes, const int32_t* idx,
                                  int64_t count, float* out, hipStream_t stream);

void alm_bm_default_options(alm_bm_options* opts);
const char* alm_bm_last_error(void);

/* sizeof(alm_bm_problem_desc), sizeof(alm_bm_options), sizeof(alm_bm_result)
 * into out[0..3) (host), so that bindings can check their struct mirrors.       */
void alm_bm_abi_sizes(int64_t* out);

/* Host helper: the MaxCut cost of Sec. 6.1, C = -L/4, as CSR + diagonal from an
 * undirected edge list (host arrays).  ei[k] != ej[k]; duplicates are summed.
 * Outputs (host, caller-allocated): row_ptr n+1, col_idx 2M, val 2M, diag n;
 * columns sorted ascending within each row.  *nnz_out receives the entry count
 * (2M minus merged duplicates).                                                  */
alm_bm_status alm_bm_maxcut_cost_host(int64_t n, int64_t m_edges, const int32_t* ei,
                                      const int32_t* ej, const double* w, int32_t* row_ptr,
                                      int32_t* col_idx, double* val, double* diag,
                                      int64_t* nnz_out);

#ifdef __cplusplus
}
#endif

#endif /* ALM_BM_H */
