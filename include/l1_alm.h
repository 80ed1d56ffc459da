/*
 * l1_alm.h -- C ABI of libl1alm, batched augmented-Lagrangian l1 solvers for
 * AMD Instinct MI355X (gfx950).
 *
 * Problems (Sec. I of Yang, Zhou, Ganesh, Sastry, Ma, "Fast l1-minimization
 * algorithms for robust face recognition"):
 *   (P1)        min ||x||_1                      s.t. b = A x            eq. (l1)
 *   (P_{1,2})   min ||x||_1                      s.t. ||b - A x||_2 <= eps  eq. (l1-l2)
 *   (QP_lambda) min 1/2 ||b - A x||_2^2 + lambda ||x||_1                eq. (Lagrangian)
 * and the cross-and-bouquet (CAB) form of (P1) (Sec. II-A, eq. (CAB)):
 *               min ||w||_1  s.t. b = [B, I] w,  w = [x; e].
 * Methods: the dual ALM (DALM, Sec. V-B, Algorithm 2) and the primal ALM
 * (PALM, Sec. V-A, eq. (alm) and Algorithm 1, FISTA inner solver).
 *
 * Conventions for every entry point
 *   - Matrices are column-major FP32 with an explicit leading dimension.  A
 *     batch of N right-hand sides is an m x N matrix: one column per instance.
 *   - Every array argument is a DEVICE pointer on the current HIP device,
 *     owned by the caller; the library never keeps a caller pointer past the
 *     call that received it.
 *   - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *     Calls enqueue work on it; outputs are valid after the stream is
 *     synchronised.  l1_alm_solve synchronises `stream` itself a few times per
 *     solve to read the number of still-active instances.
 *   - Return value: 0 on success or a negative L1_E* code; the message of the
 *     last failure on the calling thread is returned by l1_alm_last_error().
 *   - Per-instance outcomes are not errors: they are reported in `status`.
 *   - One solve at a time per plan; a plan may move between host threads
 *     only with external locking.
 */
#ifndef L1_ALM_H_
#define L1_ALM_H_

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define L1_OK          0
#define L1_EINVAL     -1   /* bad size, leading dimension, NULL pointer or option   */
#define L1_ENOTSPD    -2   /* FP64 Cholesky met a pivot <= 0 (dependent rows of A)   */
#define L1_ENOMEM     -3   /* device allocation failed                              */
#define L1_EHIP       -4   /* HIP runtime error; message in l1_alm_last_error()     */
#define L1_ENODEVICE  -5   /* no gfx950 device visible                              */
#define L1_ENOTAPE    -6   /* l1_alm_backward without a recorded fixed-count solve   */

/* per-instance status */
#define L1_CONVERGED   0
#define L1_MAXITER     1
#define L1_NONFINITE   2
/* L1_DIVERGED: the iterate left every bounded region the optimum can lie
 * in: ||w_k||_2 > div_factor * sqrt(m) * ||b||_2 (desc.div_factor, default
 * 1e6).  For (P1) on a cross-and-bouquet matrix every optimum satisfies
 * ||w*||_2 <= ||w*||_1 <= ||b||_1 <= sqrt(m) ||b||_2 (w = [0; b] is
 * feasible), so an iterate that far out is not converging.  The test runs
 * with the stopping test (never in fixed-count solves); the exact DALM
 * iterates stay on the affine set A w = b and do not reach it in practice,
 * the one-CG-step variant and PALM with a growing xi can.               */
#define L1_DIVERGED    3

typedef enum { L1_P1 = 0, L1_P12 = 1, L1_QPLAMBDA = 2 } l1_problem;
typedef enum { L1_DENSE = 0, L1_CAB = 1 } l1_structure;
/* L1_DALM_CG1: DALM with the y-step replaced by one conjugate-gradient step
 * from the current y (the cheaper heuristic of Sec. V-B, which the paper
 * reports to work on random Gaussian dictionaries but not on face
 * dictionaries).  Builds no inverse; per iteration two FP32 products, A u
 * and A^T g.  (P1) only, dense or cross-and-bouquet, L1_FP32 only; same
 * stopping test, beta default and outputs as L1_DALM; no warm start.      */
typedef enum { L1_DALM = 0, L1_PALM = 1, L1_DALM_CG1 = 2 } l1_method;
/* Arithmetic of the per-iteration matrix products.  State, elementwise
 * updates and accumulation are FP32 in every mode; the operator is rounded
 * from FP64 once per plan.
 *   L1_FP32        FP32 MFMA products.
 *   L1_BF16_REFINE BF16 MFMA products until an instance's relative change and
 *                  gap are both <= refine_switch, or for 2000 iterations,
 *                  then split-BF16 products (B = B_hi + B_lo,
 *                  u = u_hi + u_lo; hi*hi + hi*lo + lo*hi with FP32
 *                  accumulation, ~16 significant bits) until convergence.
 *                  With the FP32 refresh of the operand's reference point
 *                  (batches of more than 64 instances), BF16 iterations
 *                  progress as fast as split ones until BF16 rounding holds
 *                  the gap near 1e-4 relative, so the default threshold
 *                  there is low (1e-4) and the 2000-iteration bound usually
 *                  ends the phase; smaller batches default to 3e-3, and
 *                  problems that converge in a few hundred iterations hand
 *                  over sooner with a larger refine_switch.  An instance
 *                  can only be declared converged in the split phase.
 *   L1_BF16X3      split-BF16 products for every iteration.
 * PALM runs its FISTA products (with A^T A) in split BF16 under either BF16
 * mode, and its A x / A^T c products in FP32.                               */
typedef enum { L1_FP32 = 0, L1_BF16_REFINE = 1, L1_BF16X3 = 2 } l1_precision;

typedef struct l1_alm_plan_s* l1_alm_plan_t;   /* opaque, owned by the library */

typedef struct {
  int m;                 /* rows of the dictionary (length of b)                     */
  int n_dict;            /* columns of the dictionary (B for CAB, A otherwise)       */
  int lda;               /* leading dimension of the dictionary passed to the plan   */
  int problem;           /* l1_problem                                               */
  int structure;         /* l1_structure; L1_CAB: the caller passes B, A = [B, I]    */
  int method;            /* l1_method                                                */
  int precision;         /* l1_precision                                             */
  int max_batch;         /* upper bound on N for every solve with this plan (>= 1)   */
  double lambda;         /* QP_lambda weight (> 0); ignored otherwise                */
  double beta;           /* DALM penalty.  <= 0: per instance beta0 = ||b||_1 / m, and
                            for L1_CAB beta0 / 16 (batches of more than 64
                            instances) or beta0 / 8 (smaller L1_FP32 batches).
                            Required (> 0) for DALM on QP_lambda, where it
                            enters the factor.                                       */
  double xi;             /* PALM penalty.  <= 0: per instance 2 m / ||b||_1 (Sec. V-A) */
  double xi_growth;      /* PALM: xi <- xi * xi_growth after each outer step (<= 0 -> 1) */
  int max_inner;         /* PALM: cap on FISTA steps per outer step (<= 0 -> 100)     */
  double tol_inner;      /* PALM: FISTA relative-change tolerance (<= 0 -> solve tol) */
  double refine_switch;  /* L1_BF16_REFINE: switch threshold (<= 0 -> 1e-4, or 3e-3 for
                            batches of at most 64 instances)                         */
  int record_tape;       /* 1: fixed-count DALM solves keep checkpoints for backward */
  int checkpoint_every;  /* checkpoint spacing in iterations (<= 0 -> 10)            */
  int time_kernels;      /* 1: time the DALM iteration loop with HIP events on the
                            solve stream (see l1_alm_last_stats)                    */
  double div_factor;     /* L1_DIVERGED threshold factor (<= 0 -> 1e6)               */
  int iteration_form;    /* L1_DALM on L1_CAB (P1) with n_dict < m, or on L1_DENSE with
                            m < n_dict: 0 automatic, 1 the dense operator only, 2 the
                            structured form whenever it applies ("Iteration forms") */
} l1_alm_desc;

/* Iteration forms of L1_DALM on the cross-and-bouquet (P1).  Sec. V-B makes
 * the y-step (A A^T)^{-1} applied to a vector; with A = [B, I] the Woodbury
 * identity gives (B B^T + I)^{-1} = I - B K^{-1} B^T, K = I + B^T B.  The
 * dense form multiplies u by P = A^T (A A^T)^{-1} A (n x n) every iteration.
 * The structured form takes the first n_dict rows of P u (an n_dict x n
 * product), forms q = u_x - (P u)_x = K^{-1} (u_x - B^T u_e), and then
 * (P u)_e = u_e + B q (an m x n_dict product): 2 n_dict (n + m) flops and
 * operator bytes per instance instead of 2 n^2, in two launches instead of
 * one.  Both forms give the same iterates up to rounding, but the second
 * product carries the rounding of the first through B (||B|| ~ 30 on face
 * dictionaries).  It runs BF16 and FP32 tiles (split-BF16 tiles stay dense:
 * their 16 bits would miss the 1e-4 accuracy of the converged solution).
 * Automatic mode uses it for L1_FP32 plans while the unfinished instances
 * span at least 16 column tiles of 64 (the products, not the per-launch
 * latency, then set the time; the last instances converge densely, since
 * the amplified rounding can hold the relative change of w above the
 * stopping threshold) and when the structured products cost at most 0.8 of
 * the dense one.  On a dense dictionary with m < n_dict the y-step's factor
 * is applied the same way: t = (A A^T + shift I)^{-1} A u (an m x n_dict
 * product), then v = A^T t + c (n_dict x m): 4 m n_dict instead of
 * 2 n_dict^2, under the same automatic rule (A^T spreads the first
 * product's rounding by ||A||, 3 for a Gaussian 2000 x 8000 dictionary).
 * The tail of few instances, the FP32 refresh of the operand's reference
 * point and recorded tapes use the dense form.                              */

/* Build a plan for the dictionary A_dev (m x n_dict, column-major, leading
 * dimension desc->lda >= m).
 *   DALM: forms, on the GPU in FP64, the Gram matrix of the full matrix
 *   (A A^T, B B^T + I for CAB, A A^T + I for the P_{1,2} splitting, plus
 *   (lambda/beta) I for QP_lambda), its Cholesky factor (Sec. V-B: the
 *   y-step "directly uses" the inverse) and from it the operators the
 *   iteration applies; FP64 is used only here and in l1_alm_kkt.
 *   PALM: forms A^T A in FP64 and L = ||A^T A||_2 by FP64 power iteration
 *   (the Lipschitz constant of Sec. IV-A used in Algorithm 1).
 * Returns L1_ENOTSPD when the Gram matrix is not positive definite, L1_EINVAL
 * for an unsupported combination (QP_lambda or P_{1,2} with L1_CAB).
 * The plan copies A; the caller may free A_dev after the call returns.   */
int l1_alm_plan(const l1_alm_desc* desc, const float* A_dev, void* stream,
                l1_alm_plan_t* out);

/* Solve N instances (columns of b_dev, m x N, leading dimension ldb >= m).
 *   eps_dev   P_{1,2}: N radii (device); NULL otherwise.
 *   pen_dev   N per-instance penalties (device): beta for DALM, xi for PALM,
 *             held constant for the whole solve; NULL takes desc.beta /
 *             desc.xi, or the per-instance default when that is <= 0.  An
 *             entry that is not positive and finite falls back to the
 *             default of its instance.  Must be NULL for DALM on
 *             QP_lambda (beta enters the factor there).
 *   tol       stopping tolerance: an instance stops after iteration k when
 *             ||w_k - w_{k-1}|| <= tol ||w_k|| and the complementarity gap of
 *             the l1 block | ||w||_1 - w^T A^T y | <= tol ||w||_1 (DALM), or
 *             when the relative change and the relative primal residual
 *             ||b - A x - e|| / ||b|| are both <= tol (PALM outer loop).
 *             For DALM the test uses max(tol, floor) with the floor of the
 *             products' arithmetic (FP32 2e-6, split BF16 4e-6).
 *   max_iter  > 0: iteration cap (DALM iterations / PALM outer steps);
 *             < 0: run exactly -max_iter iterations with no stopping test
 *             (DALM: the unrolled map used by l1_alm_backward; PALM: exactly
 *             -max_iter outer steps of exactly desc.max_inner FISTA steps).
 *             PALM ignores w0_dev / y0_dev (must be NULL) and writes no y.
 *   w0_dev, y0_dev  DALM warm start (n_full x N with ld n_full, m x N with
 *             ld m), or NULL for w0 = 0, y0 = 0 (Algorithm 2 input).
 *   x_dev     n_dict x N output, leading dimension ldx >= n_dict.
 *   e_dev     m x N output (ld lde >= m): the e-block of w for CAB, the
 *             split residual block for P_{1,2} (and QP_lambda under PALM);
 *             may be NULL.
 *   y_dev     m x N dual output (DALM; ld ldy >= m) or NULL.
 *   iters_dev, status_dev  N ints each (may be NULL).
 * n_full = n_dict + m for CAB and P_{1,2}, n_dict otherwise.             */
int l1_alm_solve(l1_alm_plan_t plan, const float* b_dev, int ldb, int N,
                 const float* eps_dev, const float* pen_dev, float tol, int max_iter,
                 const float* w0_dev, const float* y0_dev,
                 float* x_dev, int ldx, float* e_dev, int lde,
                 float* y_dev, int ldy, int* iters_dev, int* status_dev,
                 void* stream);

/* Reverse-mode gradient of the last recorded fixed-count CAB DALM solve
 * (max_iter < 0, desc.record_tape = 1): given adjoints gx (n_dict x N, ld
 * n_dict) and ge (m x N, ld m) of its outputs x and e, writes
 * gb (m x N, ld m, overwritten) = d<gx,x> + <ge,e> / d b and ADDS the
 * gradient with respect to the dictionary into gA (m x n_dict, ld m).
 * The iterations are recomputed segment by segment from checkpoints kept
 * every desc.checkpoint_every iterations.  beta is held constant at the
 * values the recorded solve used (pen_dev, or the default computed from
 * b): the result is the gradient of the map with beta fixed.
 * Returns L1_ENOTAPE if no tape was recorded.                            */
int l1_alm_backward(l1_alm_plan_t plan, const float* gx_dev, const float* ge_dev,
                    float* gb_dev, float* gA_dev, void* stream);

/* FP64 optimality report for N solutions (the LP duality pair of Sec. III-A
 * and V-B; for QP_lambda the optimality condition of Sec. III-B).  Writes
 * report_dev[4*j + {0,1,2,3}] = {relative primal residual, dual infeasibility
 * max(||A^T y||_inf - 1, 0), sign disagreement on the support, relative
 * gap} for instance j.  Arguments as in l1_alm_solve; e_dev / y_dev may be
 * NULL when the problem has no such block (y is not used for QP_lambda).
 * The residual b - A x (- e) and A^T u are formed as FP64 matrix-core GEMMs
 * over the batch; the first call on a plan allocates their operands (the
 * dictionary in FP64 and workspaces, 8 (m n_dict + (2 n_dict + m) max_batch)
 * bytes), held until l1_alm_destroy.  l1_alm_kkt_noalloc computes the same
 * report without a plan or any allocation.                               */
int l1_alm_kkt(l1_alm_plan_t plan, const float* b_dev, int ldb, int N,
               const float* eps_dev, const float* x_dev, int ldx,
               const float* e_dev, int lde, const float* y_dev, int ldy,
               double* report_dev, void* stream);

/* Statistics of the last l1_alm_solve on this plan; writes min(n, 14)
 * doubles to out (host memory):
 *   [0..2]  column tiles (64 instances) of the per-iteration product that
 *           had work, summed over the iterations (an iteration of the
 *           structured form counts once), by the arithmetic of the tile:
 *           FP32, BF16, split BF16
 *   [3..5]  instances summed over those tiles and launches, by arithmetic
 *   [6]     DALM, desc.time_kernels = 1: duration (ms) of the iteration loop,
 *           from HIP events on the solve stream around every block of 16
 *           iteration launches (with their compaction); else 0
 *   [7]     number of iterations inside those blocks
 *   [8]     iterations run (the largest per-instance count; PALM: outer steps)
 *   [9]     wall time of the call on the host (ms)
 *   [10]    one-time plan construction time (ms, host wall clock)
 *   [11]    PALM: FISTA product launches issued (summed over outer steps)
 *   [12]    the part of [3..5] that ran in the structured form
 *   [13]    reserved (0)
 * The tolerance floors used by the stopping test are FP32 2e-6 and split
 * BF16 4e-6 (the level where rounding noise stalls the test).             */
int l1_alm_last_stats(l1_alm_plan_t plan, double* out, int n);

/* Launch shape of the DALM iteration product.  When few instances are
 * active the product's K range is split over 1..L1_KSPLIT_MAX workgroups per
 * output tile (a second launch adds the parts).  By default the number of
 * parts comes from a heuristic (enough workgroups for the device); a table
 * indexed by the number of active 64-instance column tiles t = 1..n
 * (n <= L1_KSPLIT_TILES) replaces it: ks_by_tiles[t - 1] parts, 0 = keep the
 * heuristic for that t.  The table is part of the plan and persists until
 * set again (n = 0 clears it).  Errors: L1_EINVAL for a NULL plan, n outside
 * [0, L1_KSPLIT_TILES] or an entry outside [0, L1_KSPLIT_MAX].            */
#define L1_KSPLIT_TILES 8
#define L1_KSPLIT_MAX 4
int l1_alm_set_ksplit(l1_alm_plan_t plan, const int* ks_by_tiles, int n);

/* Autotuner of that table for a DALM plan: for t = 2 .. min(L1_KSPLIT_TILES,
 * max_batch / 64) it times fixed-count solves of t * 64 synthetic right-hand
 * sides (`iters` iterations each, median of 3, HIP events on `stream`) for
 * every split 1..L1_KSPLIT_MAX, keeps the fastest in the plan and writes the
 * table (n entries, t = 1..n) to ks_out (host memory).  Entry 1 (one active
 * column tile) stays 0 where the tail kernel can take over the last
 * instances (it uses the heuristic's split); for operators too large for the
 * tail kernel (more than 2048 padded columns) t = 1 is tuned as well.  The timings run in the plan's first arithmetic (BF16 for
 * L1_BF16_REFINE).  Allocates and frees its own device buffers; the solve
 * workspace of the plan is overwritten.  Errors: L1_EINVAL for a non-DALM or
 * (P1,2) plan, iters outside [16, 4096] or a bad n.                        */
int l1_alm_tune_ksplit(l1_alm_plan_t plan, int iters, int* ks_out, int n, void* stream);

/* The recognition criterion of the face experiments (Sec. VI-B), applied to
 * N representations x (n_dict x N, column-major, ld ldx >= n_dict) of test
 * vectors over a dictionary whose columns are grouped by subject: subject i
 * owns columns class_ptr[i] .. class_ptr[i+1]-1 (class_ptr: C + 1 ints,
 * non-decreasing, class_ptr[0] = 0, class_ptr[C] = n_dict; ranges outside
 * that are clamped to the columns, a decreasing one counts as empty).
 * Writes, for instance j:
 *   mass_dev[i + C*j]  ||delta_i(x_j)||_1, the l1 mass of subject i's
 *                      coefficients (FP32; may be NULL)
 *   label_dev[j]       the subject of largest mass (the lowest index among
 *                      equal masses); -1 when x_j = 0
 *   score_dev[j]       its sparsity concentration index
 *                      (C * mass / ||x_j||_1 - 1) / (C - 1); 0 when x_j = 0
 * Masses and the norm are summed in FP64 in a fixed order, so the result is
 * reproducible and the label is decided in FP64.  For the cross-and-bouquet
 * form pass x only (the e block is not a subject).  Needs no plan.
 * Errors: L1_EINVAL for N < 0, n_dict < 1, ldx < n_dict, C outside
 * [2, L1_CLASSIFY_MAX_SUBJECTS] or a NULL x / class_ptr / label / score.   */
#define L1_CLASSIFY_MAX_SUBJECTS 4096
int l1_alm_classify(const float* x_dev, int ldx, int n_dict, int N, const int* class_ptr_dev,
                    int C, float* mass_dev, int* label_dev, float* score_dev, void* stream);

/* The residual rule of the sparse-representation classifier the paper
 * builds on (Sec. I; the cross-and-bouquet model b = A x + e of Sec. II-A):
 * for instance j and subject i (owning columns class_ptr[i] ..
 * class_ptr[i+1]-1 of A, with the clamping rules of l1_alm_classify)
 *   res_dev[i + C*j] = ||b_j - e_j - A delta_i(x_j)||_2      (FP32; may be NULL)
 *   label_dev[j]     = argmin_i res (the lowest i among equal residuals)
 * A_dev: m x n_dict column-major (leading dimension lda), the dictionary of
 * the solve (B for the cross-and-bouquet form); x_dev: n_dict x N (ldx);
 * e_dev: m x N (lde), or NULL for e = 0; b_dev: m x N (ldb).  Every sum is
 * formed in FP64 from the FP32 inputs in a fixed order, so the residuals
 * are reproducible and the label is decided in FP64.  Device buffers owned
 * by the caller; asynchronous on `stream`; needs no plan.
 * Errors: L1_EINVAL for N < 0, m or n_dict < 1, a leading dimension below
 * its row count, C outside [2, L1_CLASSIFY_MAX_SUBJECTS] or a NULL A, x, b,
 * class_ptr or label.                                                      */
int l1_alm_class_residuals(const float* A_dev, int m, int n_dict, int lda, const float* x_dev, int ldx,
                           const float* e_dev, int lde, const float* b_dev, int ldb, int N,
                           const int* class_ptr_dev, int C, float* res_dev, int* label_dev, void* stream);

/* The l1 problem of the alignment step (Sec. II-B, the linearised
 * registration problem; Sec. VI-C):  min ||e||_1  s.t.  b_j = B_j w + e,
 * for N instances, each with its own small m x k dictionary B_j (the
 * training images of one subject and the image Jacobian of the transform),
 * solved by the primal ALM with the exact least-squares w-step (Algorithm 1
 * with w unpenalised, as the alignment experiment runs it):
 *   e <- shrink(b - B w + theta/xi, 1/xi),  w <- (B^T B)^{-1} B^T (b - e + theta/xi),
 *   theta <- theta + xi (b - B w - e),
 * from w = 0, theta = 0, xi = 2m / ||b_j||_1 (1 when b_j = 0), stopping when
 * ||w_new - w|| < tol ||w|| (strict), or after exactly -max_iter iterations
 * with no test when max_iter < 0.  Needs no plan.
 *   B_dev      N consecutive column-major m x k matrices (B_j at B_dev + j*m*k)
 *   b_dev      m x N column-major, leading dimension ldb >= m
 *   w_dev      k x N column-major (leading dimension k), written
 *   e_dev      m x N column-major, leading dimension lde >= m, written
 *   iters_dev, status_dev  N ints each, written (L1_CONVERGED, L1_MAXITER;
 *              L1_NONFINITE for a non-finite w or a rank-deficient B_j,
 *              which is reported with w = 0, e = b and iters = 0)
 * B^T B is formed and inverted once per instance in FP64, and B^T s is
 * combined in FP64; the rest runs in FP32.  All buffers are device memory
 * owned by the caller; the call is asynchronous on `stream`.
 * Limits: 1 <= k <= L1_ALIGN_MAX_K, 1 <= m <= L1_ALIGN_MAX_M (each instance
 * is one workgroup holding its dictionary in registers).
 * Errors: L1_EINVAL for sizes outside those limits, N < 0, ldb or lde < m,
 * max_iter = 0, tol not positive and finite (when max_iter > 0), or a
 * NULL buffer.                                                            */
#define L1_ALIGN_MAX_K 16
#define L1_ALIGN_MAX_M 2048
int l1_alm_align(const float* B_dev, int m, int k, int N, const float* b_dev, int ldb, float tol,
                 int max_iter, float* w_dev, float* e_dev, int lde, int* iters_dev, int* status_dev,
                 void* stream);

/* l1_alm_kkt without a plan and without any allocation, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid allocation).  Computes the same FP64
 * report as l1_alm_kkt for a plan built on this dictionary:
 *   A_dev   the dictionary (m x n_dict, column-major, leading dimension
 *           lda >= m): A for L1_DENSE, B for L1_CAB (A = [B, I])
 *   problem, structure, lambda  as in l1_alm_desc (lambda: QP_lambda only)
 *   the remaining arguments as in l1_alm_kkt.
 * The only scratch is the FP64 residual of each instance, taken from a
 * static device array of 8 MiB (2^20 doubles) that every GPU the library
 * runs on holds until the process ends; instances are processed in launches
 * of floor(2^20 / m) so any N fits.  The call allocates nothing and needs no
 * zeroed memory.  Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (other streams, other host threads) race; serialise
 * them.  Errors: L1_EINVAL for m > 2^20 rows (the scratch limit) and for
 * the arguments l1_alm_plan / l1_alm_kkt reject.                          */
#define L1_KKT_NOALLOC_MAX_M (1 << 20)
int l1_alm_kkt_noalloc(const float* A_dev, int m, int n_dict, int lda, int problem, int structure,
                       double lambda, const float* b_dev, int ldb, int N, const float* eps_dev,
                       const float* x_dev, int ldx, const float* e_dev, int lde, const float* y_dev,
                       int ldy, double* report_dev, void* stream);

/* Release the plan and all device memory it owns. */
int l1_alm_destroy(l1_alm_plan_t plan);

/* Message of the last failing call on this thread ("" if none). */
const char* l1_alm_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* L1_ALM_H_ */
