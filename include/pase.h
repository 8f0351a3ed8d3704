/*
 * pase.h -- C ABI of the MI355X augmented subspace eigensolver (gfx950).
 *
 * Computes the nev smallest eigenpairs (lambda_i, u_i) of the Q1 finite
 * element pencil A u = lambda M u of -div(kappa grad u) = lambda u on the unit
 * square / cube with u = 0 on the boundary, kappa constant per element
 * (Xie et al., arXiv 2502.04589, Sec. 2.1).  The method is the algebraic
 * augmented subspace iteration (Alg. 3 with Alg. 1 as the correction step):
 *   (a) per eigenvector, s steps of V-cycle preconditioned CG on
 *       A w = lambda M u from w = u (Alg. 3 step 3),
 *   (b) projection onto V_H + span{W}: A W, M W, restriction P^T A W and the
 *       Gram products W^T A W, W^T M W (eq. Definition_Hh),
 *   (c) the k smallest eigenpairs of the (N_H + k) augmented pencil and the
 *       prolongation U = P y_H + W y_W (Alg. 3 steps 5-6).
 *
 * Conventions used by every entry point
 * -------------------------------------
 * - Grids: level l has n[l] elements per side and m_l = n[l]-1 interior
 *   nodes per side, N_l = m_l^dim nodes, numbered x fastest.  Level 0 is the
 *   fine mesh, level nlevels-1 is the coarse space V_H.  n[l] = 2 n[l+1].
 * - Multi-vectors are node-major: an N x k array of doubles with entry
 *   (node i, column j) at i*k + j (row-major, leading dimension k).  All
 *   multi-vector and coefficient pointers are DEVICE pointers unless the
 *   argument name ends in _host.
 * - Ownership: the caller owns every buffer it passes, including the
 *   device workspace given to pase_setup.  Pointers are borrowed for the
 *   duration of the call only (the workspace for the life of the handle).
 *   The library never frees caller memory and never allocates device
 *   memory after pase_setup.
 * - Streams: all device work is enqueued on the stream given to pase_setup
 *   (a hipStream_t passed as void*, NULL = the null stream).  Entry points
 *   that return host results synchronise that stream before returning.
 * - Errors: every call returns a pase_status; it never aborts or throws.
 *   pase_last_error(h) gives a message for the last failure on h (or, with
 *   h = NULL, for the last failure of a call that had no handle, per
 *   thread).  A handle is not thread-safe; distinct handles on distinct
 *   streams are.
 * - Determinism: reductions use fixed-order trees (no floating-point
 *   atomics); the same inputs on the same GPU give bitwise equal results.
 */
#ifndef PASE_H
#define PASE_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define PASE_MAX_LEVELS 8
#define PASE_PHASES 6            /* entries of pase_report.t_phase_ms */
#define PASE_MAX_NEV 256

typedef enum pase_status {
  PASE_OK = 0,
  PASE_E_ARG = 1,          /* invalid argument (null, size, shape) */
  PASE_E_HIP = 2,          /* a HIP runtime call failed */
  PASE_E_NOMEM = 3,        /* workspace smaller than pase_workspace_bytes */
  PASE_E_NOTCONV = 4,      /* max_outer reached; outputs hold the last iterate */
  PASE_E_BREAKDOWN = 5,    /* non-SPD Gram / Cholesky failure / NaN */
  PASE_E_UNSUPPORTED = 6   /* option or size not implemented */
} pase_status;

typedef enum pase_precision {
  PASE_PREC_FP64 = 0,      /* every step in float64 */
  PASE_PREC_MIXED = 1,     /* float32 CG / V-cycle, compensated Grams, float64 RR */
  PASE_PREC_LEARNED = 2    /* learned preconditioner with GMG fallback */
} pase_precision;

/* A device CSR matrix (0-based int32 indices): rowptr has rows + 1 entries, colind and val
 * rowptr[rows] each; duplicate entries of a row are summed.  Owned by the caller. */
typedef struct pase_csr {
  int rows, cols;
  const int* rowptr;
  const int* colind;
  const double* val;
} pase_csr;

/* Algebraic input (Alg. 3 "Require" given as matrices, as an AMG hierarchy would give them):
 * per level l (0 = fine, nlevels - 1 = the coarsest, which is V_H unless coarse_level says
 * otherwise) the SPD pencil (A_l, M_l), and for l >= 1 the transfers P[l] = I_l^{l-1}
 * (N_{l-1} x N_l) and R[l] = P[l]^T (N_l x N_{l-1}).  The V-cycle smooths with damped Jacobi on
 * A_l and solves the coarsest level densely; the coarse operators are taken as given (for the
 * method they should be the Galerkin products P^T A P, P^T M P).  The caller keeps every array
 * alive and unchanged while the handle exists. */
typedef struct pase_hierarchy_csr {
  int nlevels;                   /* 2 .. PASE_MAX_LEVELS */
  pase_csr A[PASE_MAX_LEVELS];
  pase_csr M[PASE_MAX_LEVELS];
  pase_csr P[PASE_MAX_LEVELS];   /* index 0 unused */
  pase_csr R[PASE_MAX_LEVELS];   /* index 0 unused */
} pase_hierarchy_csr;

/* The discrete problem (Alg. 3 "Require"): the fine Q1 pencil (A_h, B_h = M)
 * of the element coefficient kappa and the nested grid hierarchy whose
 * coarsest level is V_H.  I_H^h is trilinear (bilinear) interpolation,
 * I_h^H its transpose, A_H / B_H the Galerkin products. */
typedef struct pase_problem {
  int dim;                       /* 2 or 3 */
  int nlevels;                   /* 2 .. PASE_MAX_LEVELS */
  int n[PASE_MAX_LEVELS];        /* elements per side; n[l] = 2*n[l+1], n[last] >= 2 */
  const double* kappa;           /* device, n[0]^dim element values (x fastest), or NULL for kappa = 1 */
  const double* tensor;          /* 3D only, NULL for the kappa problem: the tensor-coefficient workload
                                    of Sec. 5, eq. (general): -div(T grad u) + phi u = lambda u with T
                                    symmetric positive definite and constant per element, device
                                    n[0]^3 x 6 (a11, a12, a13, a22, a23, a33 per element, x fastest);
                                    kappa must then be NULL.  Read during pase_setup only: the fine
                                    operator is assembled into a 27-point stencil per node. */
  const double* reaction;        /* with tensor: device n[0]^3 element values of phi (>= 0), or NULL
                                    for phi = 0 */
  const pase_hierarchy_csr* csr; /* non-NULL: algebraic input; dim, nlevels, n, kappa, tensor and
                                    reaction are then ignored (must be 0 / NULL for the pointers);
                                    not for the learned form */
} pase_problem;

typedef struct pase_options {
  int precision;                 /* pase_precision */
  int nev_max;                   /* largest nev a later pase_solve may ask for (sizes the workspace) */
  int cg_steps;                  /* s: CG steps per outer iteration (default 2) */
  int max_outer;                 /* outer iteration limit (default 500) */
  int nu;                        /* damped-Jacobi sweeps before and after the coarse correction (default 2) */
  double omega;                  /* Jacobi damping (default 2/3) */
  int small_solver;              /* augmented eigenproblem: 0 = structured shift-invert path with dense
                                    fallback (default), 1 = dense eigensolver only, 2 = PRECOND-A and
                                    GCG_AUG (Sec. 4, Alg. 4 and 5): matrix-free, with V_H on the level
                                    coarse_level, so N_H is not bounded by a dense eigensolver */
  int locking;                   /* 1 (default): soft locking -- the fine solves of a correction run only
                                    for the pairs whose residual exceeds tol / 10 (guard pairs: 100 tol;
                                    see guard below) (a locked pair keeps
                                    w = u; the Rayleigh-Ritz still spans every pair, and a pair whose
                                    residual rises again is unlocked); 0: every pair every correction,
                                    as the algorithm is stated. */
  int guard;                     /* extra pairs carried in the block (default 0): pase_solve iterates
                                    nev + guard pairs, stops when the nev smallest meet tol and returns
                                    those.  The guard columns start from a fixed counter-based
                                    uniform(-1, 1) sequence.  A block that reaches past a cluster cut
                                    by nev converges in far fewer corrections.  0 .. 64; the workspace
                                    holds nev_max + guard columns. */
  int start;                     /* start block of pase_solve: 0 (default) = U0 as given (U0 = NULL: a
                                    fixed counter-based uniform(-1, 1) block); 1 = the coarse start of
                                    Alg. 3 steps 1-2: the nev + guard smallest eigenvectors of the
                                    coarse pencil (A_H, B_H), interpolated to the fine mesh (U0 is
                                    ignored and may be NULL; needs small_solver = 0) */
  double fallback_ratio;         /* learned form: a column switches to the V-cycle when its residual
                                    norm does not fall below fallback_ratio times its previous value
                                    (default 0.5) */
  int coarse_level;              /* the level of the hierarchy that is V_H: 0 (default) = the coarsest;
                                    1 .. nlevels - 1 selects that level (below the coarsest only with
                                    small_solver = 2; the V-cycle still runs to the coarsest level,
                                    whose dense inverse is its bottom solve).  With the coarse start
                                    (start = 1) the start block comes from the coarsest level's
                                    eigenvectors. */
  double aug_rtol;               /* small_solver 2: GCG_AUG stops when every pair's relative residual
                                    in the augmented problem is at most max(1e-11, aug_rtol times the
                                    outer residual of the same pair) (default 1e-2; 0: always to
                                    1e-11, or until the residuals stagnate) */
} pase_options;

/* Filled by pase_solve.  Array members are optional HOST buffers (NULL = not wanted). */
typedef struct pase_report {
  int outer_iters;               /* corrections performed */
  int n_converged;               /* pairs with res_i <= tol at exit */
  double* res_host;              /* nev: res_i = ||A u - lambda M u||_2 / (|lambda| ||M u||_2) */
  double* res_literal_host;      /* nev: ||A u - lambda M u||_2 / |lambda| with u^T M u = 1 */
  double* ritz_history_host;     /* (max_outer+1) x nev: Lambda before each correction and at exit */
  int ritz_history_rows;         /* rows written to ritz_history_host */
  double t_solve_ms;             /* device time of the solve (HIP events on the handle's stream) */
  int small_fast_iters;          /* corrections whose augmented eigenproblem the structured path solved */
  int* small_path_host;          /* max_outer: per correction, 1 = structured path accepted, 2 = accepted
                                    with the count certifying the nev wanted pairs only (the guard pairs
                                    are eigenpairs of the augmented problem, not certified as the next
                                    ones), 3 = accepted on the retry from the Rayleigh-Ritz start of a
                                    principal block (after a rejection), 4 = GCG_AUG (small_solver
                                    2), 0 = dense only, -1 = rejected by a residual, -2 = rejected
                                    by the eigenvalue count, -3 = its
                                    Cholesky-QR orthonormalisation broke down (the last rejection of
                                    the correction; the dense solver then solved it) */
  int learned_fallbacks;         /* learned form: column switches to the V-cycle, summed over the solve */
  int lowprec_projection_iters;  /* mixed form: corrections whose projection ran on FP32 vectors with
                                    split-BF16 Grams (the rest ran in FP64) */
  int fine_solve_columns;        /* columns that ran the fine solves, summed over the corrections
                                    (nev x outer_iters without locking) */
  double t_phase_ms[PASE_PHASES];/* device time per phase (HIP events on the handle's stream; the
                                    stream's idle gaps while the host reads residuals are left out):
                                    [0] start block (Alg. 3 steps 1-2: coarse start or the given
                                    block, Cholesky-QR, Lambda0); [1] eigen-residuals and stop test
                                    (Alg. 3 step 4); [2] fine solves (step 3: s CG steps per column
                                    with the V-cycle, the network or the FP32 correction form);
                                    [3] projection (the complement of W, A W, M W, the coarse
                                    restriction of A W, the Grams alpha and beta, their Cholesky
                                    factor and H); [4] the augmented eigenproblem (step 5:
                                    structured path, retry and dense path, or GCG_AUG); [5]
                                    prolongation (step 6: u = P y_H + W y_W) */
  int aug_iters;                 /* small_solver 2: GCG_AUG iterations summed over the corrections */
  int aug_restarts;              /* small_solver 2: GCG_AUG iterations whose orthonormalisation or
                                    Rayleigh-Ritz broke down (each was redone without the P block,
                                    or ended the augmented solve at the last good iterate) */
} pase_report;

typedef struct pase_handle pase_handle;
typedef struct pase_unet pase_unet;

/* ---------------------------------------------------------------- core API */

/* Default options: FP64, nev_max 16, s = 2, max_outer 500, nu = 2, omega = 2/3, soft locking,
 * no guard pairs, start block U0, fallback ratio 0.5. */
void pase_options_default(pase_options* opt);

/* Device workspace needed by pase_setup for this problem and options. */
pase_status pase_workspace_bytes(const pase_problem* prob, const pase_options* opt, size_t* bytes);

/* Builds the hierarchy (Galerkin coarse stencils, coarse factorisations) inside
 * the caller's device workspace (>= pase_workspace_bytes, 256-byte aligned).
 * prob->kappa is copied; it may be freed after the call.  *out receives a
 * host-side handle released by pase_destroy (it holds a few KB of pinned host memory for the
 * per-correction transfers; no device memory is allocated outside the workspace). */
pase_status pase_setup(const pase_problem* prob, const pase_options* opt, void* workspace,
                       size_t workspace_bytes, void* stream, pase_handle** out);

/* Alg. 3 ensure: the nev smallest eigenpairs of (A_h, M).
 * U0: device N_0 x nev start block (any full-rank block; it is M-orthonormalised), or NULL for a
 * fixed counter-based uniform(-1, 1) block; ignored with opt.start = 1 (coarse eigenvectors).
 * lambda_host: nev eigenvalues, ascending.  U: device N_0 x nev, U^T M U = I.
 * U0 and U may be the same buffer.  Stops when every res_i <= tol (see
 * pase_report) or after opt.max_outer corrections (PASE_E_NOTCONV).  With opt.guard > 0 the
 * iteration carries nev + guard pairs; only the nev smallest decide convergence and are returned. */
pase_status pase_solve(pase_handle* h, int nev, double tol, const double* U0, double* lambda_host,
                       double* U, pase_report* rep);

/* Batch scheme (Sec. "Batch scheme for computing plenty of eigenpairs", Alg. 7 step 3): the pairs
 * first .. first + nb - 1 (0-based, ascending) of (A_h, M) with a working block of nb + 2 guard
 * pairs at most (opt.guard below the batch, fewer for first < guard, and opt.guard above it).
 * Start: the block's coarse eigenvectors interpolated and its coarse eigenvalues; shift theta =
 * the midpoint of the block's first and last coarse eigenvalue.  Per correction: s CG steps, the
 * composite pencil, its min(2 k, N_H + k) eigenpairs nearest theta (k = the block's width), the k
 * with the largest component in the span of the fine directions (eq. largest_component),
 * prolongation; the test on those pairs (res_i <= tol for the batch's own pairs, positions of the
 * block's ascending order); then s CG steps of post-smoothing from them.
 * lambda_host: nb eigenvalues, ascending.  U: device, the batch's nb columns with row stride
 * ldu >= nb (U^T M U = I for them).  rep->res_host (optional): nb residuals.  Needs the dense
 * small path with the coarsest level's eigenbasis (small_solver 0 with the structured path on,
 * N_H + nev_max + guard <= 3840, nev_max + guard <= 128) and block width <= nev_max + guard,
 * first + nb + guard <= N_H;
 * precision fp64 or mixed.  The pairs found are those that the coarse start resolves: batches
 * beyond what V_H separates (coarse eigenvalue error above the spectral gaps) may converge to
 * neighbouring pairs or not at all (PASE_E_NOTCONV after opt.max_outer corrections). */
pase_status pase_solve_batch(pase_handle* h, int first, int nb, double tol, double* lambda_host, double* U,
                             int ldu, pase_report* rep);

/* Alg. 7: the m smallest pairs in batches of nb (the last one ragged), solved one after another
 * by pase_solve_batch into lambda_host (m, ascending per batch) and the columns of U (device
 * N_0 x m).  rep->res_host (optional) holds m entries; the report sums iterations, times and
 * phases over the batches.  Stops at the first batch that fails and returns its status. */
pase_status pase_solve_batches(pase_handle* h, int m, int nb, double tol, double* lambda_host, double* U,
                               pase_report* rep);

pase_status pase_destroy(pase_handle* h);

const char* pase_status_string(pase_status s);
const char* pase_last_error(const pase_handle* h);

/* N_l of level l (0 = fine). */
pase_status pase_level_size(const pase_handle* h, int level, long long* N);

/* ---------------------------------------------------------------- component entry points
 * Single steps of the path, for parity tests and benchmarks.  k <= nev_max. */

/* AX = A_l X, MX = M_l X on level l (either output may be NULL). */
pase_status pase_apply(pase_handle* h, int level, int k, const double* X, double* AX, double* MX);

/* Z = V(B): one V-cycle on level 0 from a zero initial guess (the CG preconditioner). */
pase_status pase_vcycle(pase_handle* h, int k, const double* B, double* Z);

/* Alg. 3 step 3: s preconditioned CG steps per column on A w = lambda_j M u_j from w = u_j.
 * lambda_host: k values.  A learned-form handle runs the flexible PCG with its attached network
 * and the per-column V-cycle fallback (PASE_E_ARG without a network). */
pase_status pase_pcg(pase_handle* h, int k, const double* lambda_host, const double* U, double* W);

/* Xc = P^T Xf (fine level 0 -> coarsest), and Xf = P Xc (coarsest -> fine), P = I_H^h. */
pase_status pase_restrict(pase_handle* h, int k, const double* Xf, double* Xc);
pase_status pase_prolong(pase_handle* h, int k, const double* Xc, double* Xf);

/* G = X^T Y for N x k node-major X, Y (G: k x k row-major, device).  N <= N_0. */
pase_status pase_gram(pase_handle* h, long long N, int k, const double* X, const double* Y, double* G);

/* G = X^T Y (k x k, device, FP64) of FP32 operands X, Y (N x k row-major, device), k <= 128, the
 * projection Gram of the mixed form's first phase (extension (1) of the method: low-precision
 * projection, FP64 Rayleigh-Ritz).  Each value is split x = x_hi + x_lo into two BF16 numbers; a
 * product is x_hi y_hi + x_hi y_lo + x_lo y_hi on BF16 MFMA with FP32 accumulation over blocks of
 * 256 rows, the block sums added in FP64 in a fixed order.  Error per entry below about
 * 2^-15 sum_r |x_r y_r|.  Synchronises the handle's stream. */
pase_status pase_gram_bf16x3(pase_handle* h, long long N, int k, const float* X, const float* Y, double* G);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): G = X^T Y like pase_gram, without a handle or a
 * workspace.  X, Y: device N x k (row-major, leading dimension k); G: device k x k (row-major);
 * 1 <= k <= 128.  The per-block partial sums live in a 16 MiB device array of the library (one
 * copy per GPU, held until the process ends; its address is looked up on the first call on each
 * device); the call allocates nothing and does not synchronise: the work is enqueued on `stream`
 * (a hipStream_t as void*, NULL = the null stream).  Calls on one GPU share that array, so calls
 * that overlap in time on one GPU (different streams, or host threads) race; calls in one stream
 * are ordered and safe.  Every partial it reads was written by the same call, so nothing has to
 * be cleared between calls.  For k <= 64 the result is bitwise equal to pase_gram's; for larger k
 * the partials come from fewer, longer row blocks (equal to rounding).  PASE_E_ARG for null
 * pointers, N < 1 or k outside [1, 128]; PASE_E_HIP if the launch fails; the message is in
 * pase_last_error(NULL). */
pase_status pase_gram_noalloc(long long N, int k, const double* X, const double* Y, double* G, void* stream);

/* The k smallest eigenpairs of a dense symmetric n x n matrix T (row-major, device):
 * w_host (k, ascending) and V (device, n x k row-major, orthonormal columns).
 * n <= pase_small_eig_max_n(h); T is not modified. */
pase_status pase_small_eig(pase_handle* h, int n, int k, const double* T, double* w_host, double* V);
/* A grid handle's hierarchy as device CSR (the input of pase_hierarchy_csr, or for inspection):
 * which = 0 A_l, 1 M_l (N_l x N_l, 3^dim slots per row), 2 P_l = I_l^{l-1} (N_{l-1} x N_l, 2^dim
 * slots per row, level >= 1), 3 R_l = P_l^T (N_l x N_{l-1}, 3^dim slots per row, level >= 1).
 * Every row has exactly `slots` entries (entries outside the matrix's pattern hold 0), so
 * rowptr[i] = slots * i.  *rows, *cols, *slots are written; rowptr (rows + 1), colind and val
 * (rows * slots each) are device arrays, or all NULL to query the sizes only.  Synchronises the
 * handle's stream; uses the fine multi-vector space as scratch (not during a solve).  Errors:
 * PASE_E_ARG for a bad level / which, PASE_E_UNSUPPORTED for an algebraic handle. */
pase_status pase_export_csr(pase_handle* h, int level, int which, int* rows, int* cols, int* slots, int* rowptr,
                            int* colind, double* val);
int pase_small_eig_max_n(const pase_handle* h);

/* One full correction (Alg. 1 / Alg. 3 steps 3-6) from (lambda, U) with U^T M U = I:
 * U is overwritten with the new block and lambda_host with the new Ritz values. */
pase_status pase_correction(pase_handle* h, int k, double* lambda_host, double* U);

/* Benchmark support: average device time in ms of one launch of the kernel
 * selected by `which`, over `reps` back-to-back launches bracketed by two HIP
 * events on the handle's stream, at k columns, reading the handle's internal
 * fine-level buffers (call after a pase_solve with the same k so they hold
 * finite data).  Launch configuration is the one pase_solve uses.
 *   which = 0: fine-level damped-Jacobi sweep x' = x + omega D^{-1}(b - A x)
 *   which = 1: fine-level fused A X, M X
 *   which = 2: Gram W^T (A W) on FP64 MFMA (including its fixed-order reduction)
 *   which = 3: one V-cycle (all levels)
 *   which = 5: the fused CG update x += alpha p, r -= alpha q (on scratch vectors)
 *   which = 6: fine-level A X alone (the projection's SpMM)
 *   which = 7: fine-level M X alone (the complement's SpMM)
 * (which = 4 is not used) */
pase_status pase_time_kernel(pase_handle* h, int which, int k, int reps, double* ms);

/* ---------------------------------------------------------------- learned preconditioner
 * The learned form of the method (an extension the paper does not define) replaces the
 * V-cycle inside the fine-grid PCG by a small 3D convolutional network N trained on the
 * solver's own (residual, V-cycle correction) pairs, with the V-cycle as fallback.
 * Network: 3-level U-Net on the interior nodes of the fine n^3 mesh (n divisible by 4),
 * channels {16, 32, 64} (the only set the kernels are built for); per level two 3x3x3
 * convolutions without bias, each followed by ReLU; full-weighting restriction down,
 * trilinear prolongation up, skip connections by channel concatenation, final 3x3x3
 * convolution to one channel.  Inputs: r / rho(r), rho(r) = ||r||_2 / sqrt(N_0) (the root mean
 * square), and the node average of log kappa; N(r) = rho(r) net(r / rho(r), log kappa).  BF16 weights and activations on MFMA with
 * FP32 accumulation; FP32 master weights and Adam moments.
 *
 * Parameters: 11 FP32 tensors W_i[27][Cin][Cout] (offset o = 0..26 enumerates (dx, dy, dz)
 * in {-1,0,1}^3 with dx fastest) concatenated in layer order: 2->16, 16->16, 16->32,
 * 32->32, 32->64, 64->64, (64+32)->32, 32->32, (32+16)->16, 16->16, 16->1; concatenated
 * inputs list the up-sampled channels first.
 * Multi-vectors R, C, Z are device FP64, N_0 x batch, node-major (row = node, x fastest);
 * logk is device FP64 N_0 (or NULL for kappa = 1).  Errors: PASE_E_ARG for bad shapes,
 * PASE_E_NOMEM for a small workspace, PASE_E_HIP for runtime failures. */
pase_status pase_unet_param_count(const int* channels, size_t* count);
pase_status pase_unet_workspace_bytes(int n, int batch_max, const int* channels, size_t* bytes);
/* The network lives in the caller's device workspace (256-byte aligned); its work is
 * enqueued on `stream`.  Weights are undefined until pase_unet_set_weights. */
pase_status pase_unet_create(int n, int batch_max, const int* channels, void* workspace, size_t bytes,
                             void* stream, pase_unet** out);
pase_status pase_unet_destroy(pase_unet* u);
const char* pase_unet_last_error(const pase_unet* u);
/* W: device FP32 parameter vector (pase_unet_param_count entries); resets the Adam state. */
pase_status pase_unet_set_weights(pase_unet* u, const float* W);
pase_status pase_unet_get_weights(const pase_unet* u, float* W);
/* Checkpoint of the training state; both calls synchronise the network's stream.
 * pase_unet_save writes the FP32 weights, both Adam moments and the Adam step count, with the
 * channel widths, to the host file `path` (a 64-byte header -- tag "PASEUNET",
 * format version 1, the three widths, the parameter count P, the step count -- then 3 P FP32
 * values, little-endian); pase_unet_load restores them into a network created with the same
 * widths, so training resumes where it stopped (the next Adam step is step count + 1).  Errors:
 * PASE_E_ARG for a null argument, a file that cannot be opened, read or written, a foreign or
 * truncated file, or other widths (the network is then unchanged); PASE_E_HIP for copy failures. */
pase_status pase_unet_save(pase_unet* u, const char* path);
pase_status pase_unet_load(pase_unet* u, const char* path);
/* Z = N(R), column by column. */
pase_status pase_unet_apply(pase_unet* u, int batch, const double* R, const double* logk, double* Z);
/* Loss L = mean_b ||N(r_b) - c_b||^2 / ||c_b||^2 (written to *loss_host if non-NULL, which
 * synchronises the stream) and its gradient with respect to the parameters, kept for
 * pase_unet_adam_step and copied to the device vector G if non-NULL. */
pase_status pase_unet_loss_grad(pase_unet* u, int batch, const double* R, const double* C, const double* logk,
                                double* loss_host, float* G);
/* Node-wise output scale s (device, N_0 values, caller-owned and kept alive while the network
 * uses it; NULL = 1): from now on N(R) = rho(r) s * net(r / rho(r), log kappa) in apply, loss_grad
 * and fit_scale.  The learned form uses s = the inverse diagonal of A (pase_fine_diag_inverse). */
pase_status pase_unet_set_output_scale(pase_unet* u, const double* scale);
/* Output scale fit (done once before training): multiplies the weights of the three layers after
 * the last concatenation by s^(1/3), s = ||C||_F / ||N(R)||_F over the batch (targets C and
 * residuals R: device N_0 x batch each), so the output's size matches the targets' (each of those
 * layers is positively homogeneous, so the output becomes s N(R)).  s goes to *scale_host (may be
 * NULL).  PASE_E_BREAKDOWN if the output or the targets are zero (weights unchanged). */
pase_status pase_unet_fit_scale(pase_unet* u, int batch, const double* R, const double* C, const double* logk,
                                double* scale_host);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the gradient of the last loss_grad. */
pase_status pase_unet_adam_step(pase_unet* u, float lr);

/* Learned form: attaches a network (created for this fine mesh, batch_max >= nev_max) to a
 * 3D handle set up with precision PASE_PREC_LEARNED.  The network's work then runs on the
 * handle's stream.  In every outer step the s CG steps become flexible PCG preconditioned
 * by the network; a column whose residual norm does not drop below half its previous value
 * switches to the V-cycle for the rest of that outer step (the step is kept). */
pase_status pase_attach_unet(pase_handle* h, pase_unet* u);
/* Training pairs for the network: R = Lambda M U - A U for the pairs (lambda_host, U) and
 * V = one V-cycle applied to R (device N_0 x k each). */
pase_status pase_harvest(pase_handle* h, int k, const double* lambda_host, const double* U, double* R, double* V);
/* 1 / A_ii at the fine nodes (device N_0): the network's output scale in the learned form. */
pase_status pase_fine_diag_inverse(pase_handle* h, double* dinv);
/* Node average of log kappa over the elements around each interior fine node (device N_0;
 * zeros for kappa = 1): the network's second input channel. */
pase_status pase_node_logk(pase_handle* h, double* logk);

#ifdef __cplusplus
}
#endif

#endif /* PASE_H */
