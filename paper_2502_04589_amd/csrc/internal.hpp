// Internal declarations shared by the HIP translation units of libpase.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/pase.h"

#include <string>

namespace pase {

// message returned by pase_last_error(NULL) on this thread
void set_last_error(const std::string& msg);

constexpr int kBlock = 256;          // threads per block of the grid kernels
constexpr int kMaxStencil = 27;      // 3^dim neighbours

// One grid level of the hierarchy.
struct Level {
  int n = 0;                 // elements per side
  int m = 0;                 // interior nodes per side (n - 1)
  long long N = 0;           // m^dim
  double h = 0.0;            // mesh width 1/n
  const double* kappa = nullptr;   // level 0: element coefficients (n^dim)
  double* coef = nullptr;          // levels >= 1: assembled A stencil, N x 3^dim
  double* dinv = nullptr;          // 1 / diag(A), N
};

// Stencil source of the operator A on a level.
enum class ASource : int { Kappa = 0, Assembled = 1 };

// Epilogue of the stencil kernel.
enum Epi : int {
  EPI_AM = 0,       // out1 = A x (opt), out2 = M x (opt)
  EPI_RESID = 1,    // out1 = b - A x
  EPI_SWEEP = 2,    // out1 = x + omega D^{-1} (b - A x)
  EPI_EIGRES = 3,   // out1 = lambda_j M x - A x; partials of |out1|^2, |M x|^2, x.(M x) per column
  EPI_AMDOT = 4,    // out1 = A x; partials of x.(A x) per column (3D LDS-staged stencil only)
  EPI_SWEEPDOT = 5, // out1 = the sweep of EPI_SWEEP; partials of b.out1 per column (3D LDS-staged only)
  EPI_SWEEP2 = 6,   // out1 = two damped-Jacobi sweeps from x = 0 with x passed as b (constant
                    // coefficient, 3D LDS-staged only): x1 = c b, out = x1 + c (b - A x1), c = omega / a_ii
  // 3D LDS-staged stencil only, chosen by launch_fine3 for EPI_AM with one output:
  EPI_A = 7,        // out1 = A x
  EPI_M = 8,        // out2 = M x (kappa-independent: staged planes are read once)
  // 3D LDS-staged only, variable coefficient: the first two damped-Jacobi sweeps from x = 0 with x
  // and b both passed as b: the staged planes hold x1 = omega D^{-1} b (scaled as they are staged),
  // out = x1 + omega D^{-1} (b - A x1)
  EPI_SWEEP2V = 9,
  // 3D LDS-staged only, variable coefficient: the residual after one damped-Jacobi sweep from x = 0,
  // with x passed as b: the staged planes hold x1 = omega D^{-1} b, out = b - A x1 (b recovered from
  // x1 at the node)
  EPI_RESID1V = 10,
};

struct StencilArgs {
  int dim;
  int m;                 // interior nodes per side
  long long N;
  int k;                 // columns (<= 256)
  double h;
  ASource src;
  const double* kappa;   // Kappa source
  const double* coef;    // Assembled source (N x 3^dim)
  const double* dinv;
  const void* x;         // multi-vectors: double, or float when fp32
  const void* b;         // rhs for RESID / SWEEP
  const double* lam;     // EIGRES: k values (device)
  void* out1;
  void* out2;
  double* partial;       // EIGRES: [tiles][3][k]
  double omega;
  int fp32;
};

// ---- grid kernels (grid.hip)
struct GridLaunch {
  int slots;        // nodes processed side by side per pass (256 / k)
  int nb;           // nodes per block
  int tiles;        // logical tiles
  int blocks;       // launched blocks (tiles rounded up to a multiple of 8)
};
GridLaunch grid_launch(long long N, int k);
void launch_stencil(const StencilArgs& a, Epi epi, hipStream_t s);
void launch_first_sweep(int dim, long long N, int k, const double* dinv, double omega,
                        const void* b, void* x, int fp32, hipStream_t s);
// restriction xc = P^T xf (ratio 2), prolongation xf (op)= P xc; mode 0: xf = P xc, 1: xf += P xc, 2: xf -= P xc
void launch_restrict(int dim, int mf, int mc, int k, const void* xf, void* xc, int fp32, hipStream_t s);
void launch_prolong(int dim, int mf, int mc, int k, const void* xc, void* xf, int mode, int fp32, hipStream_t s);
// xf = omega D^{-1} b + P xc (the coarse correction added to one damped-Jacobi sweep from x = 0,
// formed here instead of being stored by the sweep); dinv per fine node
void launch_prolong_first(int dim, int mf, int mc, int k, const void* xc, void* xf, const void* b,
                          const double* dinv, double omega, int fp32, hipStream_t s);
// setup helpers
void launch_kappa_dinv(int dim, int n, const double* kappa, double* dinv, hipStream_t s);
void launch_kappa_coefs(int dim, int n, const double* kappa, double* coef, hipStream_t s);   // N x 3^dim
void launch_color_probe(int dim, int m, double* E, hipStream_t s);                 // N x 3^dim
void launch_extract_galerkin(int dim, int m, const double* Y, double* coef, double* dinv, hipStream_t s);
void launch_stencil_to_dense(int dim, int m, const double* coef, double hmass, int use_mass, double* D,
                             hipStream_t s);
// 3D fine-level 27-point stencil of -div(T grad) + phi from per-element T (upper triangle, 6 values)
// and phi (may be null), and 1 / diag
void launch_assemble_general(int n, const double* tensor, const double* reaction, double* coef, double* dinv,
                             hipStream_t s);

// ---- fine-level 3D LDS-staged stencil (stencil3d.hip)
struct Fine3Args {
  int m;                 // interior nodes per side
  int k;                 // columns
  double h;
  const double* kappa;   // n^3 element coefficients or nullptr (kappa = 1)
  const double* coef;    // or: an assembled 27-coefficient row of A per node (tensor-coefficient problem)
  const void* x;         // N x k (double or float)
  const void* b;
  const double* lam;
  void* out1;
  void* out2;
  double* partial;       // EIGRES: [spatial blocks][3][k]
  double omega;
  int nzc;               // z-runs per column chunk
  int fp32;              // 1: multi-vectors are float
  const void* zero;      // >= 16 zero bytes (read by out-of-domain halo lanes)
  const double* dinv;    // EPI_SWEEP2V: 1 / diag(A) per node
};
void launch_fine3(const Fine3Args& a, Epi epi, hipStream_t s);
int fine3_spatial_blocks(int m, int nzc, int k, bool fp32);
int fine3_default_nzc(int m);
int fine3_max_spatial_blocks(int m);

// ---- BLAS-like kernels (blas.hip)
// per-column dot products of N x k blocks: out[j] = sum_i X[i,j] Y[i,j] (fixed-order two-pass)
void launch_coldot(long long N, int k, const double* X, const double* Y, double* partial, int ptiles,
                   double* out, hipStream_t s);
int coldot_tiles(long long N, int k);
void launch_reduce_partials(int tiles, int width, const double* partial, double* out, hipStream_t s);
// PCG scalars / updates
void launch_pcg_alpha(int k, const double* rho, const double* pq, double* alpha, hipStream_t s);
void launch_pcg_beta(int k, const double* rho_new, const double* rho_old, double* beta, hipStream_t s);
void launch_axpy2(long long N, int k, const double* alpha, const double* P, const double* Q, double* X,
                  double* R, hipStream_t s);
// X = Xin + alpha P, R -= alpha Q (column-wise alpha); X and Xin distinct buffers
void launch_axpy2_from(long long N, int k, const double* alpha, const double* P, const double* Q, const double* Xin,
                       double* X, double* R, hipStream_t s);                    // X += a P ; R -= a Q
void launch_xpby(long long N, int k, const double* Z, const double* beta, double* P, hipStream_t s);  // P = Z + b P
void launch_copy(size_t n, const double* src, double* dst, hipStream_t s);
// Gram G = X^T Y (k x k) by FP64 MFMA over row chunks, fixed-order reduction
int gram_tiles(long long N, int k);
// G1 = X^T Y1 and, if Y2, G2 = X^T Y2 in one pass over X (partial: 2 x tiles x k x k)
void launch_gram2(long long N, int k, const double* X, const double* Y1, const double* Y2, double* partial,
                  int tiles, double* G1, double* G2, hipStream_t s);
void launch_gram(long long N, int k, const double* X, const double* Y, double* partial, int tiles, double* G,
                 hipStream_t s);
// the same when every product is symmetric (W^T A W, W^T M W, U^T M U): for 64 < k <= 128 only the
// upper tiles are multiplied and mirrored (for k <= 64 it is launch_gram2)
void launch_gram2_sym(long long N, int k, const double* X, const double* Y1, const double* Y2, double* partial,
                      int tiles, double* G1, double* G2, hipStream_t s);
// C = alpha op(A) op(B) + beta C, row-major, FP64
void launch_gemm(bool ta, bool tb, int M, int N, int K, double alpha, const double* A, int lda, const double* B,
                 int ldb, double beta, double* C, int ldc, hipStream_t s);
// FP32 multi-vector variants (scalars and reductions stay FP64)
void launch_coldot_f32(long long N, int k, const float* X, const float* Y, double* partial, double* out,
                       hipStream_t s);
void launch_axpy2_f32(long long N, int k, const double* alpha, const float* P, const float* Q, float* X, float* R,
                      hipStream_t s);
void launch_xpby_f32(long long N, int k, const float* Z, const double* beta, float* P, hipStream_t s);
void launch_gemm_f32(bool ta, bool tb, int M, int N, int K, double alpha, const float* A, int lda, const float* B,
                     int ldb, double beta, float* C, int ldc, hipStream_t s);
void launch_d2f(size_t n, const double* a, float* b, hipStream_t s);
void launch_f2d(size_t n, const float* a, double* b, hipStream_t s);
// G1 = X^T Y1 (and G2 = X^T Y2) of FP32 operands, split-BF16 products on MFMA, k <= 128 (nothing is
// launched for larger k)
void launch_gram_bf16x3(long long N, int k, const float* X, const float* Y1, const float* Y2, double* partial,
                        int tiles, double* G1, double* G2, hipStream_t s);
void launch_add_f2d(size_t n, const double* u, const float* e, double* w, hipStream_t s);
void launch_add_f2d_merge(long long N, int k, int ldw, const int* pos, const double* u, const float* e, double* w,
                          hipStream_t s);
void launch_cg_start_f32(size_t n, const double* R, float* r, float* e, hipStream_t s);
// learned form: flexible-PCG beta, per-column fallback to the V-cycle, column selection
void launch_flex_beta(int k, const double* a, const double* b, const double* c, int* mask, double* beta,
                      hipStream_t s);
void launch_fallback(int k, double ratio, const double* rn, const double* ro, int* mask, hipStream_t s);
void launch_select_cols(long long N, int k, const int* mask, const double* A, double* Z, hipStream_t s);
// C (N x ka) = columns idx[0..ka) of B (N x k), and back
void launch_gather_cols(long long N, int k, int ka, const int* idx, const double* B, double* C, hipStream_t s);
void launch_scatter_cols(long long N, int k, int ka, const int* idx, const double* C, double* B, hipStream_t s);
void launch_rsub(long long N, int k, const double* alpha, const double* Q, double* R, hipStream_t s);
void launch_zadd(long long N, int k, const double* beta, const double* P, double* Z, hipStream_t s);
void launch_axpy3(long long N, int k, const double* a0, const double* P, const double* a1, const double* Z,
                  const double* X0, double* X, hipStream_t s);
void launch_axpy3_merge(long long N, int k, int ldx, const int* pos, const double* a0, const double* P, const double* a1,
                        const double* Z, const double* X0, double* X, hipStream_t s);
void launch_merge_cols(long long N, int k, int ka, const int* pos, const double* C, const double* U, double* B,
                       hipStream_t s);
// dst (N x kout) columns [0, nc) from src (N x kin); fill: columns [nc, kout) get uniform(-1, 1)
// values from a counter-based generator (kout = dst's leading dimension)
void launch_copy_cols(long long N, int kin, int kout, int nc, const double* src, double* dst, int fill,
                      hipStream_t s);
void launch_fill_int(int n, int v, int* p, hipStream_t s);
void launch_node_logk(int n, const double* kappa, double* out, hipStream_t s);
// the network's kernels run on the given stream from now on
void unet_set_stream(pase_unet* u, hipStream_t s);
int unet_fine_n(const pase_unet* u);
int unet_batch_max(const pase_unet* u);
void launch_copy_f32(size_t n, const float* src, float* dst, hipStream_t s);
// tall-skinny: Y = X op(C) (+ Y): X N x k, C k x k (transposed if tb), Y N x k; Y must not alias X
void launch_tsmm(long long N, int k, const double* X, const double* C, double* Y, int accumulate, int tb,
                 hipStream_t s);
// small helpers
void launch_set_diag_block(int n, int nh, int k, const double* C0, const double* G, const double* H, double* T,
                           hipStream_t s);

// ---- algebraic input (csr.hip): CSR operators on node-major multi-vectors
struct CsrMat {
  const int* rowptr;
  const int* colind;
  const double* val;
};
struct CsrOpArgs {
  long long rows;
  int k;                  // columns (<= 256)
  CsrMat A, M;
  const double* dinv;     // SWEEP: 1 / diag(A)
  double omega;
  const void* x;          // double, or float when fp32
  const void* b;          // RESID / SWEEP right-hand side
  const double* lam;      // EIGRES
  void* out1;
  void* out2;
  double* partial;        // EIGRES: [csr_tiles(rows)][3][k]
  int fp32;
};
int csr_tiles(long long rows);
// epilogues EPI_AM (either output may be null), EPI_RESID, EPI_SWEEP, EPI_EIGRES
void launch_csr_op(const CsrOpArgs& a, Epi epi, hipStream_t s);
// y (=, +=, -=) A x for mode 0, 1, 2
void launch_csr_apply(const CsrMat& A, long long rows, int k, const void* x, void* y, int mode, int fp32,
                      hipStream_t s);
void launch_csr_diag_inv(const CsrMat& A, long long rows, double* dinv, hipStream_t s);
void launch_csr_to_dense(const CsrMat& A, long long rows, double* D, hipStream_t s);
// a grid hierarchy as CSR with a fixed number of slots per row (rowptr[i] = slots i, unused slots hold
// zeros): a level operator from its stencil (coef null: the Q1 mass of width hmass), P, R = P^T
void launch_export_stencil(int dim, int m, const double* coef, double hmass, int* rowptr, int* colind, double* val,
                           hipStream_t s);
void launch_export_prolong(int dim, int mf, int mc, int* rowptr, int* colind, double* val, hipStream_t s);
void launch_export_restrict(int dim, int mf, int mc, int* rowptr, int* colind, double* val, hipStream_t s);

// ---- batch scheme (batch.hip): the k of nsel <= batch_select_max() composite pairs with the
// largest component in span(u_hat), from their coordinates Y (k x nsel) in an orthonormal basis of it
int batch_select_max();
void launch_batch_select(int k, int nsel, const double* Y, int* sel, int* flag, hipStream_t s);

// ---- GCG_AUG (gcg.hip): augmented blocks are (N_H + k) x w row-major
// C (m x n) = A^T B over N rows, A: N x m (lda), B: N x n (ldb); fixed-order reduction over at most
// 128 row chunks; partial >= gram_tn_partial_doubles(N, m, n)
size_t gram_tn_partial_doubles(long long N, int m, int n);
void launch_gram_tn(long long N, int m, int n, const double* A, int lda, const double* B, int ldb, double* partial,
                    double* C, hipStream_t s);
void launch_aug_resid(long long N, int k, const double* AX, const double* BX, const double* lam, double* R,
                      hipStream_t s);                                            // R = AX - BX diag(lam)
void launch_gather_scale(long long N, int k, int ka, const int* idx, const double* src, const double* lam,
                         double* dst, hipStream_t s);                            // dst_j = src_idx[j] lam_idx[j]
void launch_aug_start(long long NH, int k, const double* ahat, double* X, hipStream_t s);   // [a_hat ; I]
void launch_assemble_rr(int k, int ny, const double* Gxx, const double* Gxy, const double* Gyy, double* H,
                        hipStream_t s);
void launch_ltl(int k, const double* Li, double* C, hipStream_t s);             // C = Li^T Li
void launch_sub(long long n, const double* a, const double* b, double* c, hipStream_t s);   // c = a - b (null = 0)
// n x n G <- D G D with D = diag(G)^{-1/2} (d gets D's diagonal); M <- M D for an n x n M
void launch_unit_diag(int n, double* G, double* d, hipStream_t s);
void launch_scale_cols_sq(int n, double* M, const double* d, hipStream_t s);

// ---- dense single-workgroup kernels (dense.hip)
// In-place lower Cholesky of an n x n SPD matrix (row-major); info[0] = 0 ok, j+1 if pivot j failed.
void launch_cholesky(int n, double* A, int lda, int* info, hipStream_t s);
// Li = L^{-1} (lower) from a lower factor L; Li must not alias L.
void launch_trinv(int n, const double* L, int ldl, double* Li, int ldi, hipStream_t s);
// lowest k eigenpairs of dense symmetric T (n x n); T is overwritten; w, V device; work >= syev_work_doubles(n,k)
size_t syev_work_doubles(int n, int k);
void launch_syev_lowest(int n, int k, double* T, double* w, double* V, double* work, int* info, hipStream_t s);
int syev_max_n();
int syev_max_k();
// G (k x k, lower part read) <- L^{-1} with G = L L^T, in LDS; *info = 1 on a non-positive pivot. k <= syev_max_k()
void launch_cholinv(int k, double* G, int* info, hipStream_t s);
// two Cholesky-QR passes over a vector-major n x k block (result back in Vt; Vt2 scratch)
void launch_vorth2(int n, int k, double* Vt, double* Vt2, double* G, int* info, hipStream_t s);

// Gershgorin bounds and pivmin of the tridiagonal in tri (d, e, tau, scalars) after a reduction
void launch_tri_finish(int n, double* tri, hipStream_t s);
// S matrices of the blocked back-transformation from the reflectors stored in the rows of T
void launch_wy_prep(int n, const double* T, const double* tri, double* Sall, hipStream_t s);

// ---- large dense kernels (dense_large.hip): coarse spaces of thousands of nodes
// C = alpha op(A) op(B) + beta C (row-major) on FP64 MFMA; the float version stores float and
// computes in FP64
void launch_gemm_mfma(bool ta, bool tb, int M, int N, int K, double alpha, const double* A, int lda,
                      const double* B, int ldb, double beta, double* C, int ldc, hipStream_t s);
void launch_gemm_mfma_f32(bool ta, bool tb, int M, int N, int K, double alpha, const float* A, int lda,
                          const float* B, int ldb, double beta, float* C, int ldc, hipStream_t s);
// blocked lower Cholesky in place (*info = 0, or j + 1 for a failed pivot j)
size_t cholesky_large_scratch_doubles(int n);
void launch_cholesky_large(int n, double* A, int lda, double* scratch, int* info, hipStream_t s);
// Li = L^{-1} by block rows (Li must not alias L)
size_t trinv_large_scratch_doubles(int n);
void launch_trinv_large(int n, const double* L, int ldl, double* Li, int ldi, double* scratch, hipStream_t s);
// the k smallest eigenpairs of a dense symmetric n x n matrix, n <= syev_large_max_n() (T overwritten)
int syev_large_max_n();
size_t syev_large_work_doubles(int n, int k);
void launch_syev_large(int n, int k, double* T, double* w, double* V, double* work, int* info, hipStream_t s);
// the nsel eigenpairs nearest theta, ascending (T overwritten; work of syev_window_work_doubles)
size_t syev_window_work_doubles(int n, int nsel);
void launch_syev_window(int n, int nsel, double theta, double* T, double* w, double* V, double* work, int* info,
                        hipStream_t s);

// ---- structured augmented eigenproblem (small.hip): Tt = [[diag(theta), Gt], [Gt^T, H]]
int small_fast_max_k();
int small_fast_max_nh();   // N_H limit
// shift-invert / Rayleigh-quotient iteration per pair; start vectors: column i of X0 ((N_H + k) x k
// row-major; first shift its Rayleigh quotient) or, if X0 is null, a fixed pseudo-random vector with
// first shift sigma[i]; Vt vector-major (N_H + k) x k
void launch_small_rqi(int nH, int k, const double* theta, const double* Gt, const double* Hm, const double* sigma,
                      const double* X0, double scale, const double* tolv, double* Vt, double* rq, hipStream_t s);
// Rayleigh quotients and residual norms of the columns of an orthonormal Vt
void launch_small_rr(int nH, int k, const double* theta, const double* Gt, const double* Hm, const double* Vt,
                     double* rq, double* res, hipStream_t s);
// acceptance: residuals <= tol_abs (times tolv[r] for the pair at position r of the ascending
// order when tolv is given) and the inertia count below max(rq) + gap equals k (or, failing that,
// the count below the nev-th value + gap equals nev: the wanted pairs certified, status[0] = 2);
// writes lam ascending, perm, status[0] (0 rejected) and status[1] (the count)
void launch_small_accept(int nH, int k, int nev, const double* theta, const double* Gt, const double* Hm,
                         const double* rq, const double* res, double tol_abs, const double* tolv, double gap,
                         double* lam, int* perm, int* status, hipStream_t s);
// principal block of Tt on the first m coarse modes and the k W-directions ((m + k)^2, row-major),
// and the zero extension of its eigenvectors ((m + k) x k) to start vectors ((nH + k) x k)
void launch_small_principal(int nH, int m, int k, const double* theta, const double* Gt, const double* Hm,
                            double* Tr, hipStream_t s);
void launch_small_expand(int nH, int m, int k, const double* Vr, double* X0, hipStream_t s);
// V (n x k row-major) = columns perm of Vt
void launch_small_emit(int n, int k, const double* Vt, const int* perm, double* V, hipStream_t s);
void launch_symmetrize(int n, double* A, hipStream_t s);

// ---- the same structured solver for large coarse spaces (small_big.hip): N_H <= small_big_max_nh(),
// k <= small_big_max_k(); rows of Gt stream from L2, each pair keeps two work vectors in `scratch`
// (small_big_scratch_doubles)
int small_big_max_k();
int small_big_max_nh();
size_t small_big_scratch_doubles(int nH, int k);
void launch_small_rqi_big(int nH, int k, const double* theta, const double* Gt, const double* Hm,
                          const double* sigma, const double* X0, double scale, const double* tolv, double* Vt,
                          double* rq, double* scratch, hipStream_t s);
void launch_small_rr_big(int nH, int k, const double* theta, const double* Gt, const double* Hm, const double* Vt,
                         double* rq, double* res, double* scratch, hipStream_t s);
void launch_small_accept_big(int nH, int k, int nev, const double* theta, const double* Gt, const double* Hm,
                             const double* rq, const double* res, double tol_abs, const double* tolv, double gap,
                             double* lam, int* perm, int* status, double* scratch, hipStream_t s);

}  // namespace pase
