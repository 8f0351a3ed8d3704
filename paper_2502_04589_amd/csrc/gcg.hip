// Kernels of the GCG_AUG path (Sec. 4, Alg. 4 and 5): products of tall blocks of different
// widths, the residual and right-hand sides of the augmented pairs, and the assembly of the
// Rayleigh-Ritz matrix.  The driver is in pase.hip.
//
// Layout: an augmented block is (N_H + k) x w row-major -- row i < N_H is coarse node i of V_H,
// the last k rows are the coordinates along the k fine directions -- so the coarse part is an
// ordinary N_H x w multi-vector that the coarse stencils apply to, and every product over all
// rows is one tall-skinny product.
#include "internal.hpp"

namespace pase {
namespace {

constexpr int kTnTile = 64;      // output tile (rows and columns of C) per block
constexpr int kTnRows = 16;      // rows of A and B staged per step
constexpr int kTnMaxTiles = 128; // row chunks (partial sums) at most

// Partial C_t = A[rows_t]^T B[rows_t] for one 64 x 64 tile of C: 256 threads as 16 x 16, each
// accumulating a 4 x 4 block; rows staged through LDS in groups of 16 (coalesced row reads).
__global__ __launch_bounds__(256) void gram_tn_kernel(long long N, int m, int n, const double* __restrict__ A,
                                                      int lda, const double* __restrict__ B, int ldb,
                                                      double* __restrict__ partial, long long rows) {
  __shared__ double sa[kTnRows][kTnTile + 1];
  __shared__ double sb[kTnRows][kTnTile + 1];
  const int t = blockIdx.x;
  const int i0 = blockIdx.y * kTnTile, j0 = blockIdx.z * kTnTile;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const long long r0 = (long long)t * rows;
  const long long r1 = (r0 + rows < N) ? r0 + rows : N;
  double acc[4][4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int p = 0; p < 4; ++p) acc[q][p] = 0.0;
  for (long long r = r0; r < r1; r += kTnRows) {
    for (int e = threadIdx.x; e < kTnRows * kTnTile; e += 256) {
      const int rr = e / kTnTile, cc = e % kTnTile;
      const long long row = r + rr;
      const bool in = row < r1;
      sa[rr][cc] = (in && i0 + cc < m) ? A[row * lda + i0 + cc] : 0.0;
      sb[rr][cc] = (in && j0 + cc < n) ? B[row * ldb + j0 + cc] : 0.0;
    }
    __syncthreads();
#pragma unroll 4
    for (int rr = 0; rr < kTnRows; ++rr) {
      double a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) a[q] = sa[rr][ty + 16 * q];
#pragma unroll
      for (int p = 0; p < 4; ++p) b[p] = sb[rr][tx + 16 * p];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int p = 0; p < 4; ++p) acc[q][p] = fma(a[q], b[p], acc[q][p]);
    }
    __syncthreads();
  }
  double* out = partial + (size_t)t * m * n;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int p = 0; p < 4; ++p) {
      const int i = i0 + ty + 16 * q, j = j0 + tx + 16 * p;
      if (i < m && j < n) out[(size_t)i * n + j] = acc[q][p];
    }
}

// R = AX - BX diag(lam)
__global__ void aug_resid_kernel(long long N, int k, const double* __restrict__ AX, const double* __restrict__ BX,
                                 const double* __restrict__ lam, double* __restrict__ R) {
  const long long n = N * k;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const int j = (int)(e % k);
    R[e] = AX[e] - BX[e] * lam[j];
  }
}

// dst (N x ka) column j = src (N x k) column idx[j], times lam[idx[j]] when lam is given
__global__ void gather_scale_kernel(long long N, int k, int ka, const int* __restrict__ idx,
                                    const double* __restrict__ src, const double* __restrict__ lam,
                                    double* __restrict__ dst) {
  const long long n = N * ka;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const long long i = e / ka;
    const int j = idx[(int)(e % ka)];
    dst[e] = src[i * k + j] * (lam ? lam[j] : 1.0);
  }
}

// Start block [a_hat ; I] (rows N_H .. N_H + k hold the identity)
__global__ void aug_start_kernel(long long NH, int k, const double* __restrict__ ahat, double* __restrict__ X) {
  const long long n = (NH + k) * k;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x) {
    const long long i = e / k;
    const int j = (int)(e % k);
    X[e] = (i < NH) ? ahat[e] : ((i - NH == j) ? 1.0 : 0.0);
  }
}

// H (n x n, n = k + ny) = [[Gxx, Gxy], [Gxy^T, Gyy]] with both diagonal blocks symmetrised
__global__ void assemble_rr_kernel(int k, int ny, const double* __restrict__ Gxx, const double* __restrict__ Gxy,
                                   const double* __restrict__ Gyy, double* __restrict__ H) {
  const int n = k + ny;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n * n; e += gridDim.x * blockDim.x) {
    const int i = e / n, j = e % n;
    double v;
    if (i < k && j < k) v = 0.5 * (Gxx[i * k + j] + Gxx[j * k + i]);
    else if (i < k) v = Gxy[i * ny + (j - k)];
    else if (j < k) v = Gxy[j * ny + (i - k)];
    else v = 0.5 * (Gyy[(i - k) * ny + (j - k)] + Gyy[(j - k) * ny + (i - k)]);
    H[e] = v;
  }
}

// C = Li^T Li (k x k) for the lower Li: the inverse of an SPD matrix from its inverted factor
__global__ void ltl_kernel(int k, const double* __restrict__ Li, double* __restrict__ C) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < k * k; e += gridDim.x * blockDim.x) {
    const int i = e / k, j = e % k;
    const int r0 = i > j ? i : j;
    double s = 0.0;
    for (int r = r0; r < k; ++r) s = fma(Li[r * k + i], Li[r * k + j], s);
    C[e] = s;
  }
}

// c = a - b (n values); a zero fill when a and b are both null
__global__ void sub_kernel(long long n, const double* __restrict__ a, const double* __restrict__ b,
                           double* __restrict__ c) {
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n; e += (long long)gridDim.x * blockDim.x)
    c[e] = (a ? a[e] : 0.0) - (b ? b[e] : 0.0);
}

// d[j] = 1 / sqrt(G_jj) (the smallest positive double when G_jj <= 0)
__global__ void inv_sqrt_diag_kernel(int n, const double* __restrict__ G, double* __restrict__ d) {
  for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < n; j += gridDim.x * blockDim.x) {
    const double g = G[(size_t)j * n + j];
    d[j] = 1.0 / sqrt(g > 2.2250738585072014e-308 ? g : 2.2250738585072014e-308);
  }
}

// G <- D G D (rows and columns scaled by d); with cols_only, only the columns: M <- M D
__global__ void scale_sym_kernel(int n, double* __restrict__ G, const double* __restrict__ d, int cols_only) {
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < n * n; e += gridDim.x * blockDim.x) {
    const int i = e / n, j = e % n;
    G[e] *= cols_only ? d[j] : d[i] * d[j];
  }
}

inline unsigned grid_for(long long n) {
  long long b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  return (unsigned)(b < 1 ? 1 : b);
}

int tn_tiles(long long N) {
  long long t = (N + 255) / 256;
  if (t > kTnMaxTiles) t = kTnMaxTiles;
  return (int)(t < 1 ? 1 : t);
}

}  // namespace

size_t gram_tn_partial_doubles(long long N, int m, int n) { return (size_t)tn_tiles(N) * m * n; }

void launch_gram_tn(long long N, int m, int n, const double* A, int lda, const double* B, int ldb, double* partial,
                    double* C, hipStream_t s) {
  if (m <= 0 || n <= 0) return;
  const int tiles = tn_tiles(N);
  long long rows = (N + tiles - 1) / tiles;
  rows = ((rows + kTnRows - 1) / kTnRows) * kTnRows;
  const dim3 grid((unsigned)tiles, (unsigned)((m + kTnTile - 1) / kTnTile), (unsigned)((n + kTnTile - 1) / kTnTile));
  gram_tn_kernel<<<grid, 256, 0, s>>>(N, m, n, A, lda, B, ldb, partial, rows);
  launch_reduce_partials(tiles, m * n, partial, C, s);
}

void launch_aug_resid(long long N, int k, const double* AX, const double* BX, const double* lam, double* R,
                      hipStream_t s) {
  aug_resid_kernel<<<grid_for(N * k), 256, 0, s>>>(N, k, AX, BX, lam, R);
}

void launch_gather_scale(long long N, int k, int ka, const int* idx, const double* src, const double* lam,
                         double* dst, hipStream_t s) {
  gather_scale_kernel<<<grid_for(N * ka), 256, 0, s>>>(N, k, ka, idx, src, lam, dst);
}

void launch_aug_start(long long NH, int k, const double* ahat, double* X, hipStream_t s) {
  aug_start_kernel<<<grid_for((NH + k) * k), 256, 0, s>>>(NH, k, ahat, X);
}

void launch_assemble_rr(int k, int ny, const double* Gxx, const double* Gxy, const double* Gyy, double* H,
                        hipStream_t s) {
  const int n = k + ny;
  assemble_rr_kernel<<<grid_for((long long)n * n), 256, 0, s>>>(k, ny, Gxx, Gxy, Gyy, H);
}

void launch_unit_diag(int n, double* G, double* d, hipStream_t s) {
  inv_sqrt_diag_kernel<<<grid_for(n), 256, 0, s>>>(n, G, d);
  scale_sym_kernel<<<grid_for((long long)n * n), 256, 0, s>>>(n, G, d, 0);
}

void launch_scale_cols_sq(int n, double* M, const double* d, hipStream_t s) {
  scale_sym_kernel<<<grid_for((long long)n * n), 256, 0, s>>>(n, M, d, 1);
}

void launch_sub(long long n, const double* a, const double* b, double* c, hipStream_t s) {
  sub_kernel<<<grid_for(n), 256, 0, s>>>(n, a, b, c);
}

void launch_ltl(int k, const double* Li, double* C, hipStream_t s) {
  ltl_kernel<<<grid_for((long long)k * k), 256, 0, s>>>(k, Li, C);
}

}  // namespace pase
