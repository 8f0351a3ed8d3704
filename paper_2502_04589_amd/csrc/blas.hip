// Multi-vector BLAS kernels: per-column dot products (CG scalars), fused CG
// updates, the tall-skinny Gram products W^T (A W), W^T (M W) on FP64 MFMA,
// and a tiled FP64 GEMM for the small dense products.  Every reduction is a
// fixed-order tree over fixed row tiles, so results are bitwise reproducible.
#include "internal.hpp"

namespace pase {

namespace {

typedef double double4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ int xcd_tile(int b, int nblocks) {
  const int per = nblocks >> 3;
  return (b & 7) * per + (b >> 3);
}

constexpr int kColdotPasses = 16;

// partial[tile][j] = sum over the tile's rows of X[i,j] * Y[i,j]
template <typename T>
__global__ __launch_bounds__(kBlock) void coldot_kernel(long long N, int k, const T* __restrict__ X,
                                                        const T* __restrict__ Y, double* __restrict__ partial,
                                                        int tiles, int rows) {
  __shared__ double red[kBlock];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= tiles) return;
  const int slots = kBlock / k;
  const int col = threadIdx.x % k;
  const int slot = threadIdx.x / k;
  const long long r0 = (long long)tile * rows;
  const long long r1 = (r0 + rows < N) ? (r0 + rows) : N;
  double acc = 0.0;
  if (slot < slots)
    for (long long r = r0 + slot; r < r1; r += slots) acc = fma((double)X[r * k + col], (double)Y[r * k + col], acc);
  red[threadIdx.x] = acc;
  __syncthreads();
  if ((int)threadIdx.x < k) {
    double s = 0.0;
    for (int q = 0; q < slots; ++q) s += red[q * k + threadIdx.x];
    partial[(size_t)tile * k + threadIdx.x] = s;
  }
}

// out[j] = sum_t partial[t][j], one block per output, fixed order
__global__ __launch_bounds__(kBlock) void reduce_partials_kernel(int tiles, int width,
                                                                 const double* __restrict__ partial,
                                                                 double* __restrict__ out) {
  __shared__ double red[kBlock];
  const int j = blockIdx.x;
  double s = 0.0;
  for (int t = threadIdx.x; t < tiles; t += kBlock) s += partial[(size_t)t * width + j];
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = kBlock / 2; w > 0; w >>= 1) {
    if (threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) out[j] = red[0];
}

__global__ void pcg_alpha_kernel(int k, const double* rho, const double* pq, double* alpha) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  const double d = pq[j];
  alpha[j] = (d > 0.0) ? rho[j] / d : 0.0;
}

__global__ void pcg_beta_kernel(int k, const double* rn, const double* ro, double* beta) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  const double d = ro[j];
  beta[j] = (d != 0.0) ? rn[j] / d : 0.0;
}

// Learned-PCG column state: 1 = on the network, 2 = switched to the V-cycle in this step,
// 0 = on the V-cycle.
//
// flexible PCG: beta = (r+^T z+ - r+^T z) / (r^T z); 0 for a column that switched in this step
// (the recurrence restarts there), whose state then becomes 0
__global__ void flex_beta_kernel(int k, const double* a, const double* b, const double* c, int* mask,
                                 double* beta) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  const double d = c[j];
  double v = (d != 0.0) ? (a[j] - b[j]) / d : 0.0;
  if (mask[j] == 2) {
    v = 0.0;
    mask[j] = 0;
  }
  beta[j] = v;
}

// learned-PCG fallback: a column keeps the network while ||r+||^2 <= ratio^2 ||r||^2
__global__ void fallback_kernel(int k, double ratio2, const double* rn, const double* ro, int* mask) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= k) return;
  if (mask[j] == 1 && !(rn[j] <= ratio2 * ro[j])) mask[j] = 2;
}

// Z[:, j] = (mask[j] == 1) ? A[:, j] : Z[:, j]
// Column gather / scatter of node-major blocks: C (N x ka) <-> the columns idx[0..ka) of B (N x k).
__global__ void gather_cols_kernel(long long N, int k, int ka, const int* __restrict__ idx,
                                   const double* __restrict__ B, double* __restrict__ C) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= N * ka) return;
  const long long n = q / ka;
  C[q] = B[n * k + idx[q - n * ka]];
}

// B (N x k): column j of U where pos[j] < 0, else column pos[j] of C (N x ka), in one pass (the
// soft-locked block with the fine solves of its active columns)
__global__ void merge_cols_kernel(long long N, int k, int ka, const int* __restrict__ pos, const double* __restrict__ C,
                                  const double* __restrict__ U, double* __restrict__ B) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= N * k) return;
  const long long n = q / k;
  const int p = pos[q - n * k];
  B[q] = (p >= 0) ? C[n * ka + p] : U[q];
}

__global__ void scatter_cols_kernel(long long N, int k, int ka, const int* __restrict__ idx,
                                    const double* __restrict__ C, double* __restrict__ B) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= N * ka) return;
  const long long n = q / ka;
  B[n * k + idx[q - n * ka]] = C[q];
}

// dst (N x kout) columns 0..nc) = src (N x kin) columns 0..nc); with fill, the columns nc..kout) of
// dst get a counter-based uniform(-1, 1) value of (node, column): the 64-bit finaliser of
// SplitMix64 (Steele, Lea and Flood 2014) applied to node * kout + column, top 53 bits.
__global__ void copy_cols_kernel(long long N, int kin, int kout, int nc, const double* __restrict__ src,
                                 double* __restrict__ dst, int fill) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= N * kout) return;
  const long long n = q / kout;
  const int j = (int)(q - n * kout);
  if (j < nc) {
    dst[q] = src[n * kin + j];
  } else if (fill) {
    unsigned long long z = (unsigned long long)q + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z = z ^ (z >> 31);
    dst[q] = 2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
  }
}

__global__ void select_cols_kernel(long long N, int k, const int* __restrict__ mask, const double* __restrict__ A,
                                   double* __restrict__ Z) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * k) return;
  if (mask[i % k] == 1) Z[i] = A[i];
}

__global__ void fill_int_kernel(int n, int v, int* p) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) p[j] = v;
}

template <typename T>
__global__ void axpy2_kernel(long long N, int k, const double* __restrict__ alpha, const T* __restrict__ P,
                             const T* __restrict__ Q, const T* Xin, T* X, T* __restrict__ R) {
  // X = Xin + alpha P (Xin may be X), R -= alpha Q (R null: the x update only)
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * k) return;
  const double a = alpha[i % k];
  X[i] = (T)fma(a, (double)P[i], (double)Xin[i]);
  if (R) R[i] = (T)fma(-a, (double)Q[i], (double)R[i]);
}

// Two CG steps with the first x update folded into the second: R -= alpha Q; Z += beta P;
// X = X0 + a0 P + a1 Z (per-column scalars)
__global__ void rsub_kernel(long long N, int k, const double* __restrict__ alpha, const double* __restrict__ Q,
                            double* __restrict__ R) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * k) return;
  R[i] = fma(-alpha[i % k], Q[i], R[i]);
}

__global__ void zadd_kernel(long long N, int k, const double* __restrict__ beta, const double* __restrict__ P,
                            double* __restrict__ Z) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * k) return;
  Z[i] = fma(beta[i % k], P[i], Z[i]);
}

__global__ void axpy3_kernel(long long N, int k, const double* __restrict__ a0, const double* __restrict__ P,
                             const double* __restrict__ a1, const double* __restrict__ Z, const double* X0,
                             double* X) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * k) return;
  const int j = (int)(i % k);
  X[i] = fma(a1[j], Z[i], fma(a0[j], P[i], X0[i]));
}

// The same x update as one pass over full blocks (leading dimension ldx): column j of X is
// X0 + a0 p + a1 z for the active columns (pos[j] = its position among the k solved ones) and X0 for
// the locked ones, so whole node rows are read and written
__global__ void axpy3_merge_kernel(long long N, int k, int ldx, const int* __restrict__ pos,
                                   const double* __restrict__ a0, const double* __restrict__ P,
                                   const double* __restrict__ a1, const double* __restrict__ Z,
                                   const double* __restrict__ X0, double* __restrict__ X) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= N * ldx) return;
  const long long n = q / ldx;
  const int a = pos[q - n * ldx];
  double v = X0[q];
  if (a >= 0) {
    const long long e = n * k + a;
    v = fma(a1[a], Z[e], fma(a0[a], P[e], v));
  }
  X[q] = v;
}

template <typename T>
__global__ void xpby_kernel(long long N, int k, const T* __restrict__ Z, const double* __restrict__ beta,
                            T* __restrict__ P) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * k) return;
  P[i] = (T)fma(beta[i % k], (double)P[i], (double)Z[i]);
}

__global__ void d2f_kernel(size_t n, const double* __restrict__ a, float* __restrict__ b) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (float)a[i];
}

// start of the correction-form CG: r = (float)R, e = 0
__global__ void cg_start_f32_kernel(size_t n, const double* __restrict__ R, float* __restrict__ r,
                                    float* __restrict__ e) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    r[i] = (float)R[i];
    e[i] = 0.0f;
  }
}

__global__ void copy_f32_kernel(size_t n, const float* __restrict__ s, float* __restrict__ d) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = s[i];
}

__global__ void add_f2d_kernel(size_t n, const double* __restrict__ u, const float* __restrict__ e,
                               double* __restrict__ w) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) w[i] = u[i] + (double)e[i];
}

// w = u + e over full rows (leading dimension ldw), e taken from column pos[j] of its k-column block
// where pos[j] >= 0 (the soft-locked columns are u itself)
__global__ void add_f2d_merge_kernel(long long N, int k, int ldw, const int* __restrict__ pos,
                                     const double* __restrict__ u, const float* __restrict__ e,
                                     double* __restrict__ w) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= N * ldw) return;
  const long long n = q / ldw;
  const int a = pos[q - n * ldw];
  w[q] = (a >= 0) ? u[q] + (double)e[n * k + a] : u[q];
}

__global__ void copy_kernel(size_t n, const double* __restrict__ s, double* __restrict__ d) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) d[i] = s[i];
}

// ---- Gram G = X^T Y on v_mfma_f64_16x16x4f64.
// Operand layout of the 16x16x4 f64 MFMA (wave64): lane l supplies
// A[l%16][l/16] and B[l/16][l%16]; accumulator register q of lane l holds
// D[l/16 + 4q][l%16] (checked on gfx950 by the Gram parity test).  Here A = X^T restricted to 16 columns of X and 4 rows,
// B = Y restricted to 4 rows and 16 columns.
constexpr int kGramMaxTilesPerWave = 16;

__global__ __launch_bounds__(kBlock) void gram_kernel(long long N, int k, const double* __restrict__ X,
                                                      const double* __restrict__ Y, double* __restrict__ partial,
                                                      int tiles, long long rows) {
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= tiles) return;
  const int wave = threadIdx.x >> 6;
  const int lane = threadIdx.x & 63;
  const int T = (k + 15) >> 4;
  const int TT = T * T;
  const long long r0 = (long long)tile * rows;
  const long long r1 = (r0 + rows < N) ? (r0 + rows) : N;
  double4_t acc[kGramMaxTilesPerWave];
#pragma unroll
  for (int t = 0; t < kGramMaxTilesPerWave; ++t) acc[t] = (double4_t){0.0, 0.0, 0.0, 0.0};
  const int li = lane & 15;   // column within a 16-wide tile
  const int lk = lane >> 4;   // row within the 4-row step
  for (long long r = r0; r < r1; r += 4) {
    const long long row = r + lk;
    const bool rok = row < r1;
#pragma unroll
    for (int t = 0; t < kGramMaxTilesPerWave; ++t) {
      const int tt = wave + 4 * t;
      if (tt < TT) {
        const int ti = tt / T, tj = tt % T;
        const int ca = ti * 16 + li, cb = tj * 16 + li;
        const double av = (rok && ca < k) ? X[row * k + ca] : 0.0;
        const double bv = (rok && cb < k) ? Y[row * k + cb] : 0.0;
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
      }
    }
  }
  double* p = partial + (size_t)tile * k * k;
#pragma unroll
  for (int t = 0; t < kGramMaxTilesPerWave; ++t) {
    const int tt = wave + 4 * t;
    if (tt < TT) {
      const int ti = tt / T, tj = tt % T;
      const int j = tj * 16 + li;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = ti * 16 + lk + 4 * q;
        if (i < k && j < k) p[(size_t)i * k + j] = acc[t][q];
      }
    }
  }
}

// ---- LDS-staged Gram: G_y = X^T Y_y for NY = 1 or 2 right-hand blocks (X read once).
// Each block owns a contiguous run of rows and walks it in chunks of kGramRows
// rows.  A chunk of X and Y_y is a contiguous run of kGramRows * k doubles: the
// block loads it with coalesced loads into registers one chunk ahead, stores it
// to LDS (zero-padded to 16-column tiles), and its four waves feed the MFMA
// tiles from LDS.  Partial k x k sums per block are reduced in a fixed order.
constexpr int kGramRows = 32;

template <int NY, int KMAX>
__global__ __launch_bounds__(kBlock) void gram_lds_kernel(long long N, int k, const double* __restrict__ X,
                                                          const double* __restrict__ Y1,
                                                          const double* __restrict__ Y2,
                                                          double* __restrict__ partial, int tiles, long long rows) {
  constexpr int TMAX = (KMAX / 16) * (KMAX / 16) / 4;   // tiles per wave
  constexpr int U = kGramRows * KMAX / kBlock;          // staged doubles per thread per matrix
  extern __shared__ double lds[];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= tiles) return;
  const int T = (k + 15) >> 4, TT = T * T;
  const int LD = T * 16 + 1;
  double* xs = lds;
  double* y1s = xs + kGramRows * LD;
  double* y2s = y1s + kGramRows * LD;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int e = tid; e < (1 + NY) * kGramRows * LD; e += kBlock) lds[e] = 0.0;
  const long long r0 = (long long)tile * rows;
  const long long r1 = (r0 + rows < N) ? (r0 + rows) : N;
  const int ck = kGramRows * k;
  // per-thread slots of a chunk: element e = tid + kBlock u -> (row e / k, col e % k)
  int soff[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = tid + kBlock * u;
    const int rr = e / k;
    soff[u] = (e < ck) ? rr * LD + (e - rr * k) : -1;
  }
  double rx[U], ry1[U], ry2[U];
  auto fetch = [&](long long rc) {
    const long long lim = (r1 - rc) * k;      // valid elements of this chunk
    const unsigned nval = (unsigned)((lim < ck) ? lim : ck);
    const double* __restrict__ px = X + rc * k;
    const double* __restrict__ py1 = Y1 + rc * k;
    const double* __restrict__ py2 = (NY == 2) ? Y2 + rc * k : Y1 + rc * k;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const unsigned e = (unsigned)(tid + kBlock * u);
      const bool ok = e < nval;
      rx[u] = ok ? px[e] : 0.0;
      ry1[u] = ok ? py1[e] : 0.0;
      if (NY == 2) ry2[u] = ok ? py2[e] : 0.0;
    }
  };
  double4_t acc1[TMAX], acc2[TMAX];
#pragma unroll
  for (int t = 0; t < TMAX; ++t) {
    acc1[t] = (double4_t){0.0, 0.0, 0.0, 0.0};
    acc2[t] = (double4_t){0.0, 0.0, 0.0, 0.0};
  }
  const int li = lane & 15, lk = lane >> 4;
  if (r0 < r1) fetch(r0);
  __syncthreads();
  for (long long rc = r0; rc < r1; rc += kGramRows) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (soff[u] >= 0) {
        xs[soff[u]] = rx[u];
        y1s[soff[u]] = ry1[u];
        if (NY == 2) y2s[soff[u]] = ry2[u];
      }
    }
    __syncthreads();
    if (rc + kGramRows < r1) fetch(rc + kGramRows);
#pragma unroll 2
    for (int st = 0; st < kGramRows / 4; ++st) {
      const int row = (4 * st + lk) * LD;
#pragma unroll
      for (int t = 0; t < TMAX; ++t) {
        const int tt = wave + 4 * t;
        if (tt < TT) {
          const int ti = tt / T, tj = tt - (tt / T) * T;
          const double av = xs[row + ti * 16 + li];
          acc1[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, y1s[row + tj * 16 + li], acc1[t], 0, 0, 0);
          if (NY == 2)
            acc2[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, y2s[row + tj * 16 + li], acc2[t], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int y = 0; y < NY; ++y) {
    double* p = partial + ((size_t)y * tiles + tile) * k * k;
#pragma unroll
    for (int t = 0; t < TMAX; ++t) {
      const int tt = wave + 4 * t;
      if (tt < TT) {
        const int ti = tt / T, tj = tt - (tt / T) * T;
        const int j = tj * 16 + li;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = ti * 16 + lk + 4 * q;
          if (i < k && j < k) p[(size_t)i * k + j] = (y == 0) ? acc1[t][q] : acc2[t][q];
        }
      }
    }
  }
}

// ---- symmetric Grams for 64 < k <= 128: G_y = X^T Y_y (NY = 1 or 2) when every G_y is symmetric
// (the projection's W^T A W and W^T M W, the Cholesky-QR Gram U^T M U).  Only the T(T+1)/2 upper
// 16 x 16 tiles are multiplied (T = ceil(k / 16)); each writes its entries and their mirror
// images into the block's partial, so the fixed-order reduction gives the full symmetric matrix.
// Eight waves share the upper tiles (at most 5 each); the block walks its rows in 32-row chunks
// staged in LDS exactly like gram_lds_kernel, X read once for both products.
constexpr int kSymThreads = 512;
constexpr int kSymTiles = 5;       // ceil(36 / 8)

template <int NY>
__global__ __launch_bounds__(kSymThreads) void gram_sym_kernel(long long N, int k, const double* __restrict__ X,
                                                             const double* __restrict__ Y1,
                                                             const double* __restrict__ Y2,
                                                             double* __restrict__ partial, int tiles,
                                                             long long rows) {
  constexpr int KMAX = 128;
  constexpr int U = kGramRows * KMAX / kSymThreads;       // staged doubles per thread per matrix
  extern __shared__ double lds[];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= tiles) return;
  const int T = (k + 15) >> 4;
  const int LD = T * 16 + 1;
  double* xs = lds;
  double* y1s = xs + kGramRows * LD;
  double* y2s = y1s + kGramRows * LD;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int e = tid; e < (1 + NY) * kGramRows * LD; e += kSymThreads) lds[e] = 0.0;
  // this wave's upper tiles: q = wave + 8 t enumerates (ti, tj), ti <= tj, row by row
  int ta[kSymTiles], tb[kSymTiles];
#pragma unroll
  for (int t = 0; t < kSymTiles; ++t) {
    int q = wave + 8 * t, i = 0;
    while (i < T && q >= T - i) {
      q -= T - i;
      ++i;
    }
    ta[t] = (i < T) ? i : -1;
    tb[t] = (i < T) ? i + q : 0;
  }
  const long long r0 = (long long)tile * rows;
  const long long r1 = (r0 + rows < N) ? (r0 + rows) : N;
  const int ck = kGramRows * k;
  int soff[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int e = tid + kSymThreads * u;
    const int rr = e / k;
    soff[u] = (e < ck) ? rr * LD + (e - rr * k) : -1;
  }
  double rx[U], ry1[U], ry2[U];
  auto fetch = [&](long long rc) {
    const long long lim = (r1 - rc) * k;
    const unsigned nval = (unsigned)((lim < ck) ? lim : ck);
    const double* __restrict__ px = X + rc * k;
    const double* __restrict__ py1 = Y1 + rc * k;
    const double* __restrict__ py2 = (NY == 2) ? Y2 + rc * k : Y1 + rc * k;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const unsigned e = (unsigned)(tid + kSymThreads * u);
      const bool ok = e < nval;
      rx[u] = ok ? px[e] : 0.0;
      ry1[u] = ok ? py1[e] : 0.0;
      if (NY == 2) ry2[u] = ok ? py2[e] : 0.0;
    }
  };
  double4_t acc1[kSymTiles], acc2[kSymTiles];
#pragma unroll
  for (int t = 0; t < kSymTiles; ++t) {
    acc1[t] = (double4_t){0.0, 0.0, 0.0, 0.0};
    acc2[t] = (double4_t){0.0, 0.0, 0.0, 0.0};
  }
  const int li = lane & 15, lk = lane >> 4;
  if (r0 < r1) fetch(r0);
  __syncthreads();
  for (long long rc = r0; rc < r1; rc += kGramRows) {
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if (soff[u] >= 0) {
        xs[soff[u]] = rx[u];
        y1s[soff[u]] = ry1[u];
        if (NY == 2) y2s[soff[u]] = ry2[u];
      }
    }
    __syncthreads();
    if (rc + kGramRows < r1) fetch(rc + kGramRows);
#pragma unroll 2
    for (int st = 0; st < kGramRows / 4; ++st) {
      const int row = (4 * st + lk) * LD;
#pragma unroll
      for (int t = 0; t < kSymTiles; ++t) {
        if (ta[t] >= 0) {
          const double av = xs[row + ta[t] * 16 + li];
          acc1[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, y1s[row + tb[t] * 16 + li], acc1[t], 0, 0, 0);
          if (NY == 2)
            acc2[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, y2s[row + tb[t] * 16 + li], acc2[t], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int y = 0; y < NY; ++y) {
    double* p = partial + ((size_t)y * tiles + tile) * k * k;
#pragma unroll
    for (int t = 0; t < kSymTiles; ++t) {
      if (ta[t] >= 0) {
        const int j = tb[t] * 16 + li;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = ta[t] * 16 + lk + 4 * q;
          const double v = (y == 0) ? acc1[t][q] : acc2[t][q];
          if (i < k && j < k) {
            p[(size_t)i * k + j] = v;
            if (ta[t] != tb[t]) p[(size_t)j * k + i] = v;
          }
        }
      }
    }
  }
}

// ---- split-BF16 Gram of FP32 operands: G_y = X^T Y_y (NY = 1 or 2, k <= KMAX = 64 or 128) on
// v_mfma_f32_16x16x32_bf16.  Each FP32 value is split as x = x_hi + x_lo with x_hi = bf16(x) and
// x_lo = bf16(x - x_hi); a product is formed as x_hi y_hi + x_hi y_lo + x_lo y_hi (the dropped
// x_lo y_lo is below 2^-16 |x y|).  The three MFMAs accumulate in FP32 over a K-block of 256 rows,
// which is then added to an FP64 accumulator; the per-block partials are reduced in FP64 in a fixed
// order.  A block walks its rows in 32-row chunks (one MFMA k-step): the chunk of each operand is a
// contiguous run of 32 k floats, loaded with coalesced accesses and stored split and transposed in
// LDS ([column][row], so a lane's 8 consecutive rows are one 16-byte read).  Operand layout of the
// instruction: lane l supplies A[l%16][8(l/16) .. +7] and B[8(l/16) .. +7][l%16]; accumulator
// register q holds D[4(l/16) + q][l%16].  KMAX = 64: four waves, four 16 x 16 tiles each; KMAX = 128:
// eight waves, eight tiles each.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float float4_t __attribute__((ext_vector_type(4)));
constexpr int kG3Rows = 32;                    // rows per chunk = K of one MFMA
constexpr int kG3Rs = kG3Rows + 8;             // LDS row stride of a column (bf16 elements)
constexpr int kG3Flush = 8;                    // chunks per FP32 K-block (256 rows)

template <int NY, int KMAX>
__global__ __launch_bounds__(KMAX * 4) void gram_bf16x3_kernel(long long N, int k, const float* __restrict__ X,
                                                               const float* __restrict__ Y1,
                                                               const float* __restrict__ Y2,
                                                               double* __restrict__ partial, int tiles,
                                                               long long rows) {
  constexpr int NT = KMAX * 4;                          // threads
  constexpr int NW = NT / 64;                           // waves
  constexpr int TPW = (KMAX / 16) * (KMAX / 16) / NW;   // tiles per wave
  constexpr int kG3SE = kG3Rows * KMAX / NT;            // staged values per thread per operand
  // [operand (X, Y1, Y2)][hi, lo][column 0..KMAX-1][row]
  __shared__ __align__(16) __bf16 st[1 + NY][2][KMAX * kG3Rs];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= tiles) return;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int T = (k + 15) >> 4, TT = T * T;
  for (int e = tid; e < (1 + NY) * 2 * KMAX * kG3Rs; e += NT) (&st[0][0][0])[e] = (__bf16)0.0f;
  const long long r0 = (long long)tile * rows;
  const long long r1 = (r0 + rows < N) ? (r0 + rows) : N;
  const int ck = kG3Rows * k;
  int soff[kG3SE];   // LDS slot (column * kG3Rs + row) of each staged value; independent of the chunk
#pragma unroll
  for (int u = 0; u < kG3SE; ++u) {
    const int e = tid + NT * u;
    const int r = e / k;
    soff[u] = (e < ck) ? (e - r * k) * kG3Rs + r : -1;
  }
  float4_t acc1[TPW], acc2[TPW];
  double4_t dacc1[TPW], dacc2[TPW];
#pragma unroll
  for (int t = 0; t < TPW; ++t) {
    acc1[t] = acc2[t] = (float4_t){0.f, 0.f, 0.f, 0.f};
    dacc1[t] = dacc2[t] = (double4_t){0.0, 0.0, 0.0, 0.0};
  }
  const int li = lane & 15, g = lane >> 4;
  int nchunk = 0;
  for (long long rc = r0; rc < r1; rc += kG3Rows) {
    const long long lim = (r1 - rc) * k;
    const int nval = (int)((lim < ck) ? lim : ck);
    float v[1 + NY][kG3SE];
#pragma unroll
    for (int u = 0; u < kG3SE; ++u) {   // clamped, unconditional loads: all in flight together
      const int e = tid + NT * u;
      const long long ec = rc * k + ((e < nval) ? e : nval - 1);
      v[0][u] = X[ec];
      v[1][u] = Y1[ec];
      if (NY == 2) v[2][u] = Y2[ec];
    }
    __syncthreads();   // the previous chunk's operands have been read
#pragma unroll
    for (int u = 0; u < kG3SE; ++u) {
      const int e = tid + NT * u;
      if (soff[u] >= 0) {
#pragma unroll
        for (int m = 0; m < 1 + NY; ++m) {
          const float x = (e < nval) ? v[m][u] : 0.0f;   // rows past the block's range are zero
          const __bf16 hi = (__bf16)x;
          st[m][0][soff[u]] = hi;
          st[m][1][soff[u]] = (__bf16)(x - (float)hi);
        }
      }
    }
    __syncthreads();
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int tt = wave + NW * t;
      if (tt < TT) {
        const int ti = tt / T, tj = tt - (tt / T) * T;
        const int ca = (16 * ti + li) * kG3Rs + 8 * g, cb = (16 * tj + li) * kG3Rs + 8 * g;
        const bf16x8_t ah = *(const bf16x8_t*)&st[0][0][ca], al = *(const bf16x8_t*)&st[0][1][ca];
        const bf16x8_t bh = *(const bf16x8_t*)&st[1][0][cb], bl = *(const bf16x8_t*)&st[1][1][cb];
        acc1[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bh, acc1[t], 0, 0, 0);
        acc1[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, bl, acc1[t], 0, 0, 0);
        acc1[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, bh, acc1[t], 0, 0, 0);
        if (NY == 2) {
          const bf16x8_t ch = *(const bf16x8_t*)&st[2][0][cb], cl = *(const bf16x8_t*)&st[2][1][cb];
          acc2[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, ch, acc2[t], 0, 0, 0);
          acc2[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah, cl, acc2[t], 0, 0, 0);
          acc2[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al, ch, acc2[t], 0, 0, 0);
        }
      }
    }
    if (++nchunk == kG3Flush) {   // end of a K-block: FP32 sums into the FP64 accumulators
      nchunk = 0;
#pragma unroll
      for (int t = 0; t < TPW; ++t) {
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          dacc1[t][q] += (double)acc1[t][q];
          dacc2[t][q] += (double)acc2[t][q];
        }
        acc1[t] = acc2[t] = (float4_t){0.f, 0.f, 0.f, 0.f};
      }
    }
  }
#pragma unroll
  for (int t = 0; t < TPW; ++t)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      dacc1[t][q] += (double)acc1[t][q];
      dacc2[t][q] += (double)acc2[t][q];
    }
#pragma unroll
  for (int y = 0; y < NY; ++y) {
    double* p = partial + ((size_t)y * tiles + tile) * k * k;
#pragma unroll
    for (int t = 0; t < TPW; ++t) {
      const int tt = wave + NW * t;
      if (tt < TT) {
        const int ti = tt / T, tj = tt - (tt / T) * T;
        const int j = 16 * tj + li;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int i = 16 * ti + 4 * g + q;
          if (i < k && j < k) p[(size_t)i * k + j] = (y == 0) ? dacc1[t][q] : dacc2[t][q];
        }
      }
    }
  }
}

__global__ void f2d_kernel(size_t n, const float* __restrict__ a, double* __restrict__ b) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (double)a[i];
}

// ---- generic tiled FP64 GEMM: C = alpha op(A) op(B) + beta C (row-major)
constexpr int GT = 64, GK = 16;

template <typename T>
__global__ __launch_bounds__(kBlock) void gemm_kernel(int ta, int tb, int M, int N, int K, double alpha,
                                                      const T* __restrict__ A, int lda,
                                                      const T* __restrict__ B, int ldb, double beta,
                                                      T* __restrict__ C, int ldc) {
  __shared__ T As[GK][GT + 1];
  __shared__ T Bs[GK][GT + 1];
  const int bm = blockIdx.y * GT, bn = blockIdx.x * GT;
  const int tx = threadIdx.x % 16, ty = threadIdx.x / 16;
  T acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += GK) {
    for (int e = threadIdx.x; e < GK * GT; e += kBlock) {
      // A tile: op(A)[bm + i][k0 + kk]
      const int kk = e / GT, i = e % GT;
      const int gi = bm + i, gk = k0 + kk;
      T v = (T)0;
      if (gi < M && gk < K) v = ta ? A[(size_t)gk * lda + gi] : A[(size_t)gi * lda + gk];
      As[kk][i] = v;
      // B tile: op(B)[k0 + kk][bn + j]
      const int j = i;
      const int gj = bn + j;
      T w = (T)0;
      if (gj < N && gk < K) w = tb ? B[(size_t)gj * ldb + gk] : B[(size_t)gk * ldb + gj];
      Bs[kk][j] = w;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < GK; ++kk) {
      T a[4], b[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        a[q] = As[kk][ty + 16 * q];
        b[q] = Bs[kk][tx + 16 * q];
      }
#pragma unroll
      for (int p = 0; p < 4; ++p)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[p][q] = fma(a[p], b[q], acc[p][q]);
    }
    __syncthreads();
  }
#pragma unroll
  for (int p = 0; p < 4; ++p)
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int i = bm + ty + 16 * p, j = bn + tx + 16 * q;
      if (i < M && j < N) {
        T* c = C + (size_t)i * ldc + j;
        *c = (beta == 0.0) ? (T)(alpha * acc[p][q]) : (T)fma(alpha, (double)acc[p][q], beta * (double)*c);
      }
    }
}

// ---- small GEMM (M <= kSmallM, K <= kSmallK), latency-oriented: the coarse-space
// products (N_H x N_H times N_H x k, k x k products) have too few 64 x 64 tiles to
// fill the chip, so a block takes a few rows and one 64-column chunk and its waves
// split K.
constexpr int kSmallM = 4096, kSmallK = 4096;

// Rows i0 .. i0+R-1 of C per block (1024 threads = 16 waves): the R rows of op(A) are staged in LDS,
// lane j of every wave owns column j of a 64-column slice, the 16 waves split K, and one load of
// op(B)[kk][j] serves all R rows.  Partial sums meet in LDS in a fixed order.
constexpr int kSmallWaves = 16;

template <typename T, int R>
__global__ __launch_bounds__(kSmallWaves * 64) void gemm_small_kernel(int ta, int tb, int M, int N, int K, double alpha,
                                                                     const T* __restrict__ A, int lda,
                                                                     const T* __restrict__ B, int ldb, double beta,
                                                                     T* __restrict__ C, int ldc) {
  extern __shared__ double gsm[];
  double* arow = gsm;                                 // [R][K]
  double* part = gsm + (size_t)R * K;                 // [kSmallWaves][R][64]
  const int i0 = blockIdx.y * R;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int j = blockIdx.x * 64 + lane;
  for (int e = threadIdx.x; e < R * K; e += kSmallWaves * 64) {
    const int r = e / K, kk = e - (e / K) * K;
    const int i = i0 + r;
    arow[e] = (i < M) ? (double)(ta ? A[(size_t)kk * lda + i] : A[(size_t)i * lda + kk]) : 0.0;
  }
  __syncthreads();
  const int kq = (K + kSmallWaves - 1) / kSmallWaves;
  const int k0 = wave * kq, k1 = (k0 + kq < K) ? k0 + kq : K;
  double acc[R];
#pragma unroll
  for (int r = 0; r < R; ++r) acc[r] = 0.0;
  if (j < N) {
    const size_t bs = tb ? 1 : (size_t)ldb;           // stride of op(B) along kk
    const T* __restrict__ bp = tb ? B + (size_t)j * ldb : B + j;
    int kk = k0;
    for (; kk + 4 <= k1; kk += 4) {
      const double b0 = (double)bp[kk * bs], b1 = (double)bp[(kk + 1) * bs];
      const double b2 = (double)bp[(kk + 2) * bs], b3 = (double)bp[(kk + 3) * bs];
#pragma unroll
      for (int r = 0; r < R; ++r) {
        const double* ar = arow + (size_t)r * K + kk;
        acc[r] = fma(ar[0], b0, fma(ar[1], b1, fma(ar[2], b2, fma(ar[3], b3, acc[r]))));
      }
    }
    for (; kk < k1; ++kk) {
      const double bv = (double)bp[kk * bs];
#pragma unroll
      for (int r = 0; r < R; ++r) acc[r] = fma(arow[(size_t)r * K + kk], bv, acc[r]);
    }
  }
#pragma unroll
  for (int r = 0; r < R; ++r) part[(wave * R + r) * 64 + lane] = acc[r];
  __syncthreads();
  if (wave < R) {
    const int r = wave, i = i0 + r;
    if (i < M && j < N) {
      double t = 0.0;
      for (int w = 0; w < kSmallWaves; ++w) t += part[(w * R + r) * 64 + lane];
      T* c = C + (size_t)i * ldc + j;
      *c = (beta == 0.0) ? (T)(alpha * t) : (T)fma(alpha, t, beta * (double)*c);
    }
  }
}

template <typename T>
void launch_gemm_small(int ta, int tb, int M, int N, int K, double alpha, const T* A, int lda, const T* B, int ldb,
                       double beta, T* C, int ldc, hipStream_t s) {
  if (K <= 1024) {
    constexpr int R = 4;
    const size_t lds = ((size_t)R * K + (size_t)kSmallWaves * R * 64) * sizeof(double);
    gemm_small_kernel<T, R><<<dim3((N + 63) / 64, (M + R - 1) / R), kSmallWaves * 64, lds, s>>>(
        ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
  } else {
    const size_t lds = ((size_t)K + (size_t)kSmallWaves * 64) * sizeof(double);
    gemm_small_kernel<T, 1><<<dim3((N + 63) / 64, M), kSmallWaves * 64, lds, s>>>(ta, tb, M, N, K, alpha, A, lda, B,
                                                                                  ldb, beta, C, ldc);
  }
}

// ---- tall-skinny Y = X op(C) (+ Y), X and Y N x k (row-major), C k x k, k <= KMAX (64 or 128), on
// MFMA (v_mfma_f64_16x16x4f64).  A block walks chunks of 64 consecutive rows; a chunk of X (and of
// Y) is one contiguous run of 64 k doubles, read and written with coalesced accesses.  Wave w
// (KMAX / 16 waves) owns output columns 16w .. 16w+15 and keeps that strip of op(C) as B fragments
// in registers; the X chunk is staged in LDS (row stride KMAX + 2) and read as A fragments; the
// 64 x k result goes back through the same LDS array for the contiguous store.
// MFMA operand layout: lane l supplies A[l%16][l/16] and B[l/16][l%16]; accumulator register q
// holds D[l/16 + 4q][l%16].
constexpr int kTsmRows = 64;

template <int TB, int KMAX>
__global__ __launch_bounds__(KMAX * 4) void tsmm_mfma_kernel(long long N, int k, const double* __restrict__ X,
                                                             const double* __restrict__ C, double* __restrict__ Y,
                                                             int accumulate, long long nchunks) {
  constexpr int NT = KMAX * 4;                  // threads: one wave per 16-column strip
  constexpr int LD = KMAX + 2;                  // 16 rows x 4 columns of an A fragment fall in distinct banks
  constexpr int SE = kTsmRows * KMAX / NT;      // staged doubles per thread
  constexpr int KS4 = KMAX / 4;
  __shared__ double xs[kTsmRows * LD];
  const int tid = threadIdx.x, lane = tid & 63;
  const int w = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int li = lane & 15, lk = lane >> 4;
  const int KS = (k + 3) >> 2;
  for (int e = tid; e < kTsmRows * LD; e += NT) xs[e] = 0.0;   // columns >= k stay zero
  // B fragments of this wave's column strip: b[s] = op(C)[4s + lk][16w + li], zero outside k
  double b[KS4];
  {
    const int j = 16 * w + li, jc = (j < k) ? j : k - 1;
#pragma unroll
    for (int s = 0; s < KS4; ++s) {
      const int kk = 4 * s + lk, kc = (kk < k) ? kk : k - 1;
      const double v = TB ? C[(size_t)jc * k + kc] : C[(size_t)kc * k + jc];
      b[s] = (kk < k && j < k) ? v : 0.0;
    }
  }
  const int ck = kTsmRows * k;
  // LDS slot of each staged element (row e / k, column e % k); independent of the chunk
  int soff[SE];
#pragma unroll
  for (int u = 0; u < SE; ++u) {
    const int e = tid + NT * u;
    const int r = e / k;
    soff[u] = (e < ck) ? r * LD + (e - r * k) : -1;
  }
  for (long long c = blockIdx.x; c < nchunks; c += gridDim.x) {
    const long long lim = (N - c * kTsmRows) * k;
    const int nval = (int)((lim < ck) ? lim : ck);   // valid doubles of this chunk
    const double* __restrict__ xp = X + c * kTsmRows * k;
    double* __restrict__ yp = Y + c * kTsmRows * k;
    double sv[SE], yv[SE];
#pragma unroll
    for (int u = 0; u < SE; ++u) {
      const int e = tid + NT * u;
      const int ec = (e < nval) ? e : nval - 1;   // clamped, unconditional: all loads in flight together
      sv[u] = xp[ec];
      yv[u] = accumulate ? yp[ec] : 0.0;
    }
    __syncthreads();   // the previous chunk's result has been read out of xs
#pragma unroll
    for (int u = 0; u < SE; ++u) {
      const int e = tid + NT * u;
      if (soff[u] >= 0) xs[soff[u]] = (e < nval) ? sv[u] : 0.0;   // rows past N are zero
    }
    __syncthreads();
    double4_t acc[4];
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) acc[rt] = (double4_t){0.0, 0.0, 0.0, 0.0};
    if (16 * w < k) {
#pragma unroll
      for (int s = 0; s < KS4; ++s) {
        if (s < KS) {
#pragma unroll
          for (int rt = 0; rt < 4; ++rt)
            acc[rt] = __builtin_amdgcn_mfma_f64_16x16x4f64(xs[(16 * rt + li) * LD + 4 * s + lk], b[s], acc[rt], 0, 0,
                                                           0);
        }
      }
    }
    __syncthreads();   // every wave is done reading the X chunk
    if (16 * w < k && 16 * w + li < k) {
#pragma unroll
      for (int rt = 0; rt < 4; ++rt)
#pragma unroll
        for (int q = 0; q < 4; ++q) xs[(16 * rt + lk + 4 * q) * LD + 16 * w + li] = acc[rt][q];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < SE; ++u) {
      const int e = tid + NT * u;
      if (e < nval) yp[e] = xs[soff[u]] + yv[u];
    }
  }
}

__global__ void set_blocks_kernel(int n, int nh, int k, const double* __restrict__ C0, const double* __restrict__ G,
                                  const double* __restrict__ H, double* __restrict__ T) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n * n) return;
  const int i = (int)(e / n), j = (int)(e % n);
  double v;
  if (i < nh && j < nh) v = C0[(size_t)i * nh + j];
  else if (i < nh) v = G[(size_t)i * k + (j - nh)];
  else if (j < nh) v = G[(size_t)j * k + (i - nh)];
  else v = H[(size_t)(i - nh) * k + (j - nh)];
  T[e] = v;
}

inline unsigned nblk(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

int coldot_tiles(long long N, int k) {
  const int slots = kBlock / k;
  const long long rows = (long long)slots * kColdotPasses;
  long long t = (N + rows - 1) / rows;
  return (int)(((t + 7) / 8) * 8);
}

void launch_coldot(long long N, int k, const double* X, const double* Y, double* partial, int ptiles, double* out,
                   hipStream_t s) {
  const int slots = kBlock / k;
  const int rows = slots * kColdotPasses;
  const int tiles = (int)((N + rows - 1) / rows);
  const int blocks = ((tiles + 7) / 8) * 8;
  (void)ptiles;
  coldot_kernel<double><<<blocks, kBlock, 0, s>>>(N, k, X, Y, partial, tiles, rows);
  reduce_partials_kernel<<<k, kBlock, 0, s>>>(tiles, k, partial, out);
}

void launch_coldot_f32(long long N, int k, const float* X, const float* Y, double* partial, double* out,
                       hipStream_t s) {
  const int slots = kBlock / k;
  const int rows = slots * kColdotPasses;
  const int tiles = (int)((N + rows - 1) / rows);
  const int blocks = ((tiles + 7) / 8) * 8;
  coldot_kernel<float><<<blocks, kBlock, 0, s>>>(N, k, X, Y, partial, tiles, rows);
  reduce_partials_kernel<<<k, kBlock, 0, s>>>(tiles, k, partial, out);
}

void launch_reduce_partials(int tiles, int width, const double* partial, double* out, hipStream_t s) {
  reduce_partials_kernel<<<width, kBlock, 0, s>>>(tiles, width, partial, out);
}

void launch_pcg_alpha(int k, const double* rho, const double* pq, double* alpha, hipStream_t s) {
  pcg_alpha_kernel<<<1, kBlock, 0, s>>>(k, rho, pq, alpha);
}

void launch_pcg_beta(int k, const double* rn, const double* ro, double* beta, hipStream_t s) {
  pcg_beta_kernel<<<1, kBlock, 0, s>>>(k, rn, ro, beta);
}

void launch_axpy2(long long N, int k, const double* alpha, const double* P, const double* Q, double* X, double* R,
                  hipStream_t s) {
  axpy2_kernel<double><<<nblk(N * k), kBlock, 0, s>>>(N, k, alpha, P, Q, X, X, R);
}

void launch_axpy2_from(long long N, int k, const double* alpha, const double* P, const double* Q, const double* Xin,
                       double* X, double* R, hipStream_t s) {
  axpy2_kernel<double><<<nblk(N * k), kBlock, 0, s>>>(N, k, alpha, P, Q, Xin, X, R);
}

void launch_flex_beta(int k, const double* a, const double* b, const double* c, int* mask, double* beta,
                      hipStream_t s) {
  flex_beta_kernel<<<1, kBlock, 0, s>>>(k, a, b, c, mask, beta);
}

void launch_fallback(int k, double ratio, const double* rn, const double* ro, int* mask, hipStream_t s) {
  fallback_kernel<<<1, kBlock, 0, s>>>(k, ratio * ratio, rn, ro, mask);
}

void launch_gather_cols(long long N, int k, int ka, const int* idx, const double* B, double* C, hipStream_t s) {
  gather_cols_kernel<<<nblk(N * ka), kBlock, 0, s>>>(N, k, ka, idx, B, C);
}

void launch_merge_cols(long long N, int k, int ka, const int* pos, const double* C, const double* U, double* B,
                       hipStream_t s) {
  merge_cols_kernel<<<nblk(N * k), kBlock, 0, s>>>(N, k, ka, pos, C, U, B);
}

void launch_scatter_cols(long long N, int k, int ka, const int* idx, const double* C, double* B, hipStream_t s) {
  scatter_cols_kernel<<<nblk(N * ka), kBlock, 0, s>>>(N, k, ka, idx, C, B);
}

void launch_copy_cols(long long N, int kin, int kout, int nc, const double* src, double* dst, int fill,
                      hipStream_t s) {
  copy_cols_kernel<<<nblk(N * kout), kBlock, 0, s>>>(N, kin, kout, nc, src, dst, fill);
}

void launch_select_cols(long long N, int k, const int* mask, const double* A, double* Z, hipStream_t s) {
  select_cols_kernel<<<nblk(N * k), kBlock, 0, s>>>(N, k, mask, A, Z);
}

void launch_fill_int(int n, int v, int* p, hipStream_t s) { fill_int_kernel<<<1, kBlock, 0, s>>>(n, v, p); }

void launch_rsub(long long N, int k, const double* alpha, const double* Q, double* R, hipStream_t s) {
  rsub_kernel<<<nblk(N * k), kBlock, 0, s>>>(N, k, alpha, Q, R);
}

void launch_zadd(long long N, int k, const double* beta, const double* P, double* Z, hipStream_t s) {
  zadd_kernel<<<nblk(N * k), kBlock, 0, s>>>(N, k, beta, P, Z);
}

void launch_axpy3(long long N, int k, const double* a0, const double* P, const double* a1, const double* Z,
                  const double* X0, double* X, hipStream_t s) {
  axpy3_kernel<<<nblk(N * k), kBlock, 0, s>>>(N, k, a0, P, a1, Z, X0, X);
}

void launch_axpy3_merge(long long N, int k, int ldx, const int* pos, const double* a0, const double* P, const double* a1,
                        const double* Z, const double* X0, double* X, hipStream_t s) {
  axpy3_merge_kernel<<<nblk(N * ldx), kBlock, 0, s>>>(N, k, ldx, pos, a0, P, a1, Z, X0, X);
}

void launch_xpby(long long N, int k, const double* Z, const double* beta, double* P, hipStream_t s) {
  xpby_kernel<double><<<nblk(N * k), kBlock, 0, s>>>(N, k, Z, beta, P);
}

void launch_axpy2_f32(long long N, int k, const double* alpha, const float* P, const float* Q, float* X, float* R,
                      hipStream_t s) {
  axpy2_kernel<float><<<nblk(N * k), kBlock, 0, s>>>(N, k, alpha, P, Q, X, X, R);
}

void launch_xpby_f32(long long N, int k, const float* Z, const double* beta, float* P, hipStream_t s) {
  xpby_kernel<float><<<nblk(N * k), kBlock, 0, s>>>(N, k, Z, beta, P);
}

void launch_d2f(size_t n, const double* a, float* b, hipStream_t s) {
  d2f_kernel<<<nblk((long long)n), kBlock, 0, s>>>(n, a, b);
}

void launch_cg_start_f32(size_t n, const double* R, float* r, float* e, hipStream_t s) {
  cg_start_f32_kernel<<<nblk((long long)n), kBlock, 0, s>>>(n, R, r, e);
}

void launch_copy_f32(size_t n, const float* src, float* dst, hipStream_t s) {
  copy_f32_kernel<<<nblk((long long)n), kBlock, 0, s>>>(n, src, dst);
}

void launch_add_f2d_merge(long long N, int k, int ldw, const int* pos, const double* u, const float* e, double* w,
                          hipStream_t s) {
  add_f2d_merge_kernel<<<nblk(N * ldw), kBlock, 0, s>>>(N, k, ldw, pos, u, e, w);
}

void launch_add_f2d(size_t n, const double* u, const float* e, double* w, hipStream_t s) {
  add_f2d_kernel<<<nblk((long long)n), kBlock, 0, s>>>(n, u, e, w);
}

void launch_copy(size_t n, const double* src, double* dst, hipStream_t s) {
  copy_kernel<<<nblk((long long)n), kBlock, 0, s>>>(n, src, dst);
}

int gram_tiles(long long N, int k) {
  (void)k;
  long long t = (N + 255) / 256;
  if (t > 512) t = 512;
  if (t < 1) t = 1;
  return (int)t;
}

void launch_gram2(long long N, int k, const double* X, const double* Y1, const double* Y2, double* partial,
                  int tiles, double* G1, double* G2, hipStream_t s) {
  long long rows = (N + tiles - 1) / tiles;
  rows = ((rows + 3) / 4) * 4;
  const int blocks = ((tiles + 7) / 8) * 8;
  const int T = (k + 15) / 16;
  const size_t lds = (size_t)(Y2 ? 3 : 2) * kGramRows * (T * 16 + 1) * sizeof(double);
  if (k <= 64) {
    if (Y2) gram_lds_kernel<2, 64><<<blocks, kBlock, lds, s>>>(N, k, X, Y1, Y2, partial, tiles, rows);
    else gram_lds_kernel<1, 64><<<blocks, kBlock, lds, s>>>(N, k, X, Y1, nullptr, partial, tiles, rows);
  } else {
    // k > 64: one right-hand block per pass (keeps the accumulators in registers)
    const size_t lds1 = (size_t)2 * kGramRows * (T * 16 + 1) * sizeof(double);
    gram_lds_kernel<1, 128><<<blocks, kBlock, lds1, s>>>(N, k, X, Y1, nullptr, partial, tiles, rows);
    if (Y2)
      gram_lds_kernel<1, 128><<<blocks, kBlock, lds1, s>>>(N, k, X, Y2, nullptr, partial + (size_t)tiles * k * k,
                                                           tiles, rows);
  }
  reduce_partials_kernel<<<k * k, kBlock, 0, s>>>(tiles, k * k, partial, G1);
  if (Y2) reduce_partials_kernel<<<k * k, kBlock, 0, s>>>(tiles, k * k, partial + (size_t)tiles * k * k, G2);
}

void launch_gram2_sym(long long N, int k, const double* X, const double* Y1, const double* Y2, double* partial,
                      int tiles, double* G1, double* G2, hipStream_t s) {
  if (k <= 64) {
    launch_gram2(N, k, X, Y1, Y2, partial, tiles, G1, G2, s);
    return;
  }
  long long rows = (N + tiles - 1) / tiles;
  rows = ((rows + 3) / 4) * 4;
  const int blocks = ((tiles + 7) / 8) * 8;
  const int T = (k + 15) / 16;
  const size_t lds = (size_t)(Y2 ? 3 : 2) * kGramRows * (T * 16 + 1) * sizeof(double);
  if (Y2) gram_sym_kernel<2><<<blocks, kSymThreads, lds, s>>>(N, k, X, Y1, Y2, partial, tiles, rows);
  else gram_sym_kernel<1><<<blocks, kSymThreads, lds, s>>>(N, k, X, Y1, nullptr, partial, tiles, rows);
  reduce_partials_kernel<<<k * k, kBlock, 0, s>>>(tiles, k * k, partial, G1);
  if (Y2) reduce_partials_kernel<<<k * k, kBlock, 0, s>>>(tiles, k * k, partial + (size_t)tiles * k * k, G2);
}

void launch_gram_bf16x3(long long N, int k, const float* X, const float* Y1, const float* Y2, double* partial,
                        int tiles, double* G1, double* G2, hipStream_t s) {
  long long rows = (N + tiles - 1) / tiles;
  rows = ((rows + 3) / 4) * 4;
  const int blocks = ((tiles + 7) / 8) * 8;
  if (k <= 64) {
    if (Y2) gram_bf16x3_kernel<2, 64><<<blocks, 256, 0, s>>>(N, k, X, Y1, Y2, partial, tiles, rows);
    else gram_bf16x3_kernel<1, 64><<<blocks, 256, 0, s>>>(N, k, X, Y1, nullptr, partial, tiles, rows);
  } else if (k <= 128) {
    // one right-hand block per pass (two would not fit the accumulators in registers)
    gram_bf16x3_kernel<1, 128><<<blocks, 512, 0, s>>>(N, k, X, Y1, nullptr, partial, tiles, rows);
    if (Y2)
      gram_bf16x3_kernel<1, 128><<<blocks, 512, 0, s>>>(N, k, X, Y2, nullptr, partial + (size_t)tiles * k * k, tiles,
                                                        rows);
  } else {
    return;   // callers keep k <= 128
  }
  reduce_partials_kernel<<<k * k, kBlock, 0, s>>>(tiles, k * k, partial, G1);
  if (Y2) reduce_partials_kernel<<<k * k, kBlock, 0, s>>>(tiles, k * k, partial + (size_t)tiles * k * k, G2);
}

void launch_f2d(size_t n, const float* a, double* b, hipStream_t s) {
  f2d_kernel<<<nblk((long long)n), kBlock, 0, s>>>(n, a, b);
}

void launch_gram(long long N, int k, const double* X, const double* Y, double* partial, int tiles, double* G,
                 hipStream_t s) {
  if (k <= 128) {
    launch_gram2(N, k, X, Y, nullptr, partial, tiles, G, nullptr, s);
    return;
  }
  long long rows = (N + tiles - 1) / tiles;
  rows = ((rows + 3) / 4) * 4;
  const int blocks = ((tiles + 7) / 8) * 8;
  gram_kernel<<<blocks, kBlock, 0, s>>>(N, k, X, Y, partial, tiles, rows);
  reduce_partials_kernel<<<k * k, kBlock, 0, s>>>(tiles, k * k, partial, G);
}

// products with a dimension above 1024 (large coarse spaces, and the tall-skinny products with
// k > 64) run on the MFMA GEMM; the smaller ones keep the latency-oriented kernels
inline bool gemm_large(int M, int K) { return M > 1024 || K > 1024; }

void launch_gemm(bool ta, bool tb, int M, int N, int K, double alpha, const double* A, int lda, const double* B,
                 int ldb, double beta, double* C, int ldc, hipStream_t s) {
  if (gemm_large(M, K)) {
    launch_gemm_mfma(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s);
    return;
  }
  if (M <= kSmallM && K <= kSmallK) {
    launch_gemm_small<double>(ta ? 1 : 0, tb ? 1 : 0, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s);
    return;
  }
  dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT);
  gemm_kernel<double><<<grid, kBlock, 0, s>>>(ta ? 1 : 0, tb ? 1 : 0, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
}

void launch_gemm_f32(bool ta, bool tb, int M, int N, int K, double alpha, const float* A, int lda, const float* B,
                     int ldb, double beta, float* C, int ldc, hipStream_t s) {
  if (gemm_large(M, K)) {
    launch_gemm_mfma_f32(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s);
    return;
  }
  if (M <= kSmallM && K <= kSmallK) {
    launch_gemm_small<float>(ta ? 1 : 0, tb ? 1 : 0, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s);
    return;
  }
  dim3 grid((N + GT - 1) / GT, (M + GT - 1) / GT);
  gemm_kernel<float><<<grid, kBlock, 0, s>>>(ta ? 1 : 0, tb ? 1 : 0, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc);
}

void launch_tsmm(long long N, int k, const double* X, const double* C, double* Y, int accumulate, int tb,
                 hipStream_t s) {
  const long long nchunks = (N + kTsmRows - 1) / kTsmRows;
  if (k <= 64) {
    const unsigned blocks = (unsigned)((nchunks < 768) ? nchunks : 768);
    if (tb) tsmm_mfma_kernel<1, 64><<<blocks, 256, 0, s>>>(N, k, X, C, Y, accumulate, nchunks);
    else tsmm_mfma_kernel<0, 64><<<blocks, 256, 0, s>>>(N, k, X, C, Y, accumulate, nchunks);
    return;
  }
  if (k <= 128) {
    const unsigned blocks = (unsigned)((nchunks < 512) ? nchunks : 512);
    if (tb) tsmm_mfma_kernel<1, 128><<<blocks, 512, 0, s>>>(N, k, X, C, Y, accumulate, nchunks);
    else tsmm_mfma_kernel<0, 128><<<blocks, 512, 0, s>>>(N, k, X, C, Y, accumulate, nchunks);
    return;
  }
  launch_gemm(false, tb != 0, (int)N, k, k, 1.0, X, k, C, k, accumulate ? 1.0 : 0.0, Y, k, s);
}

void launch_set_diag_block(int n, int nh, int k, const double* C0, const double* G, const double* H, double* T,
                           hipStream_t s) {
  set_blocks_kernel<<<nblk((long long)n * n), kBlock, 0, s>>>(n, nh, k, C0, G, H, T);
}

}  // namespace pase
