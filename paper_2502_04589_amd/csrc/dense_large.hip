// Dense FP64 linear algebra for the large coarse spaces (N_H in the thousands,
// e.g. 15^3 = 3375 interior nodes of a 16^3 coarse mesh):
//   - an FP64 GEMM on v_mfma_f64_16x16x4f64 (64 x 64 tiles staged in LDS),
//   - blocked right-looking Cholesky and blocked triangular inverse (panels on one
//     workgroup, trailing updates as GEMMs),
//   - the k smallest eigenpairs of a dense symmetric n x n matrix for n up to
//     kLargeMaxN: Householder tridiagonalisation by one cooperative grid whose
//     workgroups own cyclic rows of the matrix in global memory (one grid barrier
//     per reflector), multisection bisection, inverse iteration, Cholesky-QR of the
//     block and the blocked back-transformation.
// These serve the one-time setup of the coarse space (Cholesky factors and
// inverses of A_H and B_H, the diagonalisation C0 = Phi Theta Phi^T) and the dense
// solve of the augmented eigenproblem (Alg. 3 step 5) when its size exceeds what
// one workgroup holds.
#include <cfloat>

#include "internal.hpp"

namespace pase {

namespace {

typedef double double4_t __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ MFMA GEMM
// C = alpha op(A) op(B) + beta C (row-major), storage type T (double or float), FP64
// arithmetic.  A block computes a BM x 64 tile (BM = 64, 32 or 16, the smaller ones for products
// with few output tiles, such as N_H x N_H times N_H x k) with four waves: 2 x 2 waves of
// 32 x 32 (BM 64), 2 x 2 waves of 16 x 32 (BM 32) or 1 x 4 waves of 16 x 16 (BM 16), in 16 x 16
// sub-tiles.  K advances 16 per LDS stage; the next stage's operands are loaded into registers
// while the current one is multiplied.  MFMA operand layout: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator register q holds D[l/16 + 4q][l%16].
constexpr int kGN = 64, kGK = 16;

template <typename T, int BM>
__global__ __launch_bounds__(256) void gemm_mfma_kernel(int ta, int tb, int M, int N, int K, double alpha,
                                                        const T* __restrict__ A, int lda, const T* __restrict__ B,
                                                        int ldb, double beta, T* __restrict__ C, int ldc) {
  constexpr int WC = (BM == 16) ? 4 : 2;         // waves along the columns
  constexpr int SR = (BM == 64) ? 2 : 1;         // 16-row sub-tiles per wave
  constexpr int SC = 4 / WC;                     // 16-column sub-tiles per wave
  constexpr int UA = BM * kGK / 256;             // staged A values per thread
  __shared__ double As[kGK][BM + 2];
  __shared__ double Bs[kGK][kGN + 2];
  const int bm = blockIdx.y * BM, bn = blockIdx.x * kGN;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int wr = (wave / WC) * 16 * SR, wc = (wave % WC) * 16 * SC;
  double ra[UA], rb[4];
  // element u of this thread in a stage: (row, kk) of op(A) and (kk, col) of op(B), chosen so
  // that consecutive threads read consecutive addresses
  auto fetch = [&](int k0) {
#pragma unroll
    for (int u = 0; u < UA; ++u) {
      const int e = tid + 256 * u;
      int i, kk;
      if (ta) { i = e % BM; kk = e / BM; } else { kk = e & 15; i = e >> 4; }
      const int gi = bm + i, gk = k0 + kk;
      ra[u] = (gi < M && gk < K) ? (double)(ta ? A[(size_t)gk * lda + gi] : A[(size_t)gi * lda + gk]) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + 256 * u;
      int j, k2;
      if (tb) { k2 = e & 15; j = e >> 4; } else { j = e & 63; k2 = e >> 6; }
      const int gj = bn + j, gk2 = k0 + k2;
      rb[u] = (gj < N && gk2 < K) ? (double)(tb ? B[(size_t)gj * ldb + gk2] : B[(size_t)gk2 * ldb + gj]) : 0.0;
    }
  };
  auto stash = [&]() {
#pragma unroll
    for (int u = 0; u < UA; ++u) {
      const int e = tid + 256 * u;
      if (ta) As[e / BM][e % BM] = ra[u]; else As[e & 15][e >> 4] = ra[u];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = tid + 256 * u;
      if (tb) Bs[e & 15][e >> 4] = rb[u]; else Bs[e >> 6][e & 63] = rb[u];
    }
  };
  double4_t acc[SR][SC];
#pragma unroll
  for (int a = 0; a < SR; ++a)
#pragma unroll
    for (int b = 0; b < SC; ++b) acc[a][b] = (double4_t){0.0, 0.0, 0.0, 0.0};
  fetch(0);
  for (int k0 = 0; k0 < K; k0 += kGK) {
    __syncthreads();
    stash();
    __syncthreads();
    if (k0 + kGK < K) fetch(k0 + kGK);
#pragma unroll
    for (int s = 0; s < kGK / 4; ++s) {
      double av[SR], bv[SC];
#pragma unroll
      for (int t = 0; t < SR; ++t) av[t] = As[4 * s + lk][wr + 16 * t + li];
#pragma unroll
      for (int t = 0; t < SC; ++t) bv[t] = Bs[4 * s + lk][wc + 16 * t + li];
#pragma unroll
      for (int a = 0; a < SR; ++a)
#pragma unroll
        for (int b = 0; b < SC; ++b) acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
  }
#pragma unroll
  for (int a = 0; a < SR; ++a)
#pragma unroll
    for (int b = 0; b < SC; ++b)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int i = bm + wr + 16 * a + lk + 4 * q, j = bn + wc + 16 * b + li;
        if (i < M && j < N) {
          T* c = C + (size_t)i * ldc + j;
          const double v = alpha * acc[a][b][q];
          *c = (beta == 0.0) ? (T)v : (T)(v + beta * (double)*c);
        }
      }
}

// Products with few output tiles and a long K (N_H x N_H times N_H x k: 422 tiles of 16 x 64 for
// N_H = 3375, k = 128) leave the 16-row kernel above with under two waves per SIMD stepping through
// K in 16-wide stages, each waiting on its loads.  Here a block of 16 waves splits K four ways: the
// four waves of group g (one 16 x 16 sub-tile each, as above) stage and multiply the K-range
// [g Kq, (g+1) Kq) through their own LDS buffers, and the four partial tiles are summed in a fixed
// order at the end (the result does not depend on timing).
constexpr int kSkGroups = 4;

template <typename T>
__global__ __launch_bounds__(1024) void gemm_mfma_sk_kernel(int ta, int tb, int M, int N, int K, double alpha,
                                                             const T* __restrict__ A, int lda, const T* __restrict__ B,
                                                             int ldb, double beta, T* __restrict__ C, int ldc) {
  constexpr int BM = 16;
  // the partial tiles reuse the stage buffers once every group is done with them
  __shared__ union {
    struct {
      double As[kSkGroups][kGK][BM + 2];
      double Bs[kSkGroups][kGK][kGN + 2];
    } st;
    double Red[kSkGroups - 1][BM][kGN];
  } sm;
  auto& As = sm.st.As;
  auto& Bs = sm.st.Bs;
  auto& Red = sm.Red;
  const int bm = blockIdx.y * BM, bn = blockIdx.x * kGN;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int g = wave >> 2, gt = tid & 255, gw = wave & 3;    // group, thread and wave within it
  const int li = lane & 15, lk = lane >> 4;
  const int wc = gw * 16;
  const int nst = (K + kSkGroups * kGK - 1) / (kSkGroups * kGK);   // stages per group
  const int kb = g * nst * kGK;                                     // this group's first K
  double ra, rb[4];
  auto fetch = [&](int k0) {
    {
      int i, kk;
      if (ta) { i = gt % BM; kk = gt / BM; } else { kk = gt & 15; i = gt >> 4; }
      const int gi = bm + i, gk = k0 + kk;
      ra = (gi < M && gk < K) ? (double)(ta ? A[(size_t)gk * lda + gi] : A[(size_t)gi * lda + gk]) : 0.0;
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = gt + 256 * u;
      int j, k2;
      if (tb) { k2 = e & 15; j = e >> 4; } else { j = e & 63; k2 = e >> 6; }
      const int gj = bn + j, gk2 = k0 + k2;
      rb[u] = (gj < N && gk2 < K) ? (double)(tb ? B[(size_t)gj * ldb + gk2] : B[(size_t)gk2 * ldb + gj]) : 0.0;
    }
  };
  auto stash = [&]() {
    if (ta) As[g][gt / BM][gt % BM] = ra; else As[g][gt & 15][gt >> 4] = ra;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int e = gt + 256 * u;
      if (tb) Bs[g][e & 15][e >> 4] = rb[u]; else Bs[g][e >> 6][e & 63] = rb[u];
    }
  };
  double4_t acc = (double4_t){0.0, 0.0, 0.0, 0.0};
  fetch(kb);
  for (int st = 0; st < nst; ++st) {
    __syncthreads();
    stash();
    __syncthreads();
    if (st + 1 < nst) fetch(kb + (st + 1) * kGK);
#pragma unroll
    for (int s4 = 0; s4 < kGK / 4; ++s4)
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(As[g][4 * s4 + lk][li], Bs[g][4 * s4 + lk][wc + li], acc, 0, 0, 0);
  }
  // groups 1..3 hand their partial tiles to group 0, which adds them in group order
  __syncthreads();
  if (g > 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) Red[g - 1][lk + 4 * q][wc + li] = acc[q];
  }
  __syncthreads();
  if (g == 0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int r = lk + 4 * q;
      double v = acc[q];
#pragma unroll
      for (int h = 0; h < kSkGroups - 1; ++h) v += Red[h][r][wc + li];
      const int i = bm + r, j = bn + wc + li;
      if (i < M && j < N) {
        T* c = C + (size_t)i * ldc + j;
        const double w = alpha * v;
        *c = (beta == 0.0) ? (T)w : (T)(w + beta * (double)*c);
      }
    }
  }
}

// ------------------------------------------------------------------ blocked Cholesky
constexpr int kNB = 64;   // panel width

__global__ void ptol_kernel(int n, const double* __restrict__ A, int lda, double* __restrict__ ptol) {
  __shared__ double red[4];
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double m = 0.0;
  for (int i = tid; i < n; i += 256) m = fmax(m, A[(size_t)i * lda + i]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
  if (lane == 0) red[wave] = m;
  __syncthreads();
  if (tid == 0) *ptol = n * DBL_EPSILON * fmax(fmax(red[0], red[1]), fmax(red[2], red[3]));
}

// In-place lower Cholesky of the b x b diagonal block (b <= kNB) with a pivot threshold
// from ptol; on a failed pivot writes *info = off + j + 1 (nothing on success).
__global__ __launch_bounds__(1024) void chol_diag_kernel(int b, double* A, int lda, const double* ptol, int* info,
                                                         int off) {
  __shared__ double L[kNB][kNB + 1];
  __shared__ int fail;
  const int tid = threadIdx.x;
  for (int e = tid; e < b * b; e += 1024) {
    const int i = e / b, j = e % b;
    L[i][j] = A[(size_t)i * lda + j];
  }
  if (tid == 0) fail = 0;
  __syncthreads();
  const double pt = *ptol;
  const int tx = tid & 31, ty = tid >> 5;
  for (int j = 0; j < b; ++j) {
    const double d = L[j][j];
    if (!(d > pt)) {
      if (tid == 0) fail = j + 1;
      break;
    }
    const double sq = sqrt(d);
    __syncthreads();
    if (tid == 0) L[j][j] = sq;
    for (int i = j + 1 + tid; i < b; i += 1024) L[i][j] /= sq;
    __syncthreads();
    for (int i = j + 1 + ty; i < b; i += 32)
      for (int l = j + 1 + tx; l <= i; l += 32) L[i][l] = fma(-L[i][j], L[l][j], L[i][l]);
    __syncthreads();
  }
  __syncthreads();
  for (int e = tid; e < b * b; e += 1024) {
    const int i = e / b, j = e % b;
    A[(size_t)i * lda + j] = (j <= i) ? L[i][j] : 0.0;
  }
  if (tid == 0 && fail) *info = off + fail;
}

// Li (b x b, ld ldi) = inverse of the lower b x b block L (ld ldl), b <= kNB: L staged in LDS,
// one thread per column of the inverse (forward substitution in LDS), then written back.
__global__ __launch_bounds__(kNB) void trinv_diag_kernel(int b, const double* __restrict__ L, int ldl,
                                                         double* __restrict__ Li, int ldi) {
  __shared__ double sL[kNB][kNB + 1];
  __shared__ double sX[kNB][kNB + 1];
  for (int e = threadIdx.x; e < b * b; e += blockDim.x) {
    const int i = e / b, j = e % b;
    sL[i][j] = (j <= i) ? L[(size_t)i * ldl + j] : 0.0;
  }
  __syncthreads();
  const int c = threadIdx.x;
  if (c < b) {
    for (int i = 0; i < c; ++i) sX[i][c] = 0.0;
    for (int i = c; i < b; ++i) {
      double s = (i == c) ? 1.0 : 0.0;
      for (int l = c; l < i; ++l) s = fma(-sL[i][l], sX[l][c], s);
      sX[i][c] = s / sL[i][i];
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < b * b; e += blockDim.x) {
    const int i = e / b, j = e % b;
    Li[(size_t)i * ldi + j] = sX[i][j];
  }
}

__global__ void copy2d_kernel(int rows, int cols, const double* __restrict__ S, int lds, double* __restrict__ D,
                              int ldd) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)rows * cols) return;
  const int i = (int)(e / cols), j = (int)(e % cols);
  D[(size_t)i * ldd + j] = S[(size_t)i * lds + j];
}

__global__ void zero_upper_kernel(int n, double* __restrict__ A, int lda) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)n * n) return;
  const int i = (int)(e / n), j = (int)(e % n);
  if (j > i) A[(size_t)i * lda + j] = 0.0;
}

__global__ void zero2d_kernel(int rows, int cols, double* __restrict__ D, int ldd) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)rows * cols) return;
  D[(size_t)(e / cols) * ldd + (size_t)(e % cols)] = 0.0;
}

__global__ void set_int_kernel(int* p, int v) { *p = v; }

inline unsigned nb256(long long n) { return (unsigned)((n + 255) / 256); }

// ------------------------------------------------------------------ grid tridiagonalisation
constexpr int kLargeMaxN = 3840;   // invit's LDS (5 n doubles + n bytes) stays below 160 KiB
constexpr int kTgThreads = 512;
constexpr int kTgWaves = kTgThreads / 64;
constexpr unsigned kTgMaxSpins = 1u << 22;

__device__ __forceinline__ double ld_agent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_agent(double* p, double v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier of the NW blocks.  Everything one block writes for another (the products p and
// the published row) is written and read with agent-scope atomic accesses, which are coherent
// across the XCDs' L2 caches by themselves; each block's own matrix rows never leave it.  So
// the barrier needs no cache write-back or invalidation: a block waits until its own stores have
// completed, then arrives.  Arrival is two-level to spread the atomics: the blocks of group
// b % 8 count on their group's counter (own cache line), and the last of each group bumps the
// top counter that everyone polls.  The spin is bounded: on timeout, or when another block has
// raised *err, the block raises *err and reports false, so every wave of the grid returns.
// counters: [0] top, [16 g] group g (unsigned, 64-byte apart).
__device__ bool grid_sync(unsigned* counters, unsigned round, int NW, int* err) {
  __shared__ int ok;
  __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");
  __syncthreads();
  if (threadIdx.x == 0) {
    const int g = blockIdx.x & 7;
    const unsigned members = (unsigned)((NW - g + 7) / 8);    // blocks b < NW with b % 8 == g
    const unsigned groups = (unsigned)(NW < 8 ? NW : 8);
    const unsigned old = __hip_atomic_fetch_add(&counters[16 * (g + 1)], 1u, __ATOMIC_RELAXED,
                                                __HIP_MEMORY_SCOPE_AGENT);
    if (old + 1 == round * members) __hip_atomic_fetch_add(&counters[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const unsigned target = round * groups;
    unsigned spins = 0;
    ok = 1;
    while (__hip_atomic_load(&counters[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kTgMaxSpins || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
    }
  }
  __syncthreads();
  return ok != 0;
}

__device__ double tg_sum(double v, double (*red)[kTgWaves], int& parity) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* r = red[parity];
  parity ^= 1;
  if (lane == 0) r[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kTgWaves; ++w) s += r[w];
  return s;
}

// Householder reflector of x = row[0 .. mm-1]: v[0] = 1, v[i] = x[i] / (alpha - beta); returns tau
// (the same arithmetic in every block, so every block holds the same reflector).
__device__ double tg_reflector(const double* row, int mm, double* v, double& beta_out, double (*red)[kTgWaves],
                               int& parity) {
  double part = 0.0;
  for (int i = 1 + threadIdx.x; i < mm; i += kTgThreads) part = fma(row[i], row[i], part);
  const double xn2 = tg_sum(part, red, parity);
  const double alpha = row[0];
  if (xn2 == 0.0) {
    for (int i = threadIdx.x; i < mm; i += kTgThreads) v[i] = (i == 0) ? 1.0 : 0.0;
    beta_out = alpha;
    __syncthreads();
    return 0.0;
  }
  const double beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
  const double sc = 1.0 / (alpha - beta);
  for (int i = threadIdx.x; i < mm; i += kTgThreads) v[i] = (i == 0) ? 1.0 : row[i] * sc;
  beta_out = beta;
  __syncthreads();
  return (beta - alpha) / beta;
}

// Tridiagonalisation of the symmetric n x n matrix T (row-major, full storage, in global
// memory).  Block b of the NW co-resident blocks owns the rows r with r % NW == b; only
// it reads and writes them.  Step j (trailing block A22 = rows/columns j+1 .. n-1):
//   every block reads p_j = tau_j A22 v_j and row j+1 (before update j) from the exchange
//   buffers, forms K_j = tau_j p_j^T v_j / 2 and w_j = p_j - K_j v_j, updates its copy of
//   row j+1 and builds reflector j+1 from it; then it applies
//   A22 <- A22 - v_j w_j^T - w_j v_j^T to its own rows r >= j+2 (columns >= j+2) and, in the
//   same pass, forms p_{j+1} = tau_{j+1} A v_{j+1} for those rows and publishes it (and row
//   j+2, by its owner) for the next step; one grid barrier.
// Reflector j is stored in row j of T (entries j+2 .. n-1; entry j+1 is an implicit 1), tau in
// tri[2n ..], d and e in tri[0 ..] and tri[n ..] (the layout of the one-workgroup solver).
__global__ __launch_bounds__(kTgThreads) void tridiag_grid_kernel(int n, int NW, double* __restrict__ T,
                                                                 double* __restrict__ tri,
                                                                 double* __restrict__ xchg, unsigned* counter,
                                                                 int* err) {
  const int b = blockIdx.x;
  if (b >= NW) return;
  extern __shared__ double dyn[];
  double* v = dyn;               // reflector j (index c - (j+1))
  double* w = v + n;             // p_j, then w_j
  double* v2 = w + n;            // reflector j+1 (index c - (j+2))
  double* prow = v2 + n;         // row j+1 (global column index)
  __shared__ double red[2][kTgWaves];
  int parity = 0;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  double* pbuf = xchg;           // 2 x n, alternating per step
  double* rbuf = xchg + 2 * n;   // 2 x n
  double* d = tri;
  double* e = tri + n;
  double* tau = tri + 2 * n;
  unsigned round = 0;
  for (int c = tid; c < n; c += kTgThreads) prow[c] = T[c];
  __syncthreads();
  double beta0;
  double tcur = tg_reflector(prow + 1, n - 1, v, beta0, red, parity);
  if (b == 0 && tid == 0) {
    d[0] = prow[0];
    e[0] = beta0;
    tau[0] = tcur;
  }
  // p_0 on the owned rows r >= 1, and row 1 published by its owner
  for (int r = b + NW * wave; r < n; r += NW * kTgWaves) {
    if (r < 1) continue;
    const double* ar = T + (size_t)r * n;
    double acc = 0.0;
    for (int c0 = 1 + lane; c0 < n; c0 += 64 * 8) {
      double a[8];
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int c = c0 + 64 * u;
        a[u] = (c < n) ? ar[c] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 8; ++u) {
        const int c = c0 + 64 * u;
        if (c < n) acc = fma(a[u], v[c - 1], acc);
      }
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) st_agent(&pbuf[r - 1], tcur * acc);
    if (r == 1)
      for (int c = lane; c < n; c += 64) st_agent(&rbuf[c], ar[c]);
  }
  if (!grid_sync(counter, ++round, NW, err)) return;
  // reflector 0 goes into row 0 only now: every block has read that row before the barrier
  if (b == 0)
    for (int i = 1 + tid; i < n - 1; i += kTgThreads) T[i + 1] = v[i];
  for (int j = 0; j + 2 < n; ++j) {
    const int m = n - j - 1;
    const int par = j & 1;
    const double* pin = pbuf + par * n;
    const double* rin = rbuf + par * n;
    double* pout = pbuf + (par ^ 1) * n;
    double* rout = rbuf + (par ^ 1) * n;
    for (int i = tid; i < m; i += kTgThreads) w[i] = ld_agent(pin + i);
    for (int c = tid; c < n; c += kTgThreads) prow[c] = (c >= j + 1) ? ld_agent(rin + c) : 0.0;
    __syncthreads();
    double pv = 0.0;
    for (int i = tid; i < m; i += kTgThreads) pv = fma(w[i], v[i], pv);
    const double K = 0.5 * tcur * tg_sum(pv, red, parity);
    for (int i = tid; i < m; i += kTgThreads) w[i] = w[i] - K * v[i];
    __syncthreads();
    const double v0 = v[0], w0 = w[0];
    for (int c = j + 1 + tid; c < n; c += kTgThreads) {
      const int cc = c - (j + 1);
      prow[c] -= v0 * w[cc] + w0 * v[cc];
    }
    __syncthreads();
    const bool has_next = (j + 3 < n);
    double tnext = 0.0, bnext = 0.0;
    if (has_next) {
      tnext = tg_reflector(prow + (j + 2), m - 1, v2, bnext, red, parity);
      if (b == 0 && tid == 0) {
        d[j + 1] = prow[j + 1];
        e[j + 1] = bnext;
        tau[j + 1] = tnext;
      }
      if ((j + 1) % NW == b)
        for (int i = 1 + tid; i < m - 1; i += kTgThreads) T[(size_t)(j + 1) * n + (j + 2) + i] = v2[i];
    } else if (b == 0 && tid == 0) {
      d[j + 1] = prow[j + 1];
      e[j + 1] = prow[j + 2];
      tau[j + 1] = 0.0;
    }
    // update j on the owned rows r >= j+2 and p_{j+1} = tnext A v2 on them
    int r = b;
    if (r < j + 2) r += ((j + 2 - r + NW - 1) / NW) * NW;
    for (r += NW * wave; r < n; r += NW * kTgWaves) {
      double* ar = T + (size_t)r * n;
      const int rr = r - (j + 1);
      const double vr = v[rr], wr = w[rr];
      const bool publish = has_next && r == j + 2;
      double acc = 0.0;
      // batches of 8 loads per lane in flight (a row streams from the memory-side cache)
      for (int c0 = j + 2 + lane; c0 < n; c0 += 64 * 8) {
        double a[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int c = c0 + 64 * u;
          a[u] = (c < n) ? ar[c] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) {
          const int c = c0 + 64 * u;
          if (c < n) {
            const int cc = c - (j + 1);
            const double val = a[u] - (vr * w[cc] + wr * v[cc]);
            ar[c] = val;
            if (has_next) acc = fma(val, v2[c - (j + 2)], acc);
            if (publish) st_agent(&rout[c], val);
            if (!has_next && r == n - 1 && c == n - 1) d[n - 1] = val;
          }
        }
      }
      if (has_next) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (lane == 0) st_agent(&pout[r - (j + 2)], tnext * acc);
      }
    }
    if (!has_next) break;
    double* t1 = v;
    v = v2;
    v2 = t1;
    tcur = tnext;
    if (!grid_sync(counter, ++round, NW, err)) return;
  }
}

__global__ void tg_reset_kernel(unsigned* counter, int* err) {
  for (int i = threadIdx.x; i < 16 * 9; i += blockDim.x) counter[i] = 0u;
  if (threadIdx.x == 0) *err = 0;
}

__global__ void tg_fold_kernel(int* info, const int* err, const int* cinfo) {
  if (*err || *cinfo) *info = 2;
}

__device__ int sturm_count_l(int n, const double* d, const double* e2, double x, double pivmin) {
  int c = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  c += (q < 0.0);
  for (int i = 1; i < n; ++i) {
    q = (d[i] - x) - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    c += (q < 0.0);
  }
  return c;
}

// The (t+1)-th smallest eigenvalue of the tridiagonal, t = blockIdx.x, by 64-point
// multisection with Sturm counts (d and e^2 in LDS).
// With off given, the eigenvalue of index *off + blockIdx.x (a window of the spectrum).
__global__ __launch_bounds__(64) void bisect_large_kernel(int n, const double* __restrict__ tri,
                                                         double* __restrict__ lam, const int* __restrict__ off) {
  extern __shared__ double dyn[];
  double* d = dyn;
  double* e2 = dyn + n;
  const int t = blockIdx.x + (off ? *off : 0), lane = threadIdx.x;
  for (int i = lane; i < n; i += 64) {
    d[i] = tri[i];
    const double ei = tri[n + i];
    e2[i] = ei * ei;
  }
  __syncthreads();
  const double* sc = tri + 3 * n;
  double lo = sc[0], hi = sc[1];
  const double pivmin = sc[2];
  for (int round = 0; round < 40; ++round) {
    if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + pivmin) break;
    const double x = lo + (hi - lo) * (double)(lane + 1) / 65.0;
    const int cnt = sturm_count_l(n, d, e2, x, pivmin);
    const unsigned long long below = __ballot(cnt <= t);
    const int c = __popcll(below);
    const double nlo = (c > 0) ? __shfl(x, c - 1, 64) : lo;
    const double nhi = (c < 64) ? __shfl(x, c < 64 ? c : 63, 64) : hi;
    if (nlo == lo && nhi == hi) break;
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) lam[blockIdx.x] = 0.5 * (lo + hi);
}

// Start of the index window of W = min(2 nsel, n) eigenvalues around theta: with c eigenvalues
// below theta (a Sturm count), the nsel nearest theta form a run of consecutive indices inside
// [c - nsel, c + nsel); off = that range clamped to [0, n - W].
__global__ void window_start_kernel(int n, int nsel, double theta, const double* __restrict__ tri, int* off) {
  if (threadIdx.x != 0) return;
  const double* d = tri;
  const double* e = tri + n;
  const double pivmin = tri[3 * n + 2];
  int c = 0;
  double q = d[0] - theta;
  if (fabs(q) < pivmin) q = -pivmin;
  c += (q < 0.0);
  for (int i = 1; i < n; ++i) {
    q = (d[i] - theta) - e[i - 1] * e[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    c += (q < 0.0);
  }
  const int W = (2 * nsel < n) ? 2 * nsel : n;
  int o = c - nsel;
  if (o > n - W) o = n - W;
  if (o < 0) o = 0;
  *off = o;
}

// The nsel of the W ascending window values nearest theta (a run): the farther end is dropped
// until nsel remain, the upper one on a tie.
__global__ void nearest_run_kernel(int W, int nsel, double theta, const double* __restrict__ lamw,
                                   double* __restrict__ lam) {
  __shared__ int first;
  if (threadIdx.x == 0) {
    int l = 0, r = W;
    while (r - l > nsel) {
      if (fabs(lamw[l] - theta) > fabs(lamw[r - 1] - theta)) ++l;
      else --r;
    }
    first = l;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < nsel; i += blockDim.x) lam[i] = lamw[first + i];
}

__device__ __forceinline__ double hash_unit_l(unsigned a, unsigned b) {
  unsigned h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  h *= 0x297A2D39u;
  h ^= h >> 15;
  return (double)(h & 0xFFFFFF) / (double)0x800000 - 1.0;
}

// Eigenvector j = blockIdx.x of the tridiagonal by three steps of inverse iteration with the
// partial-pivoting LU of T - lambda_j I (lane 0 runs the sequential recurrences; d and e
// stream from global memory 16 entries at a time).  Output vector-major in Vt.
__global__ __launch_bounds__(64) void invit_large_kernel(int n, const double* __restrict__ tri,
                                                        const double* __restrict__ lam, double* __restrict__ Vt) {
  extern __shared__ double dyn[];
  double* u0 = dyn;
  double* u1 = u0 + n;
  double* u2 = u1 + n;
  double* mulv = u2 + n;
  double* x = mulv + n;
  unsigned char* piv = (unsigned char*)(x + n);
  const double* __restrict__ dg = tri;
  const double* __restrict__ eg = tri + n;
  const int j = blockIdx.x, lane = threadIdx.x;
  const double tnorm = tri[3 * n + 3];
  for (int i = lane; i < n; i += 64) x[i] = hash_unit_l(j + 1, i + 1);
  __syncthreads();
  const double tiny = DBL_EPSILON * tnorm;
  const double lj = lam[j];
  if (lane == 0) {
    double r0 = dg[0] - lj, r1 = (n > 1) ? eg[0] : 0.0, r2 = 0.0;
    for (int i0 = 0; i0 < n - 1; i0 += 16) {
      double dd[16], ee[17];
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int i = i0 + u;
        dd[u] = (i + 1 < n) ? dg[i + 1] : 0.0;
        ee[u] = (i < n) ? eg[i] : 0.0;
      }
      ee[16] = (i0 + 16 < n) ? eg[i0 + 16] : 0.0;
#pragma unroll
      for (int u = 0; u < 16; ++u) {
        const int i = i0 + u;
        if (i < n - 1) {
          const double s0 = ee[u], s1 = dd[u] - lj, s2 = (i + 2 < n) ? ee[u + 1] : 0.0;
          double mlt, n0, n1;
          if (fabs(r0) >= fabs(s0)) {
            if (r0 == 0.0) r0 = tiny;
            mlt = s0 / r0;
            piv[i] = 0;
            u0[i] = r0; u1[i] = r1; u2[i] = r2;
            n0 = s1 - mlt * r1;
            n1 = s2 - mlt * r2;
          } else {
            mlt = r0 / s0;
            piv[i] = 1;
            u0[i] = s0; u1[i] = s1; u2[i] = s2;
            n0 = r1 - mlt * s1;
            n1 = r2 - mlt * s2;
          }
          mulv[i] = mlt;
          r0 = n0; r1 = n1; r2 = 0.0;
        }
      }
    }
    if (r0 == 0.0) r0 = tiny;
    u0[n - 1] = 1.0 / r0; u1[n - 1] = 0.0; u2[n - 1] = 0.0;
    for (int i = 0; i < n - 1; ++i) u0[i] = 1.0 / u0[i];
  }
  __syncthreads();
  for (int it = 0; it < 3; ++it) {
    double xm = 0.0;
    for (int i = lane; i < n; i += 64) xm = fmax(xm, fabs(x[i]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) xm = fmax(xm, __shfl_xor(xm, o, 64));
    const double inv = (xm > 0.0) ? 1.0 / xm : 1.0;
    for (int i = lane; i < n; i += 64) x[i] *= inv;
    __syncthreads();
    if (lane == 0) {
      double xi = x[0];
      for (int i = 0; i < n - 1; ++i) {
        double xn = x[i + 1];
        if (piv[i]) { const double tt = xi; xi = xn; xn = tt; }
        xn -= mulv[i] * xi;
        x[i] = xi;
        xi = xn;
      }
      x[n - 1] = xi;
      double xp1 = 0.0, xp2 = 0.0;
      for (int i = n - 1; i >= 0; --i) {
        const double vv = (x[i] - u1[i] * xp1 - u2[i] * xp2) * u0[i];
        x[i] = vv;
        xp2 = xp1;
        xp1 = vv;
      }
    }
    __syncthreads();
  }
  double nn = 0.0;
  for (int i = lane; i < n; i += 64) nn = fma(x[i], x[i], nn);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) nn += __shfl_xor(nn, o, 64);
  const double rn = 1.0 / sqrt(nn);
  for (int i = lane; i < n; i += 64) Vt[(size_t)j * n + i] = x[i] * rn;
}

// Back-transformation of eigenvector c = blockIdx.x: x <- Q x, Q = prod_blocks (I - Y S Y^T),
// last block first, with the S matrices of wy_prep; x in LDS; result into column c of V (n x k).
constexpr int kWyB = 32;
__global__ __launch_bounds__(256) void wy_apply_large_kernel(int n, int k, const double* __restrict__ T,
                                                            const double* __restrict__ Sall,
                                                            const double* __restrict__ Vt,
                                                            double* __restrict__ V) {
  extern __shared__ double x[];
  __shared__ double w1[kWyB], w2[kWyB];
  const int c = blockIdx.x;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int i = tid; i < n; i += 256) x[i] = Vt[(size_t)c * n + i];
  __syncthreads();
  const int nref = n - 2;
  const int nblk = (nref + kWyB - 1) / kWyB;
  for (int blk = nblk - 1; blk >= 0; --blk) {
    const int j0 = blk * kWyB;
    const int b = (nref - j0 < kWyB) ? nref - j0 : kWyB;
    for (int r = wave; r < b; r += 4) {
      const int jr = j0 + r;
      double s2 = 0.0;
      for (int i = jr + 1 + lane; i < n; i += 64) {
        const double yr = (i == jr + 1) ? 1.0 : T[(size_t)jr * n + i];
        s2 = fma(yr, x[i], s2);
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) s2 += __shfl_xor(s2, o, 64);
      if (lane == 0) w1[r] = s2;
    }
    __syncthreads();
    const double* S = Sall + (size_t)blk * kWyB * kWyB;
    if (tid < b) {
      double s2 = 0.0;
      for (int l = tid; l < b; ++l) s2 = fma(S[tid * kWyB + l], w1[l], s2);
      w2[tid] = s2;
    }
    __syncthreads();
    for (int i = j0 + 1 + tid; i < n; i += 256) {
      double s2 = 0.0;
      const int rmax = (i - j0 - 1 < b - 1) ? (i - j0 - 1) : (b - 1);
      for (int r = 0; r <= rmax; ++r) {
        const int jr = j0 + r;
        const double yr = (i == jr + 1) ? 1.0 : T[(size_t)jr * n + i];
        s2 = fma(yr, w2[r], s2);
      }
      x[i] -= s2;
    }
    __syncthreads();
  }
  for (int i = tid; i < n; i += 256) V[(size_t)i * k + c] = x[i];
}

__global__ void copy_vals_kernel(int k, const double* __restrict__ a, double* __restrict__ b) {
  for (int i = threadIdx.x; i < k; i += blockDim.x) b[i] = a[i];
}

size_t chol_scratch_doubles(int n) { return (size_t)n * kNB + 8; }

}  // namespace

// ------------------------------------------------------------------ launchers
// The row tile is the largest of 64, 32, 16 that still gives at least 512 blocks (two per CU).
template <typename T>
static void gemm_mfma(bool ta, bool tb, int M, int N, int K, double alpha, const T* A, int lda, const T* B, int ldb,
                      double beta, T* C, int ldc, hipStream_t s) {
  if (M <= 0 || N <= 0) return;
  const long long cols = (N + kGN - 1) / kGN;
  const int a = ta ? 1 : 0, b = tb ? 1 : 0;
  if (cols * ((M + 63) / 64) >= 512) {
    gemm_mfma_kernel<T, 64><<<dim3((unsigned)cols, (M + 63) / 64), 256, 0, s>>>(a, b, M, N, K, alpha, A, lda, B, ldb,
                                                                                 beta, C, ldc);
  } else if (cols * ((M + 31) / 32) >= 512) {
    gemm_mfma_kernel<T, 32><<<dim3((unsigned)cols, (M + 31) / 32), 256, 0, s>>>(a, b, M, N, K, alpha, A, lda, B, ldb,
                                                                                 beta, C, ldc);
  } else if (K >= 1024) {
    gemm_mfma_sk_kernel<T><<<dim3((unsigned)cols, (M + 15) / 16), 1024, 0, s>>>(a, b, M, N, K, alpha, A, lda, B, ldb,
                                                                                beta, C, ldc);
  } else {
    gemm_mfma_kernel<T, 16><<<dim3((unsigned)cols, (M + 15) / 16), 256, 0, s>>>(a, b, M, N, K, alpha, A, lda, B, ldb,
                                                                                 beta, C, ldc);
  }
}

void launch_gemm_mfma(bool ta, bool tb, int M, int N, int K, double alpha, const double* A, int lda,
                      const double* B, int ldb, double beta, double* C, int ldc, hipStream_t s) {
  gemm_mfma<double>(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s);
}

void launch_gemm_mfma_f32(bool ta, bool tb, int M, int N, int K, double alpha, const float* A, int lda,
                          const float* B, int ldb, double beta, float* C, int ldc, hipStream_t s) {
  gemm_mfma<float>(ta, tb, M, N, K, alpha, A, lda, B, ldb, beta, C, ldc, s);
}

size_t cholesky_large_scratch_doubles(int n) { return chol_scratch_doubles(n); }

// In-place lower Cholesky of an n x n SPD matrix (row-major): panels of kNB columns factored
// on one workgroup, the panel below solved as L21 = A21 L11^{-T} and the trailing matrix
// updated as A22 -= L21 L21^T, both GEMMs.  *info is set to 0, then to j + 1 if pivot j is at or
// below n eps max_i A_ii.  scratch >= cholesky_large_scratch_doubles(n).
void launch_cholesky_large(int n, double* A, int lda, double* scratch, int* info, hipStream_t s) {
  double* ptol = scratch;
  double* L11i = scratch + 8;                      // kNB x kNB
  double* L21 = L11i + (size_t)kNB * kNB;          // (n - kNB) x kNB
  set_int_kernel<<<1, 1, 0, s>>>(info, 0);
  ptol_kernel<<<1, 256, 0, s>>>(n, A, lda, ptol);
  for (int j0 = 0; j0 < n; j0 += kNB) {
    const int b = (n - j0 < kNB) ? n - j0 : kNB;
    double* Ajj = A + (size_t)j0 * lda + j0;
    chol_diag_kernel<<<1, 1024, 0, s>>>(b, Ajj, lda, ptol, info, j0);
    const int m2 = n - j0 - b;
    if (m2 <= 0) break;
    trinv_diag_kernel<<<1, kNB, 0, s>>>(b, Ajj, lda, L11i, kNB);
    double* A21 = A + (size_t)(j0 + b) * lda + j0;
    gemm_mfma<double>(false, true, m2, b, b, 1.0, A21, lda, L11i, kNB, 0.0, L21, kNB, s);
    double* A22 = A + (size_t)(j0 + b) * lda + (j0 + b);
    gemm_mfma<double>(false, true, m2, m2, b, -1.0, L21, kNB, L21, kNB, 1.0, A22, lda, s);
    copy2d_kernel<<<nb256((long long)m2 * b), 256, 0, s>>>(m2, b, L21, kNB, A21, lda);
  }
  zero_upper_kernel<<<nb256((long long)n * n), 256, 0, s>>>(n, A, lda);
}

size_t trinv_large_scratch_doubles(int n) { return (size_t)kNB * n; }

// Li = L^{-1} for a lower n x n L (Li must not alias L), by block rows of kNB:
// Li[I,I] = L[I,I]^{-1} and Li[I, <I] = -Li[I,I] (L[I, <I] Li[<I, <I]).
void launch_trinv_large(int n, const double* L, int ldl, double* Li, int ldi, double* scratch, hipStream_t s) {
  zero2d_kernel<<<nb256((long long)n * n), 256, 0, s>>>(n, n, Li, ldi);
  for (int i0 = 0; i0 < n; i0 += kNB) {
    const int b = (n - i0 < kNB) ? n - i0 : kNB;
    double* Lii = Li + (size_t)i0 * ldi + i0;
    trinv_diag_kernel<<<1, kNB, 0, s>>>(b, L + (size_t)i0 * ldl + i0, ldl, Lii, ldi);
    if (i0 == 0) continue;
    // scratch (b x i0) = L[I, 0:i0] Li[0:i0, 0:i0]
    gemm_mfma<double>(false, false, b, i0, i0, 1.0, L + (size_t)i0 * ldl, ldl, Li, ldi, 0.0, scratch, n, s);
    gemm_mfma<double>(false, false, b, i0, b, -1.0, Lii, ldi, scratch, n, 0.0, Li + (size_t)i0 * ldi, ldi, s);
  }
}

int syev_large_max_n() { return kLargeMaxN; }

size_t syev_large_work_doubles(int n, int k) {
  const size_t nblk = (size_t)(n + kWyB - 1) / kWyB + 1;
  size_t w = (size_t)3 * n + 8 + (size_t)k + (size_t)2 * n * k + (size_t)2 * k * k + nblk * kWyB * kWyB +
             (size_t)4 * n + 80;
  w += chol_scratch_doubles(k) + trinv_large_scratch_doubles(k);
  return w;
}

size_t syev_window_work_doubles(int n, int nsel) { return syev_large_work_doubles(n, nsel) + 2 * (size_t)nsel + 8; }

namespace {

// k eigenpairs of the dense symmetric n x n matrix T (overwritten): the k smallest, or with
// window set the k nearest theta.
void syev_large_impl(int n, int k, bool window, double theta, double* T, double* w, double* V, double* work,
                     int* info, hipStream_t s) {
  double* tri = work;
  double* lam = tri + 3 * n + 8;
  double* Vt = lam + k;
  double* Vt2 = Vt + (size_t)n * k;
  double* G = Vt2 + (size_t)n * k;
  double* G2 = G + (size_t)k * k;
  const size_t nblk = (size_t)(n + kWyB - 1) / kWyB + 1;
  double* Sall = G2 + (size_t)k * k;
  double* xchg = Sall + nblk * kWyB * kWyB;            // 4 n
  unsigned* counter = (unsigned*)(xchg + 4 * (size_t)n);  // 9 counters, 64 bytes apart
  int* err = (int*)(counter + 16 * 9);
  int* cinfo = err + 1;                                // Cholesky-QR status (k above one workgroup)
  double* cscr = xchg + 4 * (size_t)n + 80;
  double* tscr = cscr + chol_scratch_doubles(k);
  set_int_kernel<<<1, 1, 0, s>>>(info, 0);
  set_int_kernel<<<1, 1, 0, s>>>(cinfo, 0);
  set_int_kernel<<<1, 1, 0, s>>>(cinfo + 1, 0);
  tg_reset_kernel<<<1, 64, 0, s>>>(counter, err);
  int dev = 0, ncu = 256;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  int NW = ncu < 256 ? ncu : 256;
  if (NW > n / 4) NW = n / 4 > 1 ? n / 4 : 1;
  const size_t lds = (size_t)4 * n * sizeof(double);
  {
    void* args[] = {(void*)&n, (void*)&NW, (void*)&T, (void*)&tri, (void*)&xchg, (void*)&counter, (void*)&err};
    // co-residency of the NW blocks is what the grid barrier needs; a refused launch is
    // reported through the barrier's error flag
    if (hipLaunchCooperativeKernel((const void*)tridiag_grid_kernel, dim3(NW), dim3(kTgThreads), args, lds, s) !=
        hipSuccess) {
      (void)hipGetLastError();
      set_int_kernel<<<1, 1, 0, s>>>(err, 1);
    }
  }
  launch_tri_finish(n, tri, s);
  if (window) {
    double* lamw = work + syev_large_work_doubles(n, k);
    int* off = (int*)(lamw + 2 * (size_t)k);
    const int W = (2 * k < n) ? 2 * k : n;
    window_start_kernel<<<1, 64, 0, s>>>(n, k, theta, tri, off);
    bisect_large_kernel<<<W, 64, 2 * (size_t)n * sizeof(double), s>>>(n, tri, lamw, off);
    nearest_run_kernel<<<1, 256, 0, s>>>(W, k, theta, lamw, lam);
  } else {
    bisect_large_kernel<<<k, 64, 2 * (size_t)n * sizeof(double), s>>>(n, tri, lam, nullptr);
  }
  invit_large_kernel<<<k, 64, 5 * (size_t)n * sizeof(double) + (size_t)n, s>>>(n, tri, lam, Vt);
  if (k <= syev_max_k()) {
    launch_vorth2(n, k, Vt, Vt2, G, info, s);
  } else {
    // two Cholesky-QR passes with GEMMs: G = Vt Vt^T = L L^T, Vt <- L^{-1} Vt
    for (int pass = 0; pass < 2; ++pass) {
      gemm_mfma<double>(false, true, k, k, n, 1.0, Vt, n, Vt, n, 0.0, G, k, s);
      launch_cholesky_large(k, G, k, cscr, cinfo + pass, s);
      launch_trinv_large(k, G, k, G2, k, tscr, s);
      gemm_mfma<double>(false, false, k, n, k, 1.0, G2, k, Vt, n, 0.0, Vt2, n, s);
      double* t = Vt;
      Vt = Vt2;
      Vt2 = t;
    }
  }
  launch_wy_prep(n, T, tri, Sall, s);
  wy_apply_large_kernel<<<k, 256, (size_t)n * sizeof(double), s>>>(n, k, T, Sall, Vt, V);
  copy_vals_kernel<<<1, 256, 0, s>>>(k, lam, w);
  tg_fold_kernel<<<1, 1, 0, s>>>(info, err, cinfo);
  tg_fold_kernel<<<1, 1, 0, s>>>(info, err, cinfo + 1);
}

}  // namespace

// The k smallest eigenpairs of the dense symmetric n x n matrix T (overwritten), n <= kLargeMaxN:
// w (device, ascending), V (device n x k row-major).  *info = 0, or non-zero when the grid
// barrier timed out or the orthonormalisation broke down.
void launch_syev_large(int n, int k, double* T, double* w, double* V, double* work, int* info, hipStream_t s) {
  syev_large_impl(n, k, false, 0.0, T, w, V, work, info, s);
}

// The nsel eigenpairs of T nearest theta (nsel <= n <= kLargeMaxN), ascending: the window of
// 2 nsel indices around theta by bisection, its nsel values nearest theta, their vectors.
void launch_syev_window(int n, int nsel, double theta, double* T, double* w, double* V, double* work, int* info,
                        hipStream_t s) {
  syev_large_impl(n, nsel, true, theta, T, w, V, work, info, s);
}

}  // namespace pase
