// Dense single-workgroup FP64 kernels for the small problems of the method:
// Cholesky factorisation, triangular inverse, and the k smallest eigenpairs
// of a dense symmetric matrix (the augmented eigenproblem of Alg. 3 step 5 in
// an M-orthonormal basis).
//
// Eigensolver: Householder reduction to tridiagonal form, bisection with
// Sturm counts for the k smallest eigenvalues, inverse iteration with
// partial-pivoting tridiagonal LU for their eigenvectors (re-orthogonalised
// inside tight clusters, then two passes of Cholesky-QR over the block), and
// back-transformation by the stored reflectors.
#include <cfloat>

#include "internal.hpp"

namespace pase {

namespace {

constexpr int kDenseThreads = 1024;
constexpr int kDenseWaves = kDenseThreads / 64;
constexpr int kSyevMaxN = 1024;

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Fixed-order block sum; every thread gets the result.  Uses red[kDenseWaves].
__device__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < kDenseWaves; ++w) s += red[w];
  return s;
}

// A pivot at or below n * eps * max_i A[i][i] counts as a breakdown (numerically
// rank-deficient Gram matrices are reported, not factored).
__global__ __launch_bounds__(kDenseThreads) void cholesky_kernel(int n, double* A, int lda, int* info) {
  __shared__ int fail;
  __shared__ double ptol;
  if (threadIdx.x == 0) {
    fail = 0;
    double dmax = 0.0;
    for (int i = 0; i < n; ++i) dmax = fmax(dmax, A[(size_t)i * lda + i]);
    ptol = n * DBL_EPSILON * dmax;
  }
  __syncthreads();
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  for (int j = 0; j < n; ++j) {
    if (threadIdx.x == 0) {
      const double d = A[(size_t)j * lda + j];
      if (!(d > ptol)) {
        fail = j + 1;
      } else {
        A[(size_t)j * lda + j] = sqrt(d);
      }
    }
    __syncthreads();
    if (fail) break;
    const double djj = A[(size_t)j * lda + j];
    for (int i = j + 1 + threadIdx.x; i < n; i += kDenseThreads) A[(size_t)i * lda + j] /= djj;
    __syncthreads();
    // trailing update of the lower triangle: A[i][l] -= A[i][j] A[l][j], j < l <= i
    for (int i = j + 1 + wave; i < n; i += kDenseWaves) {
      const double aij = A[(size_t)i * lda + j];
      for (int l = j + 1 + lane; l <= i; l += 64) A[(size_t)i * lda + l] -= aij * A[(size_t)l * lda + j];
    }
    __syncthreads();
  }
  __syncthreads();
  if (!fail) {
    for (long long e = threadIdx.x; e < (long long)n * n; e += kDenseThreads) {
      const int i = (int)(e / n), l = (int)(e % n);
      if (l > i) A[(size_t)i * lda + l] = 0.0;
    }
  }
  if (threadIdx.x == 0) *info = fail;
}

// Li = L^{-1}: thread c owns column c; rows are processed in order, so each
// thread only reads entries of its own column written earlier.
__global__ __launch_bounds__(kBlock) void trinv_kernel(int n, const double* __restrict__ L, int ldl,
                                                       double* __restrict__ Li, int ldi) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  for (int i = 0; i < c; ++i) Li[(size_t)i * ldi + c] = 0.0;
  for (int i = c; i < n; ++i) {
    double s = (i == c) ? 1.0 : 0.0;
    for (int l = c; l < i; ++l) s -= L[(size_t)i * ldl + l] * Li[(size_t)l * ldi + c];
    Li[(size_t)i * ldi + c] = s / L[(size_t)i * ldl + i];
  }
}

// ---- eigensolver helpers
__device__ int sturm_count(int n, const double* d, const double* e2, double x, double pivmin) {
  int c = 0;
  double q = d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  c += (q < 0.0);
  for (int i = 1; i < n; ++i) {
    q = d[i] - x - e2[i - 1] / q;
    if (fabs(q) < pivmin) q = -pivmin;
    c += (q < 0.0);
  }
  return c;
}

__device__ __forceinline__ double hash_unit(unsigned a, unsigned b) {
  unsigned h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  h *= 0x297A2D39u;
  h ^= h >> 15;
  return (double)(h & 0xFFFFFF) / (double)0x800000 - 1.0;   // [-1, 1)
}

// Inverse iteration for eigenvalue lam of the tridiagonal (d, e): x <- (T - lam)^{-1} x,
// with Gaussian elimination and row interchanges.  Scratch: u0,u1,u2,mul (n each), piv (n).
__device__ void tri_lu(int n, const double* d, const double* e, double lam, double tiny, double* u0, double* u1,
                       double* u2, double* mul, unsigned char* piv) {
  double r0 = d[0] - lam, r1 = (n > 1) ? e[0] : 0.0, r2 = 0.0;
  for (int i = 0; i < n - 1; ++i) {
    const double s0 = e[i], s1 = d[i + 1] - lam, s2 = (i + 2 < n) ? e[i + 1] : 0.0;
    double m, n0, n1;
    if (fabs(r0) >= fabs(s0)) {
      if (r0 == 0.0) r0 = tiny;
      m = s0 / r0;
      piv[i] = 0;
      u0[i] = r0; u1[i] = r1; u2[i] = r2;
      n0 = s1 - m * r1;
      n1 = s2 - m * r2;
    } else {
      m = r0 / s0;
      piv[i] = 1;
      u0[i] = s0; u1[i] = s1; u2[i] = s2;
      n0 = r1 - m * s1;
      n1 = r2 - m * s2;
    }
    mul[i] = m;
    r0 = n0; r1 = n1; r2 = 0.0;
  }
  if (r0 == 0.0) r0 = tiny;
  u0[n - 1] = r0;
  u1[n - 1] = 0.0;
  u2[n - 1] = 0.0;
}

__device__ void tri_solve(int n, const double* u0, const double* u1, const double* u2, const double* mul,
                          const unsigned char* piv, double* x) {
  for (int i = 0; i < n - 1; ++i) {
    if (piv[i]) { const double t = x[i]; x[i] = x[i + 1]; x[i + 1] = t; }
    x[i + 1] -= mul[i] * x[i];
  }
  for (int i = n - 1; i >= 0; --i) {
    double s = x[i];
    if (i + 1 < n) s -= u1[i] * x[i + 1];
    if (i + 2 < n) s -= u2[i] * x[i + 2];
    x[i] = s / u0[i];
  }
}

// work layout (doubles): [T-sized scratch not needed] per-thread LU scratch 5n x k, V-tri n x k, gram k x k
__global__ __launch_bounds__(kDenseThreads) void syev_lowest_kernel(int n, int k, double* __restrict__ T,
                                                                   double* __restrict__ wout,
                                                                   double* __restrict__ V,
                                                                   double* __restrict__ work, int* info) {
  __shared__ double d[kSyevMaxN], e[kSyevMaxN], e2[kSyevMaxN], tau[kSyevMaxN];
  __shared__ double v[kSyevMaxN], p[kSyevMaxN];
  __shared__ double lam[PASE_MAX_NEV];
  __shared__ int cstart[PASE_MAX_NEV + 1];
  __shared__ double red[kDenseWaves];
  __shared__ double sh_scalar[4];
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  if (tid == 0) *info = 0;

  // ---- 1. Householder tridiagonalisation (T row-major, symmetric, full storage)
  for (int j = 0; j + 2 < n; ++j) {
    const int m = n - j - 1;
    const double* row = T + (size_t)j * n + j + 1;     // x = T[j][j+1 .. n-1]
    double part = 0.0;
    for (int i = 1 + tid; i < m; i += kDenseThreads) part += row[i] * row[i];
    const double xnorm2 = block_sum(part, red);
    const double alpha = row[0];
    if (xnorm2 == 0.0) {
      if (tid == 0) { tau[j] = 0.0; e[j] = alpha; d[j] = T[(size_t)j * n + j]; }
      __syncthreads();
      continue;
    }
    const double beta = -copysign(sqrt(alpha * alpha + xnorm2), alpha);
    const double tj = (beta - alpha) / beta;
    const double scale = 1.0 / (alpha - beta);
    for (int i = tid; i < m; i += kDenseThreads) v[i] = (i == 0) ? 1.0 : row[i] * scale;
    __syncthreads();
    // store v (i >= 1) in row j for the back-transformation
    for (int i = 1 + tid; i < m; i += kDenseThreads) T[(size_t)j * n + j + 1 + i] = v[i];
    if (tid == 0) { tau[j] = tj; e[j] = beta; d[j] = T[(size_t)j * n + j]; }
    // p = tau A22 v
    double* A22 = T + (size_t)(j + 1) * n + (j + 1);
    for (int r = wave; r < m; r += kDenseWaves) {
      const double* ar = A22 + (size_t)r * n;
      double s = 0.0;
      for (int c = lane; c < m; c += 64) s = fma(ar[c], v[c], s);
      s = wave_sum(s);
      if (lane == 0) p[r] = tj * s;
    }
    __syncthreads();
    double pv = 0.0;
    for (int i = tid; i < m; i += kDenseThreads) pv += p[i] * v[i];
    const double K = 0.5 * tj * block_sum(pv, red);
    // w = p - K v (in p)
    for (int i = tid; i < m; i += kDenseThreads) p[i] -= K * v[i];
    __syncthreads();
    for (long long q = tid; q < (long long)m * m; q += kDenseThreads) {
      const int r = (int)(q / m), c = (int)(q % m);
      A22[(size_t)r * n + c] -= v[r] * p[c] + p[r] * v[c];
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (n >= 2) {
      d[n - 2] = T[(size_t)(n - 2) * n + (n - 2)];
      e[n - 2] = T[(size_t)(n - 2) * n + (n - 1)];
    }
    d[n - 1] = T[(size_t)(n - 1) * n + (n - 1)];
    e[n - 1] = 0.0;
    if (n >= 2) tau[n - 2] = 0.0;
    tau[n - 1] = 0.0;
  }
  __syncthreads();
  for (int i = tid; i < n; i += kDenseThreads) e2[i] = e[i] * e[i];
  // Gershgorin interval and pivmin
  if (tid == 0) {
    double lo = DBL_MAX, hi = -DBL_MAX, emax = 0.0;
    for (int i = 0; i < n; ++i) {
      const double r = ((i > 0) ? fabs(e[i - 1]) : 0.0) + ((i + 1 < n) ? fabs(e[i]) : 0.0);
      lo = fmin(lo, d[i] - r);
      hi = fmax(hi, d[i] + r);
      if (i + 1 < n) emax = fmax(emax, e2[i]);
    }
    const double tnorm = fmax(fabs(lo), fabs(hi));
    lo -= 2.0 * DBL_EPSILON * tnorm * n + DBL_MIN;
    hi += 2.0 * DBL_EPSILON * tnorm * n + DBL_MIN;
    sh_scalar[0] = lo;
    sh_scalar[1] = hi;
    sh_scalar[2] = DBL_MIN * fmax(1.0, emax);
    sh_scalar[3] = tnorm;
  }
  __syncthreads();
  const double glo = sh_scalar[0], ghi = sh_scalar[1], pivmin = sh_scalar[2], tnorm = sh_scalar[3];

  // ---- 2. bisection: thread t finds the (t+1)-th smallest eigenvalue
  for (int t = tid; t < k; t += kDenseThreads) {
    double lo = glo, hi = ghi;
    for (int it = 0; it < 200; ++it) {
      const double mid = 0.5 * (lo + hi);
      if (hi - lo <= 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + pivmin || mid == lo || mid == hi) break;
      if (sturm_count(n, d, e2, mid, pivmin) <= t) lo = mid;
      else hi = mid;
    }
    lam[t] = 0.5 * (lo + hi);
  }
  __syncthreads();

  // ---- 3. inverse iteration; tight clusters (gap < 1e-7 |T|) are re-orthogonalised in place
  const double clus = 1e-7 * tnorm;
  if (tid == 0) {
    int nc = 0;
    for (int t = 0; t < k; ++t)
      if (t == 0 || lam[t] - lam[t - 1] > clus) cstart[nc++] = t;
    cstart[nc] = k;
    sh_scalar[0] = (double)nc;
  }
  __syncthreads();
  const int ncl = (int)sh_scalar[0];
  double* Vt = work;                                   // n x k tridiagonal eigenvectors
  double* G = work + (size_t)n * k;                    // k x k Gram
  double* scr = G + (size_t)k * k;                     // per-cluster scratch, 5n each
  unsigned char* pivs = (unsigned char*)(scr + (size_t)5 * n * k);
  const double tiny = DBL_EPSILON * tnorm;
  for (int c = tid; c < ncl; c += kDenseThreads) {
    double* u0 = scr + (size_t)5 * n * c;
    double* u1 = u0 + n;
    double* u2 = u1 + n;
    double* mul = u2 + n;
    double* x = mul + n;
    unsigned char* piv = pivs + (size_t)n * c;
    for (int t = cstart[c]; t < cstart[c + 1]; ++t) {
      double lt = lam[t];
      if (t > cstart[c]) lt = fmax(lt, lam[t - 1] + 10.0 * tiny);   // keep shifts distinct in a cluster
      tri_lu(n, d, e, lt, tiny, u0, u1, u2, mul, piv);
      for (int i = 0; i < n; ++i) x[i] = hash_unit(t + 1, i + 1);
      for (int it = 0; it < 3; ++it) {
        double xm = 0.0;
        for (int i = 0; i < n; ++i) xm = fmax(xm, fabs(x[i]));
        if (xm > 0.0)
          for (int i = 0; i < n; ++i) x[i] /= xm;
        tri_solve(n, u0, u1, u2, mul, piv, x);
        for (int q = cstart[c]; q < t; ++q) {
          double s = 0.0;
          for (int i = 0; i < n; ++i) s += Vt[(size_t)i * k + q] * x[i];
          for (int i = 0; i < n; ++i) x[i] -= s * Vt[(size_t)i * k + q];
        }
        double nn = 0.0;
        for (int i = 0; i < n; ++i) nn += x[i] * x[i];
        nn = sqrt(nn);
        for (int i = 0; i < n; ++i) x[i] /= nn;
      }
      for (int i = 0; i < n; ++i) Vt[(size_t)i * k + t] = x[i];
    }
  }
  __syncthreads();

  // ---- 3b. two passes of Cholesky-QR over the n x k block (global orthogonality)
  for (int pass = 0; pass < 2; ++pass) {
    for (int q = tid; q < k * k; q += kDenseThreads) {
      const int a = q / k, b = q % k;
      if (b > a) continue;
      double s = 0.0;
      for (int i = 0; i < n; ++i) s += Vt[(size_t)i * k + a] * Vt[(size_t)i * k + b];
      G[(size_t)a * k + b] = s;
    }
    __syncthreads();
    if (tid == 0) {   // k x k Cholesky, lower, in G
      for (int j = 0; j < k; ++j) {
        double s = G[(size_t)j * k + j];
        for (int l = 0; l < j; ++l) s -= G[(size_t)j * k + l] * G[(size_t)j * k + l];
        if (!(s > 0.0)) { *info = 1; s = 1.0; }
        const double djj = sqrt(s);
        G[(size_t)j * k + j] = djj;
        for (int i = j + 1; i < k; ++i) {
          double t = G[(size_t)i * k + j];
          for (int l = 0; l < j; ++l) t -= G[(size_t)i * k + l] * G[(size_t)j * k + l];
          G[(size_t)i * k + j] = t / djj;
        }
      }
    }
    __syncthreads();
    // rows of Vt: x^T <- x^T L^{-T}, i.e. solve L y = x per row
    for (int i = tid; i < n; i += kDenseThreads) {
      double* xr = Vt + (size_t)i * k;
      for (int j = 0; j < k; ++j) {
        double s = xr[j];
        for (int l = 0; l < j; ++l) s -= G[(size_t)j * k + l] * xr[l];
        xr[j] = s / G[(size_t)j * k + j];
      }
    }
    __syncthreads();
  }

  // ---- 4. back-transformation V = H_0 ... H_{n-3} Vt
  for (int i = tid; i < n * k; i += kDenseThreads) V[i] = Vt[i];
  __syncthreads();
  for (int j = n - 3; j >= 0; --j) {
    const double tj = tau[j];
    if (tj == 0.0) continue;
    const int m = n - j - 1;
    // p[c] = tau * sum_i v_i V[j+1+i][c]
    for (int c = wave; c < k; c += kDenseWaves) {
      double s = 0.0;
      for (int i = lane; i < m; i += 64) {
        const double vi = (i == 0) ? 1.0 : T[(size_t)j * n + j + 1 + i];
        s = fma(vi, V[(size_t)(j + 1 + i) * k + c], s);
      }
      s = wave_sum(s);
      if (lane == 0) p[c] = tj * s;
    }
    __syncthreads();
    for (int q = tid; q < m * k; q += kDenseThreads) {
      const int i = q / k, c = q % k;
      const double vi = (i == 0) ? 1.0 : T[(size_t)j * n + j + 1 + i];
      V[(size_t)(j + 1 + i) * k + c] -= vi * p[c];
    }
    __syncthreads();
  }
  for (int t = tid; t < k; t += kDenseThreads) wout[t] = lam[t];
}

}  // namespace

void launch_cholesky(int n, double* A, int lda, int* info, hipStream_t s) {
  cholesky_kernel<<<1, kDenseThreads, 0, s>>>(n, A, lda, info);
}

void launch_trinv(int n, const double* L, int ldl, double* Li, int ldi, hipStream_t s) {
  trinv_kernel<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(n, L, ldl, Li, ldi);
}

size_t syev_work_doubles(int n, int k) {
  // Vt (n k) + G (k k) + scratch (5 n k) + pivots (n k bytes, in doubles)
  return (size_t)n * k + (size_t)k * k + (size_t)5 * n * k + ((size_t)n * k + 7) / 8 + 8;
}

void launch_syev_lowest(int n, int k, double* T, double* w, double* V, double* work, int* info, hipStream_t s) {
  syev_lowest_kernel<<<1, kDenseThreads, 0, s>>>(n, k, T, w, V, work, info);
}

int syev_max_n() { return kSyevMaxN; }

namespace {
__global__ void symmetrize_kernel(int n, double* A) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (long long)n * n) return;
  const int i = (int)(q / n), j = (int)(q % n);
  if (j >= i) return;
  const double v = 0.5 * (A[(size_t)i * n + j] + A[(size_t)j * n + i]);
  A[(size_t)i * n + j] = v;
  A[(size_t)j * n + i] = v;
}
}  // namespace

void launch_symmetrize(int n, double* A, hipStream_t s) {
  symmetrize_kernel<<<(unsigned)(((long long)n * n + kBlock - 1) / kBlock), kBlock, 0, s>>>(n, A);
}

}  // namespace pase
