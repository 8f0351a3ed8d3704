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
#include <algorithm>
#include <cfloat>

#include "internal.hpp"

namespace pase {

namespace {

constexpr int kDenseThreads = 1024;
constexpr int kDenseWaves = kDenseThreads / 64;
constexpr int kSyevMaxN = 1024;

__global__ void zero_info_kernel(int* info) { *info = 0; }
__global__ void fold_err_kernel(int* info, const int* err) {
  if (*err) *info = 2;
}

__global__ void copy_lam_kernel(int k, const double* __restrict__ a, double* __restrict__ b) {
  for (int i = threadIdx.x; i < k; i += blockDim.x) b[i] = a[i];
}

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Fixed-order block sum with one barrier: alternate between two scratch rows
// (the barrier of the call in between orders reuse of a row).
__device__ double block_sum1(double v, double (*red)[kDenseWaves], int& parity) {
  v = wave_sum(v);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* r = red[parity];
  parity ^= 1;
  if (lane == 0) r[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < kDenseWaves; ++w) s += r[w];
  return s;
}

// Cholesky of an n x n SPD matrix in place (lower), one block.  A pivot at or below
// n * eps * max_i A[i][i] counts as a breakdown (numerically rank-deficient Gram matrices are
// reported, not factored).
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

// ---- eigensolver
// Layout of the eigensolver work area (doubles):
//   tri[0:n) = d, tri[n:2n) = e, tri[2n:3n) = tau, tri[3n:3n+8) = scalars
//   lam[k], Vt[n*k] (tridiagonal eigenvectors), wy[kWyB * k * 2]
constexpr int kWyB = 32;          // reflectors per block of the back-transformation

__device__ __forceinline__ double hash_unit(unsigned a, unsigned b) {
  unsigned h = a * 0x9E3779B1u ^ (b + 0x7F4A7C15u) * 0x85EBCA77u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  h *= 0x297A2D39u;
  h ^= h >> 15;
  return (double)(h & 0xFFFFFF) / (double)0x800000 - 1.0;   // [-1, 1)
}

// 1. Householder reduction of the symmetric n x n matrix T (row-major, full
// storage) to tridiagonal form.  Reflector j is stored in row j of T
// (entries j+2 .. n-1; its entry j+1 is an implicit 1), tau[j] in tri.
// Step j applies A22 <- A22 - v w^T - w v^T (w = p - K v, p = tau A22 v) and,
// in the same pass over the trailing block, forms the product of the next
// reflector with the updated block (look-ahead): row j+1 is updated first, the
// next reflector built from it, then one read-modify-write sweep of the rest.
// Threads own columns (coalesced across threads); symmetry gives
// (A v)_r = sum_c A[c][r] v_c.
__device__ __forceinline__ void colsum_map(int cols, int& G, int t, int& r, int& g) {
  G = 1024 / cols;
  if (G > 16) G = 16;
  if (G < 1) G = 1;
  r = t % cols;
  g = t / cols;
}

__global__ __launch_bounds__(kDenseThreads) void tridiag_kernel(int n, double* __restrict__ T,
                                                               double* __restrict__ tri) {
  __shared__ double va[kSyevMaxN], pa[kSyevMaxN], vb[kSyevMaxN], pb[kSyevMaxN];
  __shared__ double part[kDenseThreads];
  __shared__ double red[2][kDenseWaves];
  int parity = 0;
  const int tid = threadIdx.x;
  double* d = tri;
  double* e = tri + n;
  double* tau = tri + 2 * n;
  double* v = va; double* p = pa; double* v2 = vb; double* p2 = pb;
  double tcur = 0.0, K = 0.0;
  if (n >= 3) {
    // reflector 0 from row 0 and p0 = tau0 A22 v0
    const int m = n - 1;
    double* row = T + 1;
    double part0 = 0.0;
    for (int i = 1 + tid; i < m; i += kDenseThreads) part0 = fma(row[i], row[i], part0);
    const double xn2 = block_sum1(part0, red, parity);
    const double alpha = row[0];
    if (tid == 0) d[0] = T[0];
    if (xn2 == 0.0) {
      tcur = 0.0;
      for (int i = tid; i < m; i += kDenseThreads) v[i] = (i == 0) ? 1.0 : 0.0;
      if (tid == 0) { tau[0] = 0.0; e[0] = alpha; }
    } else {
      const double beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
      tcur = (beta - alpha) / beta;
      const double sc = 1.0 / (alpha - beta);
      for (int i = tid; i < m; i += kDenseThreads) {
        const double vi = (i == 0) ? 1.0 : row[i] * sc;
        v[i] = vi;
        if (i > 0) row[i] = vi;
      }
      if (tid == 0) { tau[0] = tcur; e[0] = beta; }
    }
    __syncthreads();
    const double* A22 = T + (size_t)n + 1;
    int G, r, g;
    colsum_map(m, G, tid, r, g);
    double acc = 0.0;
    if (tid < G * m)
      for (int c = g; c < m; c += G) acc = fma(A22[(size_t)c * n + r], v[c], acc);
    part[tid] = acc;
    __syncthreads();
    double pv = 0.0;
    if (tid < m) {
      double sum = 0.0;
      for (int q = 0; q < G; ++q) sum += part[q * m + tid];
      p[tid] = tcur * sum;
      pv = p[tid] * v[tid];
    }
    K = 0.5 * tcur * block_sum1(pv, red, parity);
  }
  for (int j = 0; j + 2 < n; ++j) {
    const int m = n - j - 1;
    double* A22 = T + (size_t)(j + 1) * n + (j + 1);
    const bool has_next = (j + 3 < n);
    // (a) row 0 of A22: update and the norm of its tail (next reflector's x)
    double nrm = 0.0;
    const double w0 = p[0] - K * v[0];
    for (int c = tid; c < m; c += kDenseThreads) {
      const double a = A22[c] - (v[0] * (p[c] - K * v[c]) + w0 * v[c]);
      A22[c] = a;
      if (c >= 2) nrm = fma(a, a, nrm);
    }
    const double xn2 = block_sum1(nrm, red, parity);
    double tnext = 0.0;
    if (has_next) {
      const double alpha = A22[1];
      if (xn2 == 0.0) {
        for (int i = tid; i < m - 1; i += kDenseThreads) v2[i] = (i == 0) ? 1.0 : 0.0;
        if (tid == 0) { tau[j + 1] = 0.0; e[j + 1] = alpha; }
      } else {
        const double beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
        tnext = (beta - alpha) / beta;
        const double sc = 1.0 / (alpha - beta);
        for (int i = tid; i < m - 1; i += kDenseThreads) {
          const double vi = (i == 0) ? 1.0 : A22[1 + i] * sc;
          v2[i] = vi;
          if (i > 0) A22[1 + i] = vi;
        }
        if (tid == 0) { tau[j + 1] = tnext; e[j + 1] = beta; }
      }
      if (tid == 0) d[j + 1] = A22[0];
    }
    __syncthreads();
    // (b) fused sweep over A33 = A22[1:, 1:]: update, and partial products with v2
    const int cols = m - 1;
    int G, r, g;
    colsum_map(cols, G, tid, r, g);
    double acc = 0.0;
    if (tid < G * cols) {
      const int rr = r + 1;
      const double vr = v[rr], wr = p[rr] - K * v[rr];
      constexpr int kBatch = 10;
      for (int c0 = 1 + g; c0 < m; c0 += kBatch * G) {
        double a[kBatch];
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {          // issue the batch's loads together
          const int c = c0 + u * G;
          a[u] = (c < m) ? A22[(size_t)c * n + rr] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kBatch; ++u) {
          const int c = c0 + u * G;
          if (c < m) {
            const double nv = a[u] - (v[c] * wr + (p[c] - K * v[c]) * vr);
            A22[(size_t)c * n + rr] = nv;
            if (has_next) acc = fma(nv, v2[c - 1], acc);
          }
        }
      }
    }
    part[tid] = acc;
    __syncthreads();
    double pv = 0.0;
    if (has_next && tid < cols) {
      double sum = 0.0;
      for (int q = 0; q < G; ++q) sum += part[q * cols + tid];
      p2[tid] = tnext * sum;
      pv = p2[tid] * v2[tid];
    }
    const double Kn = 0.5 * tnext * block_sum1(pv, red, parity);
    double* t1 = v; v = v2; v2 = t1;
    double* t2 = p; p = p2; p2 = t2;
    tcur = tnext;
    K = Kn;
  }
  __syncthreads();
  if (tid == 0) {
    if (n < 3) d[0] = T[0];
    if (n >= 2) {
      d[n - 2] = T[(size_t)(n - 2) * n + (n - 2)];
      e[n - 2] = T[(size_t)(n - 2) * n + (n - 1)];
      tau[n - 2] = 0.0;
    }
    d[n - 1] = T[(size_t)(n - 1) * n + (n - 1)];
    e[n - 1] = 0.0;
    tau[n - 1] = 0.0;
    double lo = DBL_MAX, hi = -DBL_MAX, emax = 0.0;
    for (int i = 0; i < n; ++i) {
      const double rr = ((i > 0) ? fabs(e[i - 1]) : 0.0) + ((i + 1 < n) ? fabs(e[i]) : 0.0);
      lo = fmin(lo, d[i] - rr);
      hi = fmax(hi, d[i] + rr);
      if (i + 1 < n) emax = fmax(emax, e[i] * e[i]);
    }
    const double tnorm = fmax(fabs(lo), fabs(hi));
    double* sc = tri + 3 * n;
    sc[0] = lo - (2.0 * DBL_EPSILON * tnorm * n + DBL_MIN);
    sc[1] = hi + (2.0 * DBL_EPSILON * tnorm * n + DBL_MIN);
    sc[2] = DBL_MIN * fmax(1.0, emax);
    sc[3] = tnorm;
  }
}

// 1b. Cooperative Householder tridiagonalisation for n <= kCoopMaxN.
//
// NW workgroups each hold a cyclic slab of rows of T in LDS (block b owns rows
// i with i % NW == b), so the matrix never streams from L2.  Step j needs the
// product p_j = tau_j A22 v_j over all rows and row j+1 after update j; both are
// exchanged through global memory with one software grid barrier per step:
//   - after the barrier every block reads p_j (m values) and row j+1 as it was
//     before update j, forms w_j = p_j - K_j v_j, updates its copy of row j+1
//     and builds reflector j+1 from it (every block the same way, so v_{j+1} is
//     identical everywhere without a second barrier);
//   - one pass over its own rows applies update j and accumulates
//     p_{j+1} = tau_{j+1} A v_{j+1}; the owner of row j+2 publishes that row.
// The grid is launched 8x larger than NW and only blocks with index % 8 == 0
// work, so the working blocks share one XCD (blocks are dealt round-robin over
// the 8 XCDs) and its L2.  Exchanged data is written and read with device-scope
// atomic accesses (L1 bypass); the barrier below orders them.
constexpr int kCoopMaxN = 512;
constexpr int kCoopThreads = 512;
constexpr int kCoopWaves = kCoopThreads / 64;

__device__ __forceinline__ double ld_agent(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Software barriers of the NW working blocks (bounded spin: on timeout a block
// raises *err and returns, so every wave exits).
constexpr unsigned kCoopMaxSpins = 1u << 22;

__device__ bool barrier_spin(unsigned* counter, unsigned target, int* err, bool acquire) {
  __shared__ int ok;
  if (threadIdx.x == 0) {
    unsigned spins = 0;
    ok = 1;
    while ((acquire ? __hip_atomic_load(counter, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT)
                    : __hip_atomic_load(counter, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) < target) {
      __builtin_amdgcn_s_sleep(1);
      if (++spins > kCoopMaxSpins || __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) {
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        ok = 0;
        break;
      }
    }
  }
  __syncthreads();
  return ok != 0;
}

// Agent-scope barrier: release fence and acquire spin (L2 write-back and
// invalidate included), valid wherever the blocks run.
__device__ bool grid_barrier_fenced(unsigned* counter, unsigned target, int* err) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
  }
  return barrier_spin(counter, target, err, true);
}

// Barrier for blocks that share one XCD (checked at kernel start): every
// exchanged value is written and read with device-scope accesses, which bypass
// the per-CU L1 and meet in that XCD's L2, so it suffices that this block's
// stores have completed before it arrives; no L2 write-back or invalidate.
__device__ bool grid_barrier_xcd(unsigned* counter, unsigned target, int* err) {
  __asm__ volatile("s_waitcnt vmcnt(0)" ::: "memory");   // this wave's stores are at the L2
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_fetch_add(counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  return barrier_spin(counter, target, err, false);
}

__device__ __forceinline__ unsigned xcc_id() {
  // HW_REG_XCC_ID (hardware register 20), bits [3:0]: the XCD this wave runs on
  return (unsigned)__builtin_amdgcn_s_getreg((3 << 11) | 20) & 0xFu;
}

__device__ double block_sum_c(double v, double (*red)[kCoopWaves], int& parity) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  double* r = red[parity];
  parity ^= 1;
  if (lane == 0) r[wave] = v;
  __syncthreads();
  double s = 0.0;
  for (int w = 0; w < kCoopWaves; ++w) s += r[w];
  return s;
}

// reflector from x = row[0 .. mm-1]: v[0] = 1, v[i] = x[i] / (alpha - beta); returns tau
__device__ double make_reflector(const double* row, int mm, double* v, double& beta_out,
                                 double (*red)[kCoopWaves], int& parity) {
  double part = 0.0;
  for (int i = 1 + threadIdx.x; i < mm; i += kCoopThreads) part = fma(row[i], row[i], part);
  const double xn2 = block_sum_c(part, red, parity);
  const double alpha = row[0];
  if (xn2 == 0.0) {
    for (int i = threadIdx.x; i < mm; i += kCoopThreads) v[i] = (i == 0) ? 1.0 : 0.0;
    beta_out = alpha;
    __syncthreads();
    return 0.0;
  }
  const double beta = -copysign(sqrt(alpha * alpha + xn2), alpha);
  const double sc = 1.0 / (alpha - beta);
  for (int i = threadIdx.x; i < mm; i += kCoopThreads) v[i] = (i == 0) ? 1.0 : row[i] * sc;
  beta_out = beta;
  __syncthreads();
  return (beta - alpha) / beta;
}

__global__ __launch_bounds__(kCoopThreads) void tridiag_coop_kernel(int n, int NW, double* __restrict__ T,
                                                                   double* __restrict__ tri,
                                                                   double* __restrict__ xchg,
                                                                   unsigned* counter, int* err,
                                                                   unsigned* xccs) {
  if (blockIdx.x % 8 != 0) return;
  const int b = blockIdx.x / 8;
  if (b >= NW) return;
  const unsigned myxcc = xcc_id();
  if (threadIdx.x == 0) __hip_atomic_store(&xccs[b], myxcc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  extern __shared__ double dyn[];
  const int R = (n + NW - 1) / NW;               // owned rows (cyclic)
  double* slab = dyn;                            // R x n
  double* v = slab + (size_t)R * n;              // reflector j     (indexed by global column - (j+1))
  double* w = v + kCoopMaxN;                     // w_j / scratch
  double* v2 = w + kCoopMaxN;                    // reflector j+1
  double* prow = v2 + kCoopMaxN;                 // row j+1 copy (global column index)
  double* pp = prow + kCoopMaxN;                 // p_j (indexed like v)
  __shared__ double red[2][kCoopWaves];
  int parity = 0;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  double* pbuf = xchg;                           // 2 x kCoopMaxN, alternating per step
  double* rbuf = xchg + 2 * kCoopMaxN;           // 2 x kCoopMaxN
  double* d = tri;
  double* e = tri + n;
  double* tau = tri + 2 * n;
  unsigned target = 0;
  // load owned rows
  for (int q = 0; q < R; ++q) {
    const int r = q * NW + b;
    for (int c = tid; c < n; c += kCoopThreads) slab[(size_t)q * n + c] = (r < n) ? T[(size_t)r * n + c] : 0.0;
  }
  // reflector 0 from row 0 (every block)
  for (int c = tid; c < n; c += kCoopThreads) prow[c] = T[c];
  __syncthreads();
  double beta0;
  double tcur = make_reflector(prow + 1, n - 1, v, beta0, red, parity);
  if (b == 0 && tid == 0) { d[0] = prow[0]; e[0] = beta0; tau[0] = tcur; }
  // p_0 over owned rows r >= 1: p[r-1] = tau0 sum_{c>=1} A[r][c] v[c-1]
  for (int q = wave; q < R; q += kCoopWaves) {
    const int r = q * NW + b;
    if (r < 1 || r >= n) continue;
    const double* ar = slab + (size_t)q * n;
    double acc = 0.0;
    for (int c = 1 + lane; c < n; c += 64) acc = fma(ar[c], v[c - 1], acc);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if (lane == 0) __hip_atomic_store(&pbuf[r - 1], tcur * acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (1 % NW == b)
    for (int c = tid; c < n; c += kCoopThreads)
      __hip_atomic_store(&rbuf[c], slab[(size_t)(1 / NW) * n + c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  target += NW;
  if (!grid_barrier_fenced(counter, target, err)) return;
  // reflector 0 goes into row 0 of T only now: every block has read that row before the barrier
  if (b == 0) for (int i = 1 + tid; i < n - 1; i += kCoopThreads) T[i + 1] = v[i];
  // the cheap barrier only if every working block shares this XCD
  __shared__ int one_xcd;
  if (threadIdx.x == 0) {
    int same = 1;
    for (int q = 0; q < NW; ++q)
      same &= (__hip_atomic_load(&xccs[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == myxcc) ? 1 : 0;
    one_xcd = same;
  }
  __syncthreads();
  const bool fast_barrier = one_xcd != 0;
  for (int j = 0; j + 2 < n; ++j) {
    const int m = n - j - 1;                     // trailing size of step j (global cols j+1 .. n-1)
    const int par = j & 1;
    const double* pin = pbuf + par * kCoopMaxN;
    const double* rin = rbuf + par * kCoopMaxN;
    double* pout = pbuf + (par ^ 1) * kCoopMaxN;
    double* rout = rbuf + (par ^ 1) * kCoopMaxN;
    for (int i = tid; i < m; i += kCoopThreads) pp[i] = ld_agent(pin + i);
    for (int c = tid; c < n; c += kCoopThreads) prow[c] = (c >= j + 1) ? ld_agent(rin + c) : 0.0;
    __syncthreads();
    double pv = 0.0;
    for (int i = tid; i < m; i += kCoopThreads) pv = fma(pp[i], v[i], pv);
    const double K = 0.5 * tcur * block_sum_c(pv, red, parity);
    for (int i = tid; i < m; i += kCoopThreads) w[i] = pp[i] - K * v[i];
    __syncthreads();
    // row j+1 after update j: prow[c] -= v[0] w[c'] + w[0] v[c']  (c' = c - (j+1))
    const double v0 = v[0], w0 = w[0];
    for (int c = j + 1 + tid; c < n; c += kCoopThreads) {
      const int cc = c - (j + 1);
      prow[c] -= v0 * w[cc] + w0 * v[cc];
    }
    __syncthreads();
    const bool has_next = (j + 3 < n);
    double tnext = 0.0, bnext = 0.0;
    if (has_next) {
      tnext = make_reflector(prow + (j + 2), m - 1, v2, bnext, red, parity);
      if (b == 0 && tid == 0) { d[j + 1] = prow[j + 1]; e[j + 1] = bnext; tau[j + 1] = tnext; }
      if ((j + 1) % NW == b)
        for (int i = 1 + tid; i < m - 1; i += kCoopThreads) T[(size_t)(j + 1) * n + (j + 2) + i] = v2[i];
    } else if (b == 0 && tid == 0) {
      d[j + 1] = prow[j + 1];
      e[j + 1] = prow[j + 2];
      tau[j + 1] = 0.0;
    }
    // update j on owned rows r >= j+2 (columns >= j+2) and p_{j+1} = tnext A v2
    for (int q = wave; q < R; q += kCoopWaves) {
      const int r = q * NW + b;
      if (r < j + 2 || r >= n) continue;
      double* ar = slab + (size_t)q * n;
      const int rr = r - (j + 1);
      const double vr = v[rr], wr = w[rr];
      double acc = 0.0;
      for (int c = j + 2 + lane; c < n; c += 64) {
        const int cc = c - (j + 1);
        const double a = ar[c] - (vr * w[cc] + wr * v[cc]);
        ar[c] = a;
        acc = fma(a, v2[c - (j + 2)], acc);
      }
      if (has_next) {
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
        if (lane == 0)
          __hip_atomic_store(&pout[r - (j + 2)], tnext * acc, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    __syncthreads();
    if (has_next && (j + 2) % NW == b) {
      const double* ar = slab + (size_t)((j + 2) / NW) * n;
      for (int c = j + 2 + tid; c < n; c += kCoopThreads)
        __hip_atomic_store(&rout[c], ar[c], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (!has_next) {
      // last step: row n-1 after update j is in the slab of its owner
      if ((n - 1) % NW == b && tid == 0) d[n - 1] = slab[(size_t)((n - 1) / NW) * n + (n - 1)];
      break;
    }
    double* t1 = v; v = v2; v2 = t1;
    tcur = tnext;
    target += NW;
    if (!(fast_barrier ? grid_barrier_xcd(counter, target, err) : grid_barrier_fenced(counter, target, err))) return;
  }
}

__global__ __launch_bounds__(256) void tri_finish_kernel(int n, double* __restrict__ tri) {
  // Gershgorin interval, pivmin and |T| of the tridiagonal (one block)
  __shared__ double r_lo[4], r_hi[4], r_e[4];
  double* d = tri;
  double* e = tri + n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  double lo = DBL_MAX, hi = -DBL_MAX, emax = 0.0;
  for (int i = tid; i < n; i += 256) {
    const double el = (i > 0) ? e[i - 1] : 0.0;
    const double er = (i + 1 < n) ? e[i] : 0.0;
    const double rr = fabs(el) + fabs(er);
    lo = fmin(lo, d[i] - rr);
    hi = fmax(hi, d[i] + rr);
    emax = fmax(emax, er * er);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o, 64));
    hi = fmax(hi, __shfl_xor(hi, o, 64));
    emax = fmax(emax, __shfl_xor(emax, o, 64));
  }
  if (lane == 0) { r_lo[wave] = lo; r_hi[wave] = hi; r_e[wave] = emax; }
  __syncthreads();
  if (tid == 0) {
    for (int w = 1; w < 4; ++w) {
      lo = fmin(lo, r_lo[w]);
      hi = fmax(hi, r_hi[w]);
      emax = fmax(emax, r_e[w]);
    }
    e[n - 1] = 0.0;
    const double tnorm = fmax(fabs(lo), fabs(hi));
    double* sc = tri + 3 * n;
    sc[0] = lo - (2.0 * DBL_EPSILON * tnorm * n + DBL_MIN);
    sc[1] = hi + (2.0 * DBL_EPSILON * tnorm * n + DBL_MIN);
    sc[2] = DBL_MIN * fmax(1.0, emax);
    sc[3] = tnorm;
  }
}

__global__ void coop_reset_kernel(unsigned* counter, int* err) {
  *counter = 0u;
  *err = 0;
}

__device__ int sturm_count(int n, const double* d, const double* e2, double x, double pivmin) {
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

// 2. The (t+1)-th smallest eigenvalue of the tridiagonal, t = blockIdx.x, by
// multisection: each of the 64 lanes counts eigenvalues below one of 64
// interior points of the current interval (Sturm sequence), the interval
// shrinks 65-fold per round.
__global__ __launch_bounds__(64) void bisect_kernel(int n, const double* __restrict__ tri,
                                                   double* __restrict__ lam) {
  __shared__ double d[kSyevMaxN], e2[kSyevMaxN];
  const int t = blockIdx.x, lane = threadIdx.x;
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
    const int cnt = sturm_count(n, d, e2, x, pivmin);
    const unsigned long long below = __ballot(cnt <= t);
    const int c = __popcll(below);                   // lanes 0..c-1 have count <= t
    const double nlo = (c > 0) ? __shfl(x, c - 1, 64) : lo;
    const double nhi = (c < 64) ? __shfl(x, c < 64 ? c : 63, 64) : hi;
    if (nlo == lo && nhi == hi) break;
    lo = nlo;
    hi = nhi;
  }
  if (lane == 0) lam[t] = 0.5 * (lo + hi);
}

// 3. Eigenvectors of the tridiagonal by inverse iteration, one block per
// eigenvalue, stored vector-major (vector j at Vt[j*n .. j*n+n)).  Lane 0 runs
// the sequential LU (Gaussian elimination with row interchanges) and the
// solves in LDS.  Members of a cluster of (nearly) equal eigenvalues start
// from different pseudo-random vectors, so they span the cluster's invariant
// subspace; the Cholesky-QR passes that follow make them orthonormal (mixing
// eigenvectors whose eigenvalues differ by g changes residuals by at most g
// times the remaining contamination, which three iterations bring to the
// rounding level).
__global__ __launch_bounds__(64) void invit_kernel(int n, int k, const double* __restrict__ tri,
                                                  const double* __restrict__ lam, double* __restrict__ Vt) {
  __shared__ double d[kSyevMaxN], e[kSyevMaxN];
  __shared__ double u0[kSyevMaxN], u1[kSyevMaxN], u2[kSyevMaxN], x[kSyevMaxN];
  __shared__ unsigned char piv[kSyevMaxN];
  __shared__ double mulv[kSyevMaxN];
  const int j = blockIdx.x, lane = threadIdx.x;
  const double tnorm = tri[3 * n + 3];
  for (int i = lane; i < n; i += 64) {
    d[i] = tri[i];
    e[i] = tri[n + i];
    x[i] = hash_unit(j + 1, i + 1);
  }
  __syncthreads();
  const double tiny = DBL_EPSILON * tnorm;
  const double lj = lam[j];
  if (lane == 0) {
    double r0 = d[0] - lj, r1 = (n > 1) ? e[0] : 0.0, r2 = 0.0;
    for (int i = 0; i < n - 1; ++i) {
      const double s0 = e[i], s1 = d[i + 1] - lj, s2 = (i + 2 < n) ? e[i + 1] : 0.0;
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
    if (r0 == 0.0) r0 = tiny;
    u0[n - 1] = 1.0 / r0; u1[n - 1] = 0.0; u2[n - 1] = 0.0;
    for (int i = 0; i < n - 1; ++i) u0[i] = 1.0 / u0[i];   // solves multiply by the pivot inverses
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
        const double v = (x[i] - u1[i] * xp1 - u2[i] * xp2) * u0[i];
        x[i] = v;
        xp2 = xp1;
        xp1 = v;
      }
    }
    __syncthreads();
  }
  double nn = 0.0;
  for (int i = lane; i < n; i += 64) nn = fma(x[i], x[i], nn);
  nn = wave_sum(nn);
  const double rn = 1.0 / sqrt(nn);
  for (int i = lane; i < n; i += 64) Vt[(size_t)j * n + i] = x[i] * rn;
}

// 4a. Gram of the k vectors: G[a][b] = v_a . v_b for a >= b (one thread per pair).
__global__ __launch_bounds__(kBlock) void vgram_kernel(int n, int k, const double* __restrict__ Vt,
                                                      double* __restrict__ G) {
  // one wave per entry (a, b), b <= a: lanes stride the vector index, then a shuffle tree
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int q = blockIdx.x * (kBlock / 64) + wave;
  if (q >= k * k) return;
  const int a = q / k, b = q % k;
  if (b > a) return;
  const double* va = Vt + (size_t)a * n;
  const double* vb = Vt + (size_t)b * n;
  double s0 = 0.0, s1 = 0.0;
  int i = lane;
  for (; i + 64 < n; i += 128) {
    s0 = fma(va[i], vb[i], s0);
    s1 = fma(va[i + 64], vb[i + 64], s1);
  }
  if (i < n) s0 = fma(va[i], vb[i], s0);
  double sum = s0 + s1;
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) sum += __shfl_xor(sum, o, 64);
  if (lane == 0) G[(size_t)a * k + b] = sum;
}

// 4b. L = chol(G), G <- L^{-1} (lower), in LDS, one block.  k <= kOrthoMaxK.
//
// Right-looking Cholesky with one barrier per pivot: in step j every thread
// reads the (final) pivot G_jj and applies the rank-1 update of the trailing
// lower triangle with the unscaled column j divided by the pivot; the scaling of
// column j by 1/sqrt(pivot) is deferred to step j+1, where nothing reads it.
// The inverse is then formed column by column (forward substitution, one thread
// per column), its strictly lower part stored transposed in the unused upper
// triangle of the LDS array.
constexpr int kOrthoMaxK = 128;
__global__ __launch_bounds__(kDenseThreads) void cholinv_kernel(int k, double* __restrict__ G, int* info) {
  __shared__ double L[kOrthoMaxK][kOrthoMaxK + 1];
  __shared__ double dinv[kOrthoMaxK];
  __shared__ double wmax[kDenseThreads / 64];
  __shared__ int bad;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  if (tid == 0) bad = 0;
  double dm = 0.0;
  for (int q = tid; q < k * k; q += kDenseThreads) {
    const int a = q / k, b = q % k;
    const double g = G[(size_t)a * k + b];
    L[a][b] = (b <= a) ? g : 0.0;
    if (a == b) dm = fmax(dm, g);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) dm = fmax(dm, __shfl_xor(dm, o, 64));
  if (lane == 0) wmax[wave] = dm;
  __syncthreads();
  dm = 0.0;
  for (int w = 0; w < kDenseThreads / 64; ++w) dm = fmax(dm, wmax[w]);
  const double ptol = k * DBL_EPSILON * dm;   // pivots at or below this count as rank deficiency
  // 2D thread layout for the trailing updates: 32 x 32
  const int tx = tid & 31, ty = tid >> 5;
  double prev_scale = 1.0;
  for (int j = 0; j < k; ++j) {
    const double dj = L[j][j];
    const double pe = (dj > 0.0) ? dj : 1.0;
    if (tid == 0 && !(dj > ptol)) bad = 1;
    if (j > 0) {   // finish column j-1 (nothing reads it in this step)
      for (int i = j - 1 + tid; i < k; i += kDenseThreads)
        L[i][j - 1] = (i == j - 1) ? 1.0 / prev_scale : L[i][j - 1] * prev_scale;
    }
    const double rp = 1.0 / pe;
    for (int i = j + 1 + ty; i < k; i += 32) {
      const double lij = L[i][j] * rp;
      for (int l = j + 1 + tx; l <= i; l += 32) L[i][l] = fma(-lij, L[l][j], L[i][l]);
    }
    prev_scale = 1.0 / sqrt(pe);
    __syncthreads();
  }
  if (tid == 0) L[k - 1][k - 1] = 1.0 / prev_scale;   // column k-1 has no entries below the diagonal
  __syncthreads();
  for (int c = tid; c < k; c += kDenseThreads) dinv[c] = 1.0 / L[c][c];
  __syncthreads();
  // inverse X = L^{-1}, right-looking: entry (i, c), i > c, lives at L[c][i] (zero on entry) and
  // accumulates sum_{l < j} L[i][l] X[l][c] until step j = i, when X[i][c] = -acc dinv[i]; at step
  // j every pair (i > j, c <= j) adds L[i][j] X[j][c], with row j's values formed on the fly (row
  // j - 1 is scaled in the same step: nothing reads it any more), one barrier per step
  for (int j = 0; j < k; ++j) {
    if (j > 0)
      for (int c = tid; c < j - 1; c += kDenseThreads) L[c][j - 1] = -L[c][j - 1] * dinv[j - 1];
    const double dj = dinv[j];
    for (int i = j + 1 + ty; i < k; i += 32) {
      const double lij = L[i][j];
      for (int c = tx; c <= j; c += 32) {
        const double xjc = (c == j) ? dj : -L[c][j] * dj;
        L[c][i] = fma(lij, xjc, L[c][i]);
      }
    }
    __syncthreads();
  }
  for (int c = tid; c < k - 1; c += kDenseThreads) L[c][k - 1] = -L[c][k - 1] * dinv[k - 1];
  __syncthreads();
  for (int q = tid; q < k * k; q += kDenseThreads) {
    const int i = q / k, c = q % k;
    G[q] = (i > c) ? L[c][i] : ((i == c) ? dinv[c] : 0.0);
  }
  if (tid == 0 && bad) *info = 1;
}

// 4b'. The same for k <= 64 in one wave.  Cholesky by rows: lane i keeps row i of the
// trailing matrix in registers (static indices: every loop is unrolled to 64 and guarded by
// k); at pivot j the scaled column j is broadcast through LDS and each lane updates its row.
// Inverse by columns: L goes to LDS by rows, lane c forms column c of L^{-1} by forward
// substitution, reading the rows of L as LDS broadcasts (x[l] = 0 for l < c, so the sums need
// no lane-dependent bounds).
__global__ __launch_bounds__(64) void cholinv_wave_kernel(int k, double* __restrict__ G, int* info) {
  __shared__ double col[64];
  __shared__ double Ls[64][65];
  const int i = threadIdx.x;
  double r[64];
  // unconditional loads from clamped addresses, all in flight at once, then the selects
  const int ic = (i < k) ? i : k - 1;
#pragma unroll
  for (int l = 0; l < 64; ++l) r[l] = G[ic * k + ((l < k) ? l : k - 1)];
#pragma unroll
  for (int l = 0; l < 64; ++l) r[l] = (i < k && l < k && l <= i) ? r[l] : (l == i ? 1.0 : 0.0);
  double dm = (i < k) ? r[0] : 0.0;
#pragma unroll
  for (int l = 1; l < 64; ++l)
    if (l == i && i < k) dm = r[l];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) dm = fmax(dm, __shfl_xor(dm, o, 64));
  // G = I + E with max |E| <= 1e-9 (the second pass of a Cholesky-QR): L = I + tril(E) - diag(E) / 2
  // and L^{-1} = I - tril(E) + diag(E) / 2 up to O(k |E|^2) <= 1e-16, so no factorisation is needed
  double em = 0.0;
#pragma unroll
  for (int l = 0; l < 64; ++l) em = fmax(em, fabs(r[l] - ((l == i) ? 1.0 : 0.0)));
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) em = fmax(em, __shfl_xor(em, o, 64));
  if (em <= 1e-9) {
    if (i < k) {
#pragma unroll
      for (int l = 0; l < 64; ++l)
        if (l < k) G[i * k + l] = (l < i) ? -r[l] : ((l == i) ? 1.0 - 0.5 * (r[l] - 1.0) : 0.0);
    }
    return;
  }
  const double ptol = k * DBL_EPSILON * dm;   // pivots at or below this count as rank deficiency
  bool bad = false;
#pragma unroll
  for (int j = 0; j < 64; ++j) {
    if (j < k) {                              // uniform; the unrolled body keeps static indices
      // one LDS exchange per pivot: the unscaled column j (its entry j is the pivot d); row i
      // becomes L[i][j] = a_ij / sqrt(d) and the trailing update is a_il -= a_ij a_lj / d
      col[i] = r[j];
      __syncthreads();
      const double d = col[j];
      bad = bad || !(d > ptol);
      const double pe = (d > 0.0) ? d : 1.0;
      const double rd = 1.0 / pe;
      const double sq = sqrt(pe);
      const double lij = r[j] * rd;
      // unconditional update: in a lane i < l it only writes the strict upper triangle of row i,
      // which no later pivot reads (col[l] is read only for l > j >= i) and is cleared below
#pragma unroll
      for (int l = j + 1; l < 64; ++l) r[l] = fma(-lij, col[l], r[l]);
      r[j] = (i > j) ? r[j] / sq : ((i == j) ? sq : r[j]);
      __syncthreads();
    }
  }
#pragma unroll
  for (int l = 0; l < 64; ++l) Ls[i][l] = (l <= i) ? r[l] : 0.0;
  __syncthreads();
  // column c = i of X = L^{-1}
  const int c = i;
  double x[64];
#pragma unroll
  for (int a = 0; a < 64; ++a) {
    if (a >= k) continue;                     // uniform
    double acc[4] = {0.0, 0.0, 0.0, 0.0};     // four short chains instead of one long one
#pragma unroll
    for (int l = 0; l < a; ++l) acc[l & 3] = fma(Ls[a][l], x[l], acc[l & 3]);
    const double rhs = (a == c) ? 1.0 : -((acc[0] + acc[1]) + (acc[2] + acc[3]));
    x[a] = (a < c) ? 0.0 : rhs / Ls[a][a];
  }
  if (c < k) {
#pragma unroll
    for (int a = 0; a < 64; ++a)
      if (a < k) G[a * k + c] = x[a];
  }
  if (i == 0 && bad) *info = 1;
}

// 4c. Vo = L^{-1} Vi in the vector index: vo_j = sum_{l <= j} Li[j][l] vi_l.
__global__ __launch_bounds__(kBlock) void vorth_apply_kernel(int n, int k, const double* __restrict__ Li,
                                                            const double* __restrict__ Vi,
                                                            double* __restrict__ Vo) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (long long)n * k) return;
  const int j = (int)(q / n), i = (int)(q % n);
  double s = 0.0;
  for (int l = 0; l <= j; ++l) s = fma(Li[(size_t)j * k + l], Vi[(size_t)l * n + i], s);
  Vo[q] = s;
}

// 4d. S matrices of the blocked back-transformation, one block of kWyB
// reflectors per workgroup: S[r][r] = tau_r, S[0:r, r] = -tau_r S[0:r,0:r] (Y^T Y)[0:r, r].
__global__ __launch_bounds__(kBlock) void wy_prep_kernel(int n, const double* __restrict__ T,
                                                        const double* __restrict__ tri,
                                                        double* __restrict__ Sall) {
  __shared__ double YY[kWyB][kWyB + 1];
  __shared__ double S[kWyB][kWyB + 1];
  const int blk = blockIdx.x;
  const int j0 = blk * kWyB;
  const int nref = n - 2;
  const int b = (nref - j0 < kWyB) ? nref - j0 : kWyB;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const double* tau = tri + 2 * n;
  for (int pr = wave; pr < b * b; pr += kBlock / 64) {
    const int l = pr / b, r = pr % b;
    if (l > r) continue;
    const int jl = j0 + l, jr = j0 + r;
    double s2 = 0.0;
    for (int i = jr + 1 + lane; i < n; i += 64) {
      const double yl = (i == jl + 1) ? 1.0 : T[(size_t)jl * n + i];
      const double yr = (i == jr + 1) ? 1.0 : T[(size_t)jr * n + i];
      s2 = fma(yl, yr, s2);
    }
    s2 = wave_sum(s2);
    if (lane == 0) { YY[l][r] = s2; YY[r][l] = s2; }
  }
  __syncthreads();
  if (wave == 0) {
    for (int r = 0; r < b; ++r) {
      double s2 = 0.0;
      if (lane < r)
        for (int q = lane; q < r; ++q) s2 = fma(S[lane][q], YY[q][r], s2);
      if (lane < r) S[lane][r] = -tau[j0 + r] * s2;     // lane l owns row l of S
      if (lane == r) S[r][r] = tau[j0 + r];
      if (lane > r && lane < b) S[lane][r] = 0.0;
    }
  }
  __syncthreads();
  double* So = Sall + (size_t)blk * kWyB * kWyB;
  for (int q = tid; q < kWyB * kWyB; q += kBlock) {
    const int r = q / kWyB, c = q % kWyB;
    So[q] = (r < b && c < b) ? S[r][c] : 0.0;
  }
}

// 4e. Back-transformation of one eigenvector per workgroup, x <- Q x with
// Q = prod_blocks (I - Y S Y^T), last block first; result stored into column c
// of V (n x k, row-major).
__global__ __launch_bounds__(kBlock) void wy_apply_kernel(int n, int k, const double* __restrict__ T,
                                                         const double* __restrict__ Sall,
                                                         const double* __restrict__ Vt, double* __restrict__ V) {
  __shared__ double x[kSyevMaxN];
  __shared__ double w1[kWyB], w2[kWyB];
  const int c = blockIdx.x;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  for (int i = tid; i < n; i += kBlock) x[i] = Vt[(size_t)c * n + i];
  __syncthreads();
  const int nref = n - 2;
  const int nblk = (nref + kWyB - 1) / kWyB;
  for (int blk = nblk - 1; blk >= 0; --blk) {
    const int j0 = blk * kWyB;
    const int b = (nref - j0 < kWyB) ? nref - j0 : kWyB;
    for (int r = wave; r < b; r += kBlock / 64) {
      const int jr = j0 + r;
      double s2 = 0.0;
      for (int i = jr + 1 + lane; i < n; i += 64) {
        const double yr = (i == jr + 1) ? 1.0 : T[(size_t)jr * n + i];
        s2 = fma(yr, x[i], s2);
      }
      s2 = wave_sum(s2);
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
    for (int i = j0 + 1 + tid; i < n; i += kBlock) {
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
  for (int i = tid; i < n; i += kBlock) V[(size_t)i * k + c] = x[i];
}

}  // namespace

void launch_cholesky(int n, double* A, int lda, int* info, hipStream_t s) {
  cholesky_kernel<<<1, kDenseThreads, 0, s>>>(n, A, lda, info);
}

void launch_trinv(int n, const double* L, int ldl, double* Li, int ldi, hipStream_t s) {
  trinv_kernel<<<(n + kBlock - 1) / kBlock, kBlock, 0, s>>>(n, L, ldl, Li, ldi);
}

size_t syev_work_doubles(int n, int k) {
  // tri (3n + 8) + lam (k) + Vt, Vt2 (n k each) + G (k k) + S blocks (+ a second k x k
  // for the triangular inverse when k exceeds the one-block Cholesky-inverse)
  const size_t nblk = (size_t)(n + kWyB - 1) / kWyB + 1;
  const size_t big = (k > kOrthoMaxK)
                         ? (size_t)k * k + std::max(cholesky_large_scratch_doubles(k), trinv_large_scratch_doubles(k))
                         : 0;
  return (size_t)3 * n + 8 + (size_t)k + (size_t)2 * n * k + (size_t)k * k + nblk * kWyB * kWyB +
         4 * kCoopMaxN + 72 + big;
}

int syev_max_k() { return kOrthoMaxK; }

void launch_cholinv(int k, double* G, int* info, hipStream_t s) {
  if (k <= 64) cholinv_wave_kernel<<<1, 64, 0, s>>>(k, G, info);
  else cholinv_kernel<<<1, kDenseThreads, 0, s>>>(k, G, info);
}

void launch_syev_lowest(int n, int k, double* T, double* w, double* V, double* work, int* info, hipStream_t s) {
  double* tri = work;
  double* lam = tri + 3 * n + 8;
  double* Vt = lam + k;
  double* Vt2 = Vt + (size_t)n * k;
  double* G = Vt2 + (size_t)n * k;
  double* Sall = G + (size_t)k * k;
  const size_t nblk = (size_t)(n + kWyB - 1) / kWyB + 1;
  double* xchg = Sall + nblk * kWyB * kWyB;                  // 4 x kCoopMaxN
  unsigned* coop_counter = (unsigned*)(xchg + 4 * kCoopMaxN);
  int* coop_err = (int*)(coop_counter + 1);
  zero_info_kernel<<<1, 1, 0, s>>>(info);
  const unsigned gb = (unsigned)((k * k + kBlock / 64 - 1) / (kBlock / 64));   // vgram: one wave per entry
  const unsigned ab = (unsigned)(((long long)n * k + kBlock - 1) / kBlock);
  // cooperative path: NW blocks whose row slabs fit in LDS
  int NW = 0;
  if (n >= 8 && n <= kCoopMaxN) {
    for (int nw = 8; nw <= 32; nw *= 2) {
      const size_t lds = ((size_t)((n + nw - 1) / nw) * n + 5 * kCoopMaxN) * sizeof(double);
      if (lds <= 150 * 1024) { NW = nw; break; }
    }
  }
  if (NW > 0) {
    const size_t lds = ((size_t)((n + NW - 1) / NW) * n + 5 * kCoopMaxN) * sizeof(double);
    coop_reset_kernel<<<1, 1, 0, s>>>(coop_counter, coop_err);
    tridiag_coop_kernel<<<8 * NW, kCoopThreads, lds, s>>>(n, NW, T, tri, xchg, coop_counter, coop_err,
                                                        (unsigned*)(xchg + 4 * kCoopMaxN + 1));
    tri_finish_kernel<<<1, 256, 0, s>>>(n, tri);
  } else {
    tridiag_kernel<<<1, kDenseThreads, 0, s>>>(n, T, tri);
  }
  bisect_kernel<<<k, 64, 0, s>>>(n, tri, lam);
  invit_kernel<<<k, 64, 0, s>>>(n, k, tri, lam, Vt);
  double* G2 = xchg + 4 * kCoopMaxN + 8;                    // after the barrier counter and flag
  for (int pass = 0; pass < 2; ++pass) {
    vgram_kernel<<<gb, kBlock, 0, s>>>(n, k, Vt, G);
    if (k <= kOrthoMaxK) {
      launch_cholinv(k, G, info, s);
      vorth_apply_kernel<<<ab, kBlock, 0, s>>>(n, k, G, Vt, Vt2);
    } else {
      // blocked Cholesky and triangular inverse (MFMA panel updates), scratch after G2
      launch_cholesky_large(k, G, k, G2 + (size_t)k * k, info, s);
      launch_trinv_large(k, G, k, G2, k, G2 + (size_t)k * k, s);
      vorth_apply_kernel<<<ab, kBlock, 0, s>>>(n, k, G2, Vt, Vt2);
    }
    double* t = Vt; Vt = Vt2; Vt2 = t;
  }
  if (n > 2) wy_prep_kernel<<<(n - 2 + kWyB - 1) / kWyB, kBlock, 0, s>>>(n, T, tri, Sall);
  wy_apply_kernel<<<k, kBlock, 0, s>>>(n, k, T, Sall, Vt, V);
  copy_lam_kernel<<<1, 256, 0, s>>>(k, lam, w);
  if (NW > 0) fold_err_kernel<<<1, 1, 0, s>>>(info, coop_err);
}

int syev_max_n() { return kSyevMaxN; }

void launch_tri_finish(int n, double* tri, hipStream_t s) { tri_finish_kernel<<<1, 256, 0, s>>>(n, tri); }

void launch_wy_prep(int n, const double* T, const double* tri, double* Sall, hipStream_t s) {
  if (n > 2) wy_prep_kernel<<<(n - 2 + kWyB - 1) / kWyB, kBlock, 0, s>>>(n, T, tri, Sall);
}

void launch_vorth2(int n, int k, double* Vt, double* Vt2, double* G, int* info, hipStream_t s) {
  const unsigned gb = (unsigned)((k * k + kBlock / 64 - 1) / (kBlock / 64));   // vgram: one wave per entry
  const unsigned ab = (unsigned)(((long long)n * k + kBlock - 1) / kBlock);
  for (int pass = 0; pass < 2; ++pass) {
    vgram_kernel<<<gb, kBlock, 0, s>>>(n, k, pass ? Vt2 : Vt, G);
    launch_cholinv(k, G, info, s);
    vorth_apply_kernel<<<ab, kBlock, 0, s>>>(n, k, G, pass ? Vt2 : Vt, pass ? Vt : Vt2);
  }
}

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
