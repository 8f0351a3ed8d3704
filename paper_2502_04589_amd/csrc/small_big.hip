// Structured solver of the augmented eigenproblem (Alg. 3 step 5) for large coarse
// spaces: N_H up to kBigMaxH and k up to kBK pairs.
//
// Same method as small.hip: in the M-orthonormal basis [P L_B^{-T} Phi, W_perp L^{-T}]
// the augmented matrix is Tt = [[Theta, Gt], [Gt^T, H]] (Theta diagonal), and for a
// shift mu, (Tt - mu I)^{-1} is applied exactly through the k x k Schur complement
//     S(mu) = H - mu I - Gt^T (Theta - mu I)^{-1} Gt;
// Sylvester's law of inertia counts the eigenvalues below mu as
// #{theta_j < mu} + (negative eigenvalues of S(mu)).  Here the rows of Gt (N_H x k, a few
// MB) no longer fit one thread each: they stream from L2 in 4-row steps into the MFMA
// operands, S(mu) (k x k) and its in-place LU live in LDS, and the two work vectors of
// each pair live in a global scratch slice.
#include <cfloat>

#include "internal.hpp"

namespace pase {

namespace {

constexpr int kBK = 128;           // k <= kBK
constexpr int kBT = 512;           // threads per workgroup
constexpr int kBW = kBT / 64;
constexpr int kBigMaxH = 4096;     // N_H limit
constexpr int kBMaxFactor = 3;
constexpr int kBMaxSolve = 6;

typedef double double4_t __attribute__((ext_vector_type(4)));

struct BLds {
  double S[kBK][kBK + 1];          // S(mu), then its LU factors (unit-lower multipliers below the diagonal)
  double part[4][kBK];
  double vh[kBK];                  // a k-vector (x_H, y_H, ...)
  double vb[kBK];
  double red[kBW];
  int ipiv[kBK];
};

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// fixed-order block sum; every thread gets the result
__device__ double bsum(double v, double* red) {
  v = wsum(v);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kBW; ++w) s += red[w];
  return s;
}

__device__ __forceinline__ double hash_pm1(unsigned a, unsigned b) {
  unsigned h = a * 0x9E3779B1u ^ (b + 0x632BE5ABu) * 0x85EBCA77u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  h *= 0x297A2D39u;
  h ^= h >> 15;
  return (double)(h & 0xFFFFFF) / (double)0x800000 - 1.0;
}

// S = H - mu I - sum_r d_r g_r g_r^T, d_r = 1 / (theta_r - mu), g_r = row r of Gt, on
// v_mfma_f64_16x16x4f64.  A step covers 4 rows, and lane (li, lk) loads Gt[r0 + lk][16 c + li]
// for the 8 column blocks c.  Wave w accumulates the tiles w, w + 8, ... of the T x T grid.  With
// T = 8 (k > 112) tile t of wave w is (t, w): its A operand is block t (a compile-time index) and
// its B operand block w, loaded once more per step; for smaller T the blocks of each tile are
// picked out of the row by a run-time index.
// acc (this wave's tiles w, w + 8, ... of the T x T grid) += sum over rows rb <= r < re of
// d_r g_r g_r^T (re > rb)
__device__ void schur_rows_acc(int rb, int re, int k, const double* __restrict__ Gt,
                               const double* __restrict__ theta, double mu, double4_t (&acc)[8]) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int T = (k + 15) >> 4, TT = T * T;
  const bool full = (T == 8);
  const int colw = 16 * wave + li;     // B-operand column of every tile when T = 8
  // the next step's row values are loaded while this step's MFMAs run (two waves per SIMD
  // leave little else to hide the L2 latency)
  double gn[8], gwn, thn;
  auto fetch = [&](int r0) {
    const int row = r0 + lk;
    const int rc = (row < re) ? row : re - 1;
    thn = theta[rc];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
      const int col = 16 * c + li;
      gn[c] = (c < T && col < k) ? Gt[(size_t)rc * k + col] : 0.0;
    }
    gwn = (full && colw < k) ? Gt[(size_t)rc * k + colw] : 0.0;
  };
  fetch(rb);
  for (int r0 = rb; r0 < re; r0 += 4) {
    const bool rok = r0 + lk < re;
    const double dv = rok ? 1.0 / (thn - mu) : 0.0;
    double g[8];
#pragma unroll
    for (int c = 0; c < 8; ++c) g[c] = rok ? gn[c] : 0.0;
    const double gw = rok ? gwn : 0.0;
    if (r0 + 4 < re) fetch(r0 + 4);
    if (full) {
#pragma unroll
      for (int t = 0; t < 8; ++t) acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(dv * g[t], gw, acc[t], 0, 0, 0);
      continue;
    }
#pragma unroll
    for (int t = 0; t < 8; ++t) {
      const int tt = wave + 8 * t;
      if (tt < TT) {
        const int ti = tt / T, tj = tt - (tt / T) * T;
        double av = 0.0, bv = 0.0;
#pragma unroll
        for (int c = 0; c < 8; ++c) {
          if (c == ti) av = g[c];
          if (c == tj) bv = g[c];
        }
        acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(dv * av, bv, acc[t], 0, 0, 0);
      }
    }
  }
}

__device__ void form_schur_big(int nH, int k, const double* __restrict__ Gt, const double* __restrict__ theta,
                               const double* __restrict__ Hm, double mu, BLds& L) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int T = (k + 15) >> 4, TT = T * T;
  double4_t acc[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) acc[t] = (double4_t){0.0, 0.0, 0.0, 0.0};
  schur_rows_acc(0, nH, k, Gt, theta, mu, acc);
  __syncthreads();
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int tt = wave + 8 * t;
    if (tt < TT) {
      const int ti = tt / T, tj = tt - (tt / T) * T;
      const int c = 16 * tj + li;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 16 * ti + lk + 4 * q;
        if (r < k && c < k) L.S[r][c] = Hm[(size_t)r * k + c] - ((r == c) ? mu : 0.0) - acc[t][q];
      }
    }
  }
  __syncthreads();
}

// In-place LU with partial pivoting of L.S (k x k); rows are exchanged whole, so the
// multipliers below the diagonal follow their rows (LAPACK getrf order).
__device__ void lu_big(int k, BLds& L) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int tx = tid & 31, ty = tid >> 5;   // 32 columns x 16 rows
  __shared__ int piv_s;
  for (int j = 0; j < k; ++j) {
    if (wave == 0) {
      // largest |S[r][j]| over r >= j, ties to the lowest row: key = magnitude bits with the
      // low 7 bits replaced by 127 - r
      unsigned long long key = 0ull;
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int r = lane + 64 * h;
        if (r >= j && r < k) {
          const unsigned long long kk =
              ((unsigned long long)__double_as_longlong(fabs(L.S[r][j])) & ~127ull) | (unsigned long long)(127 - r);
          key = (kk > key) ? kk : key;
        }
      }
#pragma unroll
      for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long k2 = (unsigned long long)__shfl_xor((long long)key, o, 64);
        key = (k2 > key) ? k2 : key;
      }
      if (lane == 0) {
        const int p = 127 - (int)(key & 127ull);
        piv_s = (p >= j && p < k) ? p : j;
        L.ipiv[j] = piv_s;
      }
    }
    __syncthreads();
    const int p = piv_s;
    if (p != j) {
      for (int t = tid; t < k; t += kBT) {
        const double a = L.S[j][t];
        L.S[j][t] = L.S[p][t];
        L.S[p][t] = a;
      }
    }
    __syncthreads();
    const double rp = 1.0 / L.S[j][j];
    for (int r = j + 1 + ty; r < k; r += 16) {
      const double lr = L.S[r][j] * rp;
      for (int c = j + 1 + tx; c < k; c += 32) L.S[r][c] = fma(-lr, L.S[j][c], L.S[r][c]);
      if (tx == 0) L.S[r][j] = lr;
    }
    __syncthreads();
  }
}

__device__ __forceinline__ double lane_get(double b0, double b1, int j) {
  const double v0 = __shfl(b0, j & 63, 64), v1 = __shfl(b1, j & 63, 64);
  return (j < 64) ? v0 : v1;
}

// Wave 0: solves S y = b with the factors of lu_big; entries r = lane and r = lane + 64 in
// (b0, b1) on entry, y on exit.
__device__ void lu_solve_big(int k, const BLds& L, double& b0, double& b1) {
  const int lane = threadIdx.x & 63;
  for (int j = 0; j < k; ++j) {
    const int p = L.ipiv[j];
    if (p != j) {
      const double bj = lane_get(b0, b1, j), bp = lane_get(b0, b1, p);
      if (lane == (j & 63)) { if (j < 64) b0 = bp; else b1 = bp; }
      if (lane == (p & 63)) { if (p < 64) b0 = bj; else b1 = bj; }
    }
  }
  for (int j = 0; j < k; ++j) {
    const double zj = lane_get(b0, b1, j);
    if (lane > j && lane < k) b0 = fma(-L.S[lane][j], zj, b0);
    if (lane + 64 > j && lane + 64 < k) b1 = fma(-L.S[lane + 64][j], zj, b1);
  }
  for (int j = k - 1; j >= 0; --j) {
    const double yj = lane_get(b0, b1, j) / L.S[j][j];
    if (lane == (j & 63)) { if (j < 64) b0 = yj; else b1 = yj; }
    if (lane < j) b0 = fma(-L.S[lane][j], yj, b0);
    if (lane + 64 < j && lane + 64 < k) b1 = fma(-L.S[lane + 64][j], yj, b1);
  }
}

// out[a] = sum_{r < nH} c_r x_r Gt[r][a] (c_r = 1 / (theta_r - mu) when dmu is set, else 1), a < k,
// into LDS; x is a global vector of the workgroup.  With dmu, c_r x_r is formed once per row into
// cx (nH doubles of the workgroup's global scratch, not x) instead of by every column's thread.
__device__ void colsum_big(int nH, int k, const double* __restrict__ Gt, const double* __restrict__ theta,
                           bool dmu, double mu, const double* x, double* cx, BLds& L, double* out) {
  const int tid = threadIdx.x;
  const int a = tid & (kBK - 1), grp = tid >> 7;
  const double* v = x;
  if (dmu) {
    for (int r = tid; r < nH; r += kBT) cx[r] = x[r] / (theta[r] - mu);
    __syncthreads();
    v = cx;
  }
  // rows r = grp + 4 j; four rows per trip, so four row loads are in flight at once
  double s = 0.0;
  if (a < k) {
    const double* __restrict__ g = Gt + a;
    int r = grp;
    for (; r + 12 < nH; r += 16) {
      const double g0 = g[(size_t)r * k], g1 = g[(size_t)(r + 4) * k];
      const double g2 = g[(size_t)(r + 8) * k], g3 = g[(size_t)(r + 12) * k];
      const double v0 = v[r], v1 = v[r + 4], v2 = v[r + 8], v3 = v[r + 12];
      s = fma(v0, g0, s);
      s = fma(v1, g1, s);
      s = fma(v2, g2, s);
      s = fma(v3, g3, s);
    }
    for (; r < nH; r += 4) s = fma(v[r], g[(size_t)r * k], s);
  }
  L.part[grp][a] = s;
  __syncthreads();
  if (tid < k) out[tid] = (L.part[0][tid] + L.part[1][tid]) + (L.part[2][tid] + L.part[3][tid]);
  __syncthreads();
}

// Gt^T is kept column-major as GtT (k x nH, GtT[a nH + r] = Gt[r][a]) for the products Gt v: a thread
// takes a row r, reads its k entries with loads that are consecutive across the wave, and the LDS
// vector v by broadcasts; no cross-lane reductions.
__global__ void gt_transpose_kernel(int nH, int k, const double* __restrict__ Gt, double* __restrict__ GtT) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (long long)nH * k) return;
  const int r = (int)(q / k), a = (int)(q - (long long)r * k);
  GtT[(size_t)a * nH + r] = Gt[q];
}

__device__ __forceinline__ double gt_row_dot(int nH, int k, const double* __restrict__ GtT, int r, const double* v) {
  double s0 = 0.0, s1 = 0.0;
  int a = 0;
  for (; a + 1 < k; a += 2) {
    s0 = fma(GtT[(size_t)a * nH + r], v[a], s0);
    s1 = fma(GtT[(size_t)(a + 1) * nH + r], v[a + 1], s1);
  }
  if (a < k) s0 = fma(GtT[(size_t)a * nH + r], v[a], s0);
  return s0 + s1;
}

// One workgroup per pair i: shift-invert solves at the start vector's Rayleigh quotient (or
// sigma[i]), then Rayleigh-quotient shifts, as in the one-workgroup solver; the unit vector goes to
// Vt[i*n ..] (n = N_H + k) and its Rayleigh quotient to rq[i].  xs: 2 n doubles per pair.
__global__ __launch_bounds__(kBT) void srqi_big_kernel(int nH, int k, const double* __restrict__ theta,
                                                     const double* __restrict__ Gt, const double* __restrict__ GtT,
                                                     const double* __restrict__ Hm,
                                                     const double* __restrict__ sigma,
                                                     const double* __restrict__ X0, double scale,
                                                     const double* __restrict__ tolv, double* __restrict__ Vt,
                                                     double* __restrict__ rq, double* __restrict__ xs) {
  __shared__ BLds L;
  const int i = blockIdx.x;
  const int n = nH + k;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  double* x = xs + (size_t)i * 2 * n;
  double* y = x + n;
  double nx = 0.0;
  for (int r = tid; r < n; r += kBT) {
    const double v = X0 ? X0[(size_t)r * k + i] : hash_pm1((unsigned)i + 1u, (unsigned)r);
    x[r] = v;
    nx = fma(v, v, nx);
  }
  nx = bsum(nx, L.red);
  const double inx = 1.0 / sqrt(nx);
  for (int r = tid; r < n; r += kBT) x[r] *= inx;
  __syncthreads();
  double mu = sigma[i];
  if (X0) {
    // x^T Tt x = sum_r x_r (theta_r x_r + 2 g_r . x_H) + x_H^T H x_H
    for (int a = tid; a < k; a += kBT) L.vh[a] = x[nH + a];
    __syncthreads();
    double part = 0.0;
    for (int r = tid; r < nH; r += kBT) part = fma(x[r], fma(theta[r], x[r], 2.0 * gt_row_dot(nH, k, GtT, r, L.vh)), part);
    if (tid < k) {
      double hx = 0.0;
      for (int b = 0; b < k; ++b) hx = fma(Hm[(size_t)tid * k + b], L.vh[b], hx);
      part = fma(L.vh[tid], hx, part);
    }
    mu = bsum(part, L.red);
  }
  double rho = mu;
  const double stop = (tolv ? fmax(1e-13, 1e-12 * tolv[i]) : 1e-13) * scale;
  form_schur_big(nH, k, Gt, theta, Hm, mu, L);
  lu_big(k, L);
  int nfac = 1, since = 0;
  const int hold = X0 ? 3 : 2;
  for (int it = 0; it < kBMaxSolve; ++it) {
    if (since >= hold && nfac < kBMaxFactor) {
      mu = rho;
      form_schur_big(nH, k, Gt, theta, Hm, mu, L);
      lu_big(k, L);
      ++nfac;
      since = 0;
    }
    // rhs = x_H - Gt^T (d o x_Theta), then y_H = S^{-1} rhs
    colsum_big(nH, k, Gt, theta, true, mu, x, y, L, L.vb);   // y is free until y_Theta below
    if (wave == 0) {
      double b0 = (lane < k) ? x[nH + lane] - L.vb[lane] : 0.0;
      double b1 = (lane + 64 < k) ? x[nH + lane + 64] - L.vb[lane + 64] : 0.0;
      lu_solve_big(k, L, b0, b1);
      if (lane < k) L.vh[lane] = b0;
      if (lane + 64 < k) L.vh[lane + 64] = b1;
    }
    __syncthreads();
    // y_Theta = d o (x_Theta - Gt y_H), y_H as solved
    for (int r = tid; r < nH; r += kBT) y[r] = (x[r] - gt_row_dot(nH, k, GtT, r, L.vh)) / (theta[r] - mu);
    for (int a = tid; a < k; a += kBT) y[nH + a] = L.vh[a];
    __syncthreads();
    double yy = 0.0, yx = 0.0;
    for (int r = tid; r < n; r += kBT) {
      yy = fma(y[r], y[r], yy);
      yx = fma(y[r], x[r], yx);
    }
    yy = bsum(yy, L.red);
    yx = bsum(yx, L.red);
    const double ny = sqrt(yy);
    rho = mu + yx / yy;                       // Tt y = x + mu y
    const double dm = rho - mu;
    double rr = 0.0;
    for (int r = tid; r < n; r += kBT) {
      const double e = (x[r] - dm * y[r]) / ny;
      rr = fma(e, e, rr);
      x[r] = y[r] / ny;
    }
    rr = bsum(rr, L.red);
    __syncthreads();
    ++since;
    if (!(rr == rr) || !(ny == ny)) break;
    if (it >= 1 && sqrt(rr) <= stop) break;
  }
  __syncthreads();
  for (int r = tid; r < n; r += kBT) Vt[(size_t)i * n + r] = x[r];
  if (tid == 0) rq[i] = rho;
}

// Rayleigh quotient and residual of column i of an orthonormal Vt with the explicit operator:
// w = Tt v (into the pair's scratch), rho = v.w, res = ||w - rho v||.
__global__ __launch_bounds__(kBT) void srr_big_kernel(int nH, int k, const double* __restrict__ theta,
                                                    const double* __restrict__ Gt, const double* __restrict__ GtT,
                                                    const double* __restrict__ Hm,
                                                    const double* __restrict__ Vt, double* __restrict__ rq,
                                                    double* __restrict__ res, double* __restrict__ xs) {
  __shared__ BLds L;
  const int i = blockIdx.x;
  const int n = nH + k;
  const int tid = threadIdx.x;
  const double* x = Vt + (size_t)i * n;
  double* w = xs + (size_t)i * 2 * n;
  for (int a = tid; a < k; a += kBT) L.vh[a] = x[nH + a];
  __syncthreads();
  colsum_big(nH, k, Gt, theta, false, 0.0, x, nullptr, L, L.vb);   // Gt^T x_Theta
  if (tid < k) {
    double s = L.vb[tid];
    for (int b = 0; b < k; ++b) s = fma(Hm[(size_t)tid * k + b], L.vh[b], s);
    w[nH + tid] = s;
  }
  for (int r = tid; r < nH; r += kBT) w[r] = fma(theta[r], x[r], gt_row_dot(nH, k, GtT, r, L.vh));
  __syncthreads();
  double xw = 0.0;
  for (int r = tid; r < n; r += kBT) xw = fma(x[r], w[r], xw);
  const double rho = bsum(xw, L.red);
  double rr = 0.0;
  for (int r = tid; r < n; r += kBT) {
    const double e = w[r] - rho * x[r];
    rr = fma(e, e, rr);
  }
  rr = bsum(rr, L.red);
  if (tid == 0) {
    rq[i] = rho;
    res[i] = sqrt(rr);
  }
}

// Number of eigenvalues of Tt below mu by Sylvester's law of inertia: #{theta_j < mu} plus the
// negative pivots of an LDL^T of S(mu) without pivoting.  *trusted = false when a pivot is tiny
// or the factor grows (the count is then not certain).  Every thread gets the result.
// The count from S(mu) already in L.S (overwritten by its factor).
__device__ int inertia_count(int nH, int k, const double* __restrict__ theta, double mu, BLds& L, bool* trusted) {
  __shared__ int ok_s, neg_s;
  __shared__ double amax_s;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  if (tid == 0) {
    ok_s = 1;
    neg_s = 0;
  }
  if (wave == 0) {
    double m = 0.0;
    for (int r = 0; r < k; ++r) {
      if (lane <= r && lane < k) m = fmax(m, fabs(L.S[r][lane]));
      if (lane + 64 <= r && lane + 64 < k) m = fmax(m, fabs(L.S[r][lane + 64]));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if (lane == 0) amax_s = m;
  }
  __syncthreads();
  const double amax = amax_s;
  const int tx = tid & 31, ty = tid >> 5;
  for (int j = 0; j < k; ++j) {
    const double d = L.S[j][j];
    if (tid == 0) {
      if (!(fabs(d) > 1e-12 * amax)) ok_s = 0;
      if (d < 0.0) ++neg_s;
    }
    const double rd = 1.0 / d;
    for (int r = j + 1 + ty; r < k; r += 16) {
      const double lr = L.S[r][j] * rd;
      for (int t = j + 1 + tx; t <= r; t += 32) L.S[r][t] = fma(-lr, L.S[t][j], L.S[r][t]);
    }
    __syncthreads();
  }
  if (wave == 0) {
    double m = 0.0;
    for (int r = 0; r < k; ++r) {
      if (lane <= r && lane < k) m = fmax(m, fabs(L.S[r][lane]));
      if (lane + 64 <= r && lane + 64 < k) m = fmax(m, fabs(L.S[r][lane + 64]));
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if (lane == 0 && !(m <= 1e6 * amax)) ok_s = 0;
  }
  int cth = 0;
  for (int r = tid; r < nH; r += kBT) cth += (theta[r] < mu) ? 1 : 0;
  cth = (int)bsum((double)cth, L.red);
  const int count = cth + neg_s;
  *trusted = ok_s != 0;
  __syncthreads();
  return count;
}

// Acceptance: ascending order of the Rayleigh quotients, every residual within its tolerance,
// and the inertia count below mu* = (largest Rayleigh quotient) + gap equal to k.  A Rayleigh
// quotient theta_j can lie below its eigenvalue by up to its residual norm r_j, so when that count
// falls short, a count of k below max_j (theta_j + r_j) + gap, a shift above every eigenvalue the
// pairs approximate, certifies them too.  When both fail and the block carries guard pairs
// (nev < k), the count below the nev-th Rayleigh quotient + gap equal to nev still certifies the
// wanted pairs as the nev smallest (status[0] = 2: the guard pairs are then eigenpairs of Tt but not
// certified as the next ones).  status[0] = 0 rejects; status[1] = the last count.  lam ascending,
// perm = source column.
// Three launches: the order and residual checks with the three shifts (one workgroup), the sums
// over row chunks of Gt^T D(mu) Gt for each shift (one workgroup per chunk and shift, partial
// k x k blocks in part), and the Schur complements with their LDL^T counts (one workgroup).
__global__ __launch_bounds__(kBT) void saccept_pre_kernel(int k, int nev, const double* __restrict__ rq,
                                                        const double* __restrict__ res, double tol_abs,
                                                        const double* __restrict__ tolv, double gap,
                                                        double* __restrict__ lam, int* __restrict__ perm,
                                                        double* __restrict__ mus, int* __restrict__ status) {
  __shared__ double srt[kBK], sup[kBK];
  __shared__ int ok_s;
  const int tid = threadIdx.x;
  if (tid == 0) ok_s = 1;
  __syncthreads();
  if (tid < k) {
    const double v = rq[tid], e = res[tid];
    int rank = 0;
    for (int j = 0; j < k; ++j) {
      const double vj = rq[j];
      rank += (vj < v || (vj == v && j < tid)) ? 1 : 0;
    }
    const double tl = tolv ? tol_abs * tolv[(rank < k) ? rank : k - 1] : tol_abs;
    const bool good = (v == v && e == e && fabs(v) < DBL_MAX && e <= tl);
    srt[rank] = v;
    sup[rank] = v + e;
    perm[rank] = tid;
    if (!good) ok_s = 0;
  }
  __syncthreads();
  for (int j = tid; j < k; j += kBT) lam[j] = srt[j];
  if (tid == 0) {
    status[0] = ok_s;           // provisional: 1 = checks passed, the counts decide
    status[1] = 0;
    double up = srt[k - 1];
    for (int j = 0; j < k; ++j) up = fmax(up, sup[j]);
    mus[0] = srt[k - 1] + gap;
    mus[1] = up + gap;
    mus[2] = srt[(nev < k ? nev : k) - 1] + gap;
  }
}

__global__ __launch_bounds__(kBT) void saccept_part_kernel(int nH, int k, int nev, int rows,
                                                         const double* __restrict__ theta,
                                                         const double* __restrict__ Gt,
                                                         const double* __restrict__ mus,
                                                         const int* __restrict__ status, double* __restrict__ part) {
  const int sh = blockIdx.y;
  if (status[0] == 0 || (sh == 2 && nev >= k)) return;
  const int rb = blockIdx.x * rows;
  const int re = (rb + rows < nH) ? rb + rows : nH;
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int li = lane & 15, lk = lane >> 4;
  const int T = (k + 15) >> 4, TT = T * T;
  double4_t acc[8];
#pragma unroll
  for (int t = 0; t < 8; ++t) acc[t] = (double4_t){0.0, 0.0, 0.0, 0.0};
  if (rb < re) schur_rows_acc(rb, re, k, Gt, theta, mus[sh], acc);
  double* dst = part + ((size_t)sh * gridDim.x + blockIdx.x) * k * k;
#pragma unroll
  for (int t = 0; t < 8; ++t) {
    const int tt = wave + 8 * t;
    if (tt < TT) {
      const int ti = tt / T, tj = tt - (tt / T) * T;
      const int c = 16 * tj + li;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int r = 16 * ti + lk + 4 * q;
        if (r < k && c < k) dst[(size_t)r * k + c] = acc[t][q];
      }
    }
  }
}

__global__ __launch_bounds__(kBT) void saccept_final_kernel(int nH, int k, int nev, int nchunk,
                                                          const double* __restrict__ theta,
                                                          const double* __restrict__ Hm,
                                                          const double* __restrict__ mus,
                                                          const double* __restrict__ part,
                                                          int* __restrict__ status) {
  __shared__ BLds L;
  if (status[0] == 0) return;
  const int tid = threadIdx.x;
  int verdict = 0, count = 0;
  for (int sh = 0; sh < 3 && verdict == 0; ++sh) {
    if (sh == 2 && nev >= k) break;
    const double mu = mus[sh];
    const double* ps = part + (size_t)sh * nchunk * k * k;
    for (int e = tid; e < k * k; e += kBT) {
      const int r = e / k, c = e - (e / k) * k;
      double a = 0.0;
      for (int ch = 0; ch < nchunk; ++ch) a += ps[(size_t)ch * k * k + e];
      L.S[r][c] = Hm[(size_t)r * k + c] - ((r == c) ? mu : 0.0) - a;
    }
    __syncthreads();
    bool trusted = false;
    count = inertia_count(nH, k, theta, mu, L, &trusted);
    if (sh < 2) verdict = (trusted && count == k) ? 1 : 0;
    else verdict = (trusted && count == nev) ? 2 : 0;
    __syncthreads();
  }
  if (tid == 0) {
    status[0] = verdict;
    status[1] = count;
  }
}

// row chunks of the acceptance's Schur sums: at most 32, and at most what the scratch holds
int accept_chunk_rows(int nH, int k) {
  int nchunk = (nH + k) / k;
  if (nchunk > 32) nchunk = 32;
  if (nchunk < 1) nchunk = 1;
  int rows = (nH + nchunk - 1) / nchunk;
  rows = (rows + 3) & ~3;
  return rows;
}

}  // namespace

int small_big_max_k() { return kBK; }
int small_big_max_nh() { return kBigMaxH; }
// the per-pair work vectors (2 (nH + k) k) and 16 more, then G^T column-major (nH k)
size_t small_big_scratch_doubles(int nH, int k) { return (size_t)3 * (nH + k) * k + 16 + (size_t)nH * k; }
static double* gtt_slice(int nH, int k, double* scratch) { return scratch + (size_t)3 * (nH + k) * k + 16; }

void launch_small_rqi_big(int nH, int k, const double* theta, const double* Gt, const double* Hm,
                          const double* sigma, const double* X0, double scale, const double* tolv, double* Vt,
                          double* rq, double* scratch, hipStream_t s) {
  double* GtT = gtt_slice(nH, k, scratch);
  gt_transpose_kernel<<<(unsigned)(((long long)nH * k + 255) / 256), 256, 0, s>>>(nH, k, Gt, GtT);
  srqi_big_kernel<<<k, kBT, 0, s>>>(nH, k, theta, Gt, GtT, Hm, sigma, X0, scale, tolv, Vt, rq, scratch);
}

void launch_small_rr_big(int nH, int k, const double* theta, const double* Gt, const double* Hm, const double* Vt,
                         double* rq, double* res, double* scratch, hipStream_t s) {
  // G^T as the RQI launch left it (srr follows it in every sequence)
  srr_big_kernel<<<k, kBT, 0, s>>>(nH, k, theta, Gt, gtt_slice(nH, k, scratch), Hm, Vt, rq, res, scratch);
}

void launch_small_accept_big(int nH, int k, int nev, const double* theta, const double* Gt, const double* Hm,
                             const double* rq, const double* res, double tol_abs, const double* tolv, double gap,
                             double* lam, int* perm, int* status, double* scratch, hipStream_t s) {
  // scratch (the solver's per-pair work vectors, free again here): the partial sums, then the shifts
  const int rows = accept_chunk_rows(nH, k);
  const int nchunk = (nH + rows - 1) / rows;
  double* part = scratch;
  double* mus = scratch + (size_t)3 * nchunk * k * k;
  saccept_pre_kernel<<<1, kBT, 0, s>>>(k, nev, rq, res, tol_abs, tolv, gap, lam, perm, mus, status);
  saccept_part_kernel<<<dim3((unsigned)nchunk, 3), kBT, 0, s>>>(nH, k, nev, rows, theta, Gt, mus, status, part);
  saccept_final_kernel<<<1, kBT, 0, s>>>(nH, k, nev, nchunk, theta, Hm, mus, part, status);
}

}  // namespace pase
