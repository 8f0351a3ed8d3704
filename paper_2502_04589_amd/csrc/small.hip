// Structured solver of the augmented eigenproblem (Alg. 3 step 5).
//
// In the M-orthonormal basis [P L_B^{-T} Phi, W_perp L^{-T}] of the augmented
// space, where C0 = L_B^{-1} A_H L_B^{-T} = Phi Theta Phi^T is diagonalised once
// at setup, the augmented matrix is
//     Tt = [[Theta, Gt], [Gt^T, H]]   (Theta diagonal N_H x N_H, Gt N_H x k, H k x k).
// For a shift mu away from the diagonal of Theta, (Tt - mu I)^{-1} is applied
// exactly through the k x k Schur complement
//     S(mu) = H - mu I - Gt^T (Theta - mu I)^{-1} Gt,
// and Sylvester's law of inertia gives the number of eigenvalues of Tt below mu
// as #{theta_j < mu} + (number of negative eigenvalues of S(mu)).
//
// Fast path (one workgroup per wanted pair): shift-invert steps at the previous
// outer iteration's Ritz value, then Rayleigh-quotient steps; the block is
// orthonormalised, every pair's residual ||Tt v - rho v|| is formed with the
// explicit operator, and an inertia count just above the largest Ritz value
// certifies that no eigenvalue below it was missed.  A block that fails any test
// is not used: the runtime then solves the dense problem instead.
#include <cfloat>

#include "internal.hpp"

namespace pase {

namespace {

constexpr int kSK = 64;            // k <= kSK
constexpr int kRT = 512;           // threads per workgroup; thread j holds row j of Gt
constexpr int kRW = kRT / 64;
constexpr int kRMaxH = kRT;        // N_H <= kRMaxH
constexpr int kRound = 128;        // rows of Gt staged in LDS per round
constexpr int kGsLd = 68;
constexpr int kMaxFactor = 3;      // factorisations per pair
constexpr int kMaxSolve = 6;       // shift-invert solves per pair

typedef double double4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double wsum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Fixed-order block sum; every thread gets the result.
__device__ double bsum(double v, double* red) {
  v = wsum(v);
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int w = 0; w < kRW; ++w) s += red[w];
  return s;
}

__device__ __forceinline__ double hash_pm1(unsigned a, unsigned b) {
  unsigned h = a * 0x9E3779B1u ^ (b + 0x632BE5ABu) * 0x85EBCA77u;
  h ^= h >> 15;
  h *= 0x2C1B3C6Du;
  h ^= h >> 12;
  h *= 0x297A2D39u;
  h ^= h >> 15;
  return (double)(h & 0xFFFFFF) / (double)0x800000 - 1.0;   // [-1, 1)
}

struct RLds {
  double S[kSK][kSK + 1];              // Schur complement, then its U factor
  double M[kSK][kSK + 1];              // unit-lower LU factor (multipliers)
  double Gs[kRound][kGsLd];            // staged rows of Gt (also used between factorisation and solve)
  double ds[kRound];
  double xs[kRMaxH + kSK], ys[kRMaxH + kSK];
  double part[kRW][kSK];
  double red[kRW];
  int ipiv[kSK];
};

// Thread j < nH: g[a] = Gt[j][a] (a < k), zero elsewhere.  The loads are
// unconditional (row and column clamped into range, then masked), so they are
// all in flight together instead of one branch and wait per element.
__device__ __forceinline__ void load_row(int nH, int k, const double* __restrict__ Gt, double* g) {
  const int j = threadIdx.x;
  const bool rowok = j < nH;
  const double* __restrict__ rp = Gt + (size_t)(rowok ? j : nH - 1) * k;
#pragma unroll
  for (int a = 0; a < kSK; ++a) {
    const double v = rp[(a < k) ? a : k - 1];
    g[a] = (rowok && a < k) ? v : 0.0;
  }
}

// sum_a g[a] v[a] over kSK entries (v in LDS); scheduling fences keep at most 16
// LDS values live at a time next to the register-resident row.
__device__ __forceinline__ double rowdot(const double* g, const double* v) {
  double s0 = 0.0, s1 = 0.0;
#pragma unroll
  for (int c = 0; c < kSK; c += 16) {
#pragma unroll
    for (int a = c; a < c + 16; a += 2) {
      s0 = fma(g[a], v[a], s0);
      s1 = fma(g[a + 1], v[a + 1], s1);
    }
    __builtin_amdgcn_sched_barrier(0);
  }
  return s0 + s1;
}

// dst[a] = w g[a], in groups of 16 stores (fences keep the products from piling up).
__device__ __forceinline__ void stage_row(double* dst, const double* g, double w) {
#pragma unroll
  for (int c = 0; c < kSK; c += 16) {
#pragma unroll
    for (int a = c; a < c + 16; ++a) dst[a] = w * g[a];
    __builtin_amdgcn_sched_barrier(0);
  }
}

// S = H - mu I - sum_j d_j g_j g_j^T (d_j = dv of thread j), by v_mfma_f64_16x16x4f64 over
// rounds of kRound rows staged from registers.  MFMA operand layout: lane l supplies
// A[l%16][l/16], B[l/16][l%16]; accumulator register q holds D[l/16 + 4q][l%16].
__device__ void form_schur_r(int nH, int k, const double* g, double dv, const double* __restrict__ Hm, double mu,
                             RLds& L) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  const int T = (k + 15) >> 4, TT = T * T;
  const int li = lane & 15, lk = lane >> 4;
  double4_t acc[2];
  acc[0] = (double4_t){0.0, 0.0, 0.0, 0.0};
  acc[1] = acc[0];
  for (int r0 = 0; r0 < nH; r0 += kRound) {
    __syncthreads();
    if (tid >= r0 && tid < r0 + kRound) {
      const int rr = tid - r0;
      stage_row(L.Gs[rr], g, 1.0);
      L.ds[rr] = (tid < nH) ? dv : 0.0;
    }
    __syncthreads();
    const int nst = (nH - r0 >= kRound) ? kRound / 4 : (nH - r0 + 3) / 4;
    for (int st = 0; st < nst; ++st) {
      const int row = 4 * st + lk;
      const double dr = L.ds[row];
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        const int tt = wave + kRW * t;
        if (tt < TT) {
          const int ti = tt / T, tj = tt - (tt / T) * T;
          const double av = dr * L.Gs[row][16 * ti + li];
          const double bv = L.Gs[row][16 * tj + li];
          acc[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[t], 0, 0, 0);
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int t = 0; t < 2; ++t) {
    const int tt = wave + kRW * t;
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

// out[a] = sum_j w_j g_j[a] for a < k into L.part-reduced L.ys-free buffer `dst` (LDS, k values).
__device__ void colsum_r(int nH, int k, const double* g, double w, RLds& L, double* dst) {
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  double s = 0.0;
  for (int r0 = 0; r0 < nH; r0 += kRound) {
    __syncthreads();
    if (tid >= r0 && tid < r0 + kRound) {
      const int rr = tid - r0;
      double ww = (tid < nH) ? w : 0.0;
      // opaque per round: keeps the 64 products from being hoisted out of the
      // round loop as a second register-resident copy of the row
      __asm__ volatile("" : "+v"(ww));
      stage_row(L.Gs[rr], g, ww);
    }
    __syncthreads();
    // wave w sums rows w, w + 8, ... of this round for column a = lane
#pragma unroll 4
    for (int rr = wave; rr < kRound; rr += kRW) s += L.Gs[rr][lane];
  }
  L.part[wave][lane] = s;
  __syncthreads();
  if (tid < k) {
    double t = 0.0;
#pragma unroll
    for (int w = 0; w < kRW; ++w) t += L.part[w][tid];
    dst[tid] = t;
  }
  __syncthreads();
}

// In-place LU with partial pivoting of L.S (k x k): U in L.S (upper), unit-lower
// multipliers in L.M, ipiv[j] = row exchanged with j.  Two barriers per pivot;
// every wave finds the pivot itself (same data, same order, same result).
__device__ void lu_factor_r(int k, RLds& L) {
  const int tid = threadIdx.x, lane = tid & 63;
  const int tx = tid & 15, ty = tid >> 4;   // 16 x 32
  for (int j = 0; j < k; ++j) {
    // pivot search on one 64-bit key per lane: the bits of |S[lane][j]| (ordered like the
    // values, being non-negative) with the low 6 bits replaced by 63 - lane, so the maximum
    // key is the largest magnitude and, among magnitudes equal to 2^-46 relative, the lowest row
    unsigned long long key = 0ull;
    if (lane >= j && lane < k)
      key = ((unsigned long long)__double_as_longlong(fabs(L.S[lane][j])) & ~63ull) | (unsigned long long)(63 - lane);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
      const unsigned long long k2 = (unsigned long long)__shfl_xor((long long)key, o, 64);
      key = (k2 > key) ? k2 : key;
    }
    const int p = 63 - (int)(key & 63ull);
    if (tid == 0) L.ipiv[j] = p;
    if (p != j) {
      for (int t = tid; t < k; t += kRT) {
        const double a = L.S[j][t];
        L.S[j][t] = L.S[p][t];
        L.S[p][t] = a;
        if (t < j) {
          const double m = L.M[j][t];
          L.M[j][t] = L.M[p][t];
          L.M[p][t] = m;
        }
      }
    }
    __syncthreads();
    const double rp = 1.0 / L.S[j][j];
    for (int r = j + 1 + ty; r < k; r += 32) {
      const double lr = L.S[r][j] * rp;
      if (tx == 0) L.M[r][j] = lr;
      for (int t = j + 1 + tx; t < k; t += 16) L.S[r][t] = fma(-lr, L.S[j][t], L.S[r][t]);
    }
    __syncthreads();
  }
}

// Wave 0: solve S y = b with the LU factors; lane r holds b_r on entry, y_r on exit.
__device__ double lu_solve_wave(int k, const RLds& L, double b) {
  const int lane = threadIdx.x & 63;
  for (int j = 0; j < k; ++j) {
    const int p = L.ipiv[j];
    if (p != j) {
      const double bj = __shfl(b, j, 64), bp = __shfl(b, p, 64);
      if (lane == j) b = bp;
      if (lane == p) b = bj;
    }
  }
  for (int j = 0; j < k; ++j) {
    const double zj = __shfl(b, j, 64);
    if (lane > j && lane < k) b = fma(-L.M[lane][j], zj, b);
  }
  for (int j = k - 1; j >= 0; --j) {
    const double yj = __shfl(b, j, 64) / L.S[j][j];
    if (lane == j) b = yj;
    if (lane < j) b = fma(-L.S[lane][j], yj, b);
  }
  return (lane < k) ? b : 0.0;
}

// One workgroup per wanted pair i: shift-invert solves at sigma[i] with one
// factorisation, then Rayleigh-quotient shifts, until the step residual
// ||x_old - (rho - mu) y|| / ||y|| is below 1e-13 of the scale (with per-pair acceptance
// factors tolv, 1e-12 tolv[i] of it: a tenth of what the acceptance test asks) or the budget ends.
// Output: unit vector Vt[i*n .. i*n+n) (n = N_H + k) and its Rayleigh quotient.
__global__ __launch_bounds__(kRT) void srqi_kernel(int nH, int k, const double* __restrict__ theta,
                                                 const double* __restrict__ Gt, const double* __restrict__ Hm,
                                                 const double* __restrict__ sigma, const double* __restrict__ X0,
                                                 double scale, const double* __restrict__ tolv,
                                                 double* __restrict__ Vt, double* __restrict__ rq) {
  __shared__ RLds L;
  const int i = blockIdx.x;
  const int n = nH + k;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  double g[kSK];
  load_row(nH, k, Gt, g);
  const double th = (tid < nH) ? theta[tid] : 0.0;
  double nx = 0.0;
  for (int r = tid; r < n; r += kRT) {
    const double v = X0 ? X0[(size_t)r * k + i] : hash_pm1((unsigned)i + 1u, (unsigned)r);
    L.xs[r] = v;
    nx = fma(v, v, nx);
  }
  nx = bsum(nx, L.red);
  const double inx = 1.0 / sqrt(nx);
  for (int r = tid; r < n; r += kRT) L.xs[r] *= inx;
  double mu = sigma[i];
  if (X0) {
    // first shift: Rayleigh quotient of the start vector, x^T Tt x
    __syncthreads();
    const double xj0 = (tid < nH) ? L.xs[tid] : 0.0;
    double part = 0.0;
    if (tid < nH) part = xj0 * fma(th, xj0, 2.0 * rowdot(g, L.xs + nH));
    if (tid < k) {
      double hx = 0.0;
      for (int b = 0; b < k; ++b) hx = fma(Hm[(size_t)tid * k + b], L.xs[nH + b], hx);
      part = fma(L.xs[nH + tid], hx, part);
    }
    mu = bsum(part, L.red);
  }
  double rho = mu;
  const double stop = (tolv ? fmax(1e-13, 1e-12 * tolv[i]) : 1e-13) * scale;
  double dv = (tid < nH) ? 1.0 / (th - mu) : 0.0;
  form_schur_r(nH, k, g, dv, Hm, mu, L);
  lu_factor_r(k, L);
  int nfac = 1, since = 0;
  const int hold = X0 ? 3 : 2;               // solves per factorisation before a new shift
  for (int it = 0; it < kMaxSolve; ++it) {
    if (since >= hold && nfac < kMaxFactor) {   // Rayleigh-quotient shift
      mu = rho;
      dv = (tid < nH) ? 1.0 / (th - mu) : 0.0;
      form_schur_r(nH, k, g, dv, Hm, mu, L);
      lu_factor_r(k, L);
      ++nfac;
      since = 0;
    }
    // rhs = x_H - Gt^T (d o x_Theta)
    __syncthreads();
    const double xj = (tid < nH) ? L.xs[tid] : 0.0;
    colsum_r(nH, k, g, dv * xj, L, L.ys + nH);
    if (wave == 0) {
      const double b = (lane < k) ? L.xs[nH + lane] - L.ys[nH + lane] : 0.0;
      const double yh = lu_solve_wave(k, L, b);
      if (lane < k) L.ys[nH + lane] = yh;
    }
    __syncthreads();
    // y_Theta = d o (x_Theta - Gt y_H)
    if (tid < nH) L.ys[tid] = dv * (xj - rowdot(g, L.ys + nH));
    __syncthreads();
    double yy = 0.0, yx = 0.0;
    for (int r = tid; r < n; r += kRT) {
      yy = fma(L.ys[r], L.ys[r], yy);
      yx = fma(L.ys[r], L.xs[r], yx);
    }
    yy = bsum(yy, L.red);
    yx = bsum(yx, L.red);
    const double ny = sqrt(yy);
    rho = mu + yx / yy;                       // T y = x + mu y
    const double dm = rho - mu;
    double rr = 0.0;
    for (int r = tid; r < n; r += kRT) {
      const double e = (L.xs[r] - dm * L.ys[r]) / ny;
      rr = fma(e, e, rr);
      L.xs[r] = L.ys[r] / ny;
    }
    rr = bsum(rr, L.red);
    ++since;
    if (!(rr == rr) || !(ny == ny)) break;   // NaN: left to the acceptance test
    if (it >= 1 && sqrt(rr) <= stop) break;
  }
  __syncthreads();
  for (int r = tid; r < n; r += kRT) Vt[(size_t)i * n + r] = L.xs[r];
  if (tid == 0) rq[i] = rho;
}

// Rayleigh quotient and residual of column i of an orthonormal Vt with the
// explicit operator: w = Tt v, rho = v.w, res = ||w - rho v||.
__global__ __launch_bounds__(kRT) void srr_kernel(int nH, int k, const double* __restrict__ theta,
                                                const double* __restrict__ Gt, const double* __restrict__ Hm,
                                                const double* __restrict__ Vt, double* __restrict__ rq,
                                                double* __restrict__ res) {
  __shared__ RLds L;
  const int i = blockIdx.x;
  const int n = nH + k;
  const int tid = threadIdx.x;
  double g[kSK];
  load_row(nH, k, Gt, g);
  for (int r = tid; r < n; r += kRT) L.xs[r] = Vt[(size_t)i * n + r];
  __syncthreads();
  const double xj = (tid < nH) ? L.xs[tid] : 0.0;
  colsum_r(nH, k, g, xj, L, L.ys + nH);        // Gt^T x_Theta
  if (tid < k) {
    double s = L.ys[nH + tid];
    for (int b = 0; b < k; ++b) s = fma(Hm[(size_t)tid * k + b], L.xs[nH + b], s);
    L.ys[nH + tid] = s;
  }
  if (tid < nH) L.ys[tid] = fma(theta[tid], xj, rowdot(g, L.xs + nH));
  __syncthreads();
  double xw = 0.0;
  for (int r = tid; r < n; r += kRT) xw = fma(L.xs[r], L.ys[r], xw);
  const double rho = bsum(xw, L.red);
  double rr = 0.0;
  for (int r = tid; r < n; r += kRT) {
    const double e = L.ys[r] - rho * L.xs[r];
    rr = fma(e, e, rr);
  }
  rr = bsum(rr, L.red);
  if (tid == 0) {
    rq[i] = rho;
    res[i] = sqrt(rr);
  }
}

// Eigenvalues of Tt below mu by Sylvester's law of inertia: #{theta_j < mu} plus the negative
// pivots of an LDL^T of S(mu) without pivoting.  *trusted = false when a pivot is tiny or the
// factor grows (the count is then not certain).  Every thread gets the result.
__device__ int inertia_r(int nH, int k, const double* g, double th, const double* __restrict__ Hm, double mu,
                         RLds& L, bool* trusted) {
  __shared__ int ok_s, neg_s, cth_s;
  __shared__ double amax_s;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  if (tid == 0) {
    ok_s = 1;
    neg_s = 0;
    cth_s = 0;
  }
  const double dv = (tid < nH) ? 1.0 / (th - mu) : 0.0;
  form_schur_r(nH, k, g, dv, Hm, mu, L);
  if (wave == 0) {
    double m = 0.0;
    for (int r = 0; r < k; ++r)
      if (lane <= r && lane < k) m = fmax(m, fabs(L.S[r][lane]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if (lane == 0) amax_s = m;
  }
  __syncthreads();
  const double amax = amax_s;
  const int tx = tid & 15, ty = tid >> 4;
  for (int j = 0; j < k; ++j) {
    const double d = L.S[j][j];
    if (tid == 0) {
      if (!(fabs(d) > 1e-12 * amax)) ok_s = 0;
      if (d < 0.0) ++neg_s;
    }
    const double rd = 1.0 / d;
    for (int r = j + 1 + ty; r < k; r += 32) {
      const double lr = L.S[r][j] * rd;
      for (int t = j + 1 + tx; t <= r; t += 16) L.S[r][t] = fma(-lr, L.S[t][j], L.S[r][t]);
    }
    __syncthreads();
  }
  if (wave == 0) {
    double m = 0.0;
    for (int r = 0; r < k; ++r)
      if (lane <= r && lane < k) m = fmax(m, fabs(L.S[r][lane]));
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if (lane == 0 && !(m <= 1e6 * amax)) ok_s = 0;
  }
  const int cth = (tid < nH && th < mu) ? 1 : 0;
  const unsigned long long bl = __ballot(cth != 0);
  if (lane == 0) atomicAdd(&cth_s, __popcll(bl));
  __syncthreads();
  const int count = cth_s + neg_s;
  *trusted = ok_s != 0;
  __syncthreads();
  return count;
}

// Acceptance of the fast path (one workgroup).  Sorts the Rayleigh quotients,
// requires every residual <= tol_abs and finite values, then counts the
// eigenvalues of Tt below mu* = lambda_max + gap by inertia; the count must be k.  A Rayleigh
// quotient theta_j can lie below its eigenvalue by up to its residual norm r_j, so when that count
// falls short, a count of k below max_j (theta_j + r_j) + gap (above every eigenvalue the pairs
// approximate) certifies them too.
// When both fail and the block carries guard pairs (nev < k), a count of nev below the
// nev-th Rayleigh quotient + gap still certifies the wanted pairs as the nev smallest
// (status[0] = 2: the guard pairs are eigenpairs of Tt, not certified as the next ones).
// Writes lam (ascending) and perm (column of Vt for each output position);
// status[0] = 0 rejects; status[1] = the last count (0 if not reached).
__global__ __launch_bounds__(kRT) void saccept_kernel(int nH, int k, int nev, const double* __restrict__ theta,
                                                    const double* __restrict__ Gt, const double* __restrict__ Hm,
                                                    const double* __restrict__ rq, const double* __restrict__ res,
                                                    double tol_abs, const double* __restrict__ tolv, double gap,
                                                    double* __restrict__ lam, int* __restrict__ perm,
                                                    int* __restrict__ status) {
  __shared__ RLds L;
  __shared__ double srt[kSK];
  __shared__ double up_s;
  __shared__ int ok_s;
  const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
  if (tid == 0) ok_s = 1;
  __syncthreads();
  if (wave == 0) {
    const double v = (lane < k) ? rq[lane] : DBL_MAX;
    const double e = (lane < k) ? res[lane] : 0.0;
    int rank = 0;
    for (int j = 0; j < k; ++j) {
      const double vj = __shfl(v, j, 64);
      rank += (vj < v || (vj == v && j < lane)) ? 1 : 0;
    }
    // tolerance of the pair at this position of the ascending order (per position, or one for all)
    const double tl = (tolv && lane < k) ? tol_abs * tolv[(rank < k) ? rank : k - 1] : tol_abs;
    const bool good = (lane >= k) || (v == v && e == e && fabs(v) < DBL_MAX && e <= tl);
    if (lane < k) {
      srt[rank] = v;
      perm[rank] = lane;
    }
    const unsigned long long bad = __ballot(!good);
    if (lane == 0 && bad) ok_s = 0;
    double up = (lane < k) ? v + e : -DBL_MAX;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) up = fmax(up, __shfl_xor(up, o, 64));
    if (lane == 0) up_s = up;
  }
  __syncthreads();
  for (int j = tid; j < k; j += kRT) lam[j] = srt[j];
  if (!ok_s) {
    if (tid == 0) {
      status[0] = 0;
      status[1] = 0;
    }
    return;
  }
  double g[kSK];
  load_row(nH, k, Gt, g);
  const double th = (tid < nH) ? theta[tid] : 0.0;
  bool trusted = false;
  int count = inertia_r(nH, k, g, th, Hm, srt[k - 1] + gap, L, &trusted);
  int verdict = (trusted && count == k) ? 1 : 0;
  if (!verdict) {
    count = inertia_r(nH, k, g, th, Hm, fmax(up_s, srt[k - 1]) + gap, L, &trusted);
    verdict = (trusted && count == k) ? 1 : 0;
  }
  if (!verdict && nev < k) {
    count = inertia_r(nH, k, g, th, Hm, srt[nev - 1] + gap, L, &trusted);
    verdict = (trusted && count == nev) ? 2 : 0;
  }
  if (tid == 0) {
    status[0] = verdict;
    status[1] = count;
  }
}

// Tr ((m + k) x (m + k)) = the principal block of Tt on its first m coarse modes and the k
// W-directions: [[diag(theta[0:m]), Gt[0:m, :]], [Gt[0:m, :]^T, H]].
__global__ void principal_kernel(int m, int k, const double* __restrict__ theta, const double* __restrict__ Gt,
                                 const double* __restrict__ Hm, double* __restrict__ Tr) {
  const int n = m + k;
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n * n) return;
  const int i = q / n, j = q - (q / n) * n;
  double v;
  if (i < m && j < m) v = (i == j) ? theta[i] : 0.0;
  else if (i < m) v = Gt[(size_t)i * k + (j - m)];
  else if (j < m) v = Gt[(size_t)j * k + (i - m)];
  else v = Hm[(size_t)(i - m) * k + (j - m)];
  Tr[q] = v;
}

// X0 ((nH + k) x k) from the principal block's eigenvectors Vr ((m + k) x k): coarse rows 0..m-1,
// zeros for the coarse modes m..nH-1, then the k W-direction rows.
__global__ void expand_kernel(int nH, int m, int k, const double* __restrict__ Vr, double* __restrict__ X0) {
  const long long q = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (long long)(nH + k) * k) return;
  const int r = (int)(q / k), c = (int)(q - (q / k) * k);
  double v = 0.0;
  if (r < m) v = Vr[(size_t)r * k + c];
  else if (r >= nH) v = Vr[(size_t)(r - nH + m) * k + c];
  X0[q] = v;
}

// V (n x k row-major) from the orthonormal vector-major Vt, columns in the
// accepted order.
__global__ void semit_kernel(int n, int k, const double* __restrict__ Vt, const int* __restrict__ perm,
                             double* __restrict__ V) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n * k) return;
  const int r = q / k, c = q - (q / k) * k;
  V[q] = Vt[(size_t)perm[c] * n + r];
}

}  // namespace

int small_fast_max_k() { return kSK; }
int small_fast_max_nh() { return kRMaxH; }

void launch_small_rqi(int nH, int k, const double* theta, const double* Gt, const double* Hm, const double* sigma,
                      const double* X0, double scale, const double* tolv, double* Vt, double* rq, hipStream_t s) {
  srqi_kernel<<<k, kRT, 0, s>>>(nH, k, theta, Gt, Hm, sigma, X0, scale, tolv, Vt, rq);
}

void launch_small_rr(int nH, int k, const double* theta, const double* Gt, const double* Hm, const double* Vt,
                     double* rq, double* res, hipStream_t s) {
  srr_kernel<<<k, kRT, 0, s>>>(nH, k, theta, Gt, Hm, Vt, rq, res);
}

void launch_small_accept(int nH, int k, int nev, const double* theta, const double* Gt, const double* Hm,
                         const double* rq, const double* res, double tol_abs, const double* tolv, double gap,
                         double* lam, int* perm, int* status, hipStream_t s) {
  saccept_kernel<<<1, kRT, 0, s>>>(nH, k, nev, theta, Gt, Hm, rq, res, tol_abs, tolv, gap, lam, perm, status);
}

void launch_small_principal(int nH, int m, int k, const double* theta, const double* Gt, const double* Hm,
                            double* Tr, hipStream_t s) {
  (void)nH;
  const int n = m + k;
  principal_kernel<<<(unsigned)((n * n + kBlock - 1) / kBlock), kBlock, 0, s>>>(m, k, theta, Gt, Hm, Tr);
}

void launch_small_expand(int nH, int m, int k, const double* Vr, double* X0, hipStream_t s) {
  const long long tot = (long long)(nH + k) * k;
  expand_kernel<<<(unsigned)((tot + kBlock - 1) / kBlock), kBlock, 0, s>>>(nH, m, k, Vr, X0);
}

void launch_small_emit(int n, int k, const double* Vt, const int* perm, double* V, hipStream_t s) {
  semit_kernel<<<(unsigned)((n * k + kBlock - 1) / kBlock), kBlock, 0, s>>>(n, k, Vt, perm, V);
}

}  // namespace pase
