// Algebraic input: level operators and transfers as CSR matrices (Alg. 3's "Require" takes A_H,
// B_H, A_h, B_h, I_H^h and I_h^H as matrices), applied to node-major multi-vectors.
//
// One wavefront per row: the row's nonzeros are walked with wave-uniform (scalar) loads of the
// column index and value, and each lane accumulates columns lane, lane + 64, ... of the k
// contiguous values of the referenced rows (coalesced 512-byte segments).  A block of 4 waves
// owns a contiguous run of rows; the eigen-residual's column sums are reduced per block in LDS
// and written as partials[block][3][k] for the fixed-order reduction.
//
// The export kernels write the grid hierarchy of a handle as CSR with a fixed number of slots per
// row (unused slots hold an explicit zero), so that row pointers are slots * i.
#include "internal.hpp"

namespace pase {
namespace {

constexpr int kCsrWaves = 4;
constexpr int kCsrQ = 4;             // columns per lane: k <= 256

// Column of slot q of a lane: lane + 64 q, or with PAIR (k even) the pairs 2 lane + 128 (q / 2)
// + (q % 2), so that a lane's two adjacent columns are one vector load
template <bool PAIR>
__device__ __forceinline__ int col_of(int lane, int q) {
  return PAIR ? 2 * lane + 128 * (q >> 1) + (q & 1) : lane + 64 * q;
}

template <typename T> struct Pair2;
template <> struct Pair2<double> { typedef double2 type; };
template <> struct Pair2<float> { typedef float2 type; };

// x values of the lane's columns in row c of X
template <typename T, bool PAIR>
__device__ __forceinline__ void load_row(const T* __restrict__ X, long long c, int lane, int k, double (&xv)[kCsrQ]) {
  if constexpr (PAIR) {
    typedef typename Pair2<T>::type V2;
#pragma unroll
    for (int h = 0; h < kCsrQ / 2; ++h) {
      const int col = 2 * lane + 128 * h;
      if (col < k) {
        const V2 v = *(const V2*)(X + c * k + col);
        xv[2 * h] = (double)v.x;
        xv[2 * h + 1] = (double)v.y;
      } else {
        xv[2 * h] = xv[2 * h + 1] = 0.0;
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < kCsrQ; ++q) {
      const int col = lane + 64 * q;
      xv[q] = (col < k) ? (double)X[c * k + col] : 0.0;
    }
  }
}

// acc[q] += sum over row r of A: val * X[col, col_of(lane, q)]; four nonzeros at a time so that
// their row loads are in flight together
template <typename T, bool PAIR>
__device__ __forceinline__ void csr_row(const CsrMat& A, long long r, int lane, int k, const T* __restrict__ X,
                                        double (&acc)[kCsrQ]) {
  const int p0 = A.rowptr[r], p1 = A.rowptr[r + 1];
  int p = p0;
  for (; p + 4 <= p1; p += 4) {
    long long c[4];
    double v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      c[u] = A.colind[p + u];
      v[u] = A.val[p + u];
    }
    double xv[4][kCsrQ];
#pragma unroll
    for (int u = 0; u < 4; ++u) load_row<T, PAIR>(X, c[u], lane, k, xv[u]);
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int q = 0; q < kCsrQ; ++q) acc[q] = fma(v[u], xv[u][q], acc[q]);
  }
  for (; p < p1; ++p) {
    double xv[kCsrQ];
    load_row<T, PAIR>(X, A.colind[p], lane, k, xv);
    const double v = A.val[p];
#pragma unroll
    for (int q = 0; q < kCsrQ; ++q) acc[q] = fma(v, xv[q], acc[q]);
  }
}

template <typename T, int EPI, bool PAIR>
__global__ __launch_bounds__(64 * kCsrWaves) void csr_op_kernel(CsrOpArgs a, long long rpb) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const long long r0 = (long long)blockIdx.x * rpb;
  const long long r1 = (r0 + rpb < a.rows) ? r0 + rpb : a.rows;
  const int k = a.k;
  const T* __restrict__ X = (const T*)a.x;
  const T* __restrict__ B = (const T*)a.b;
  T* __restrict__ O1 = (T*)a.out1;
  T* __restrict__ O2 = (T*)a.out2;
  const bool needA = (EPI != EPI_AM) || O1;
  const bool needM = (EPI == EPI_EIGRES) || (EPI == EPI_AM && O2);
  double s0[kCsrQ], s1[kCsrQ], s2[kCsrQ];
#pragma unroll
  for (int q = 0; q < kCsrQ; ++q) s0[q] = s1[q] = s2[q] = 0.0;
  for (long long r = r0 + wave; r < r1; r += kCsrWaves) {
    double ax[kCsrQ], mx[kCsrQ], xc[kCsrQ];
#pragma unroll
    for (int q = 0; q < kCsrQ; ++q) ax[q] = mx[q] = xc[q] = 0.0;
    if (needA) csr_row<T, PAIR>(a.A, r, lane, k, X, ax);
    if (needM) csr_row<T, PAIR>(a.M, r, lane, k, X, mx);
    const double wd = (EPI == EPI_SWEEP) ? a.omega * a.dinv[r] : 0.0;
#pragma unroll
    for (int q = 0; q < kCsrQ; ++q) {
      const int col = col_of<PAIR>(lane, q);
      if (col >= k) continue;
      const long long e = r * k + col;
      if (EPI == EPI_SWEEP || EPI == EPI_EIGRES) xc[q] = (double)X[e];
      if (EPI == EPI_AM) {
        if (O1) O1[e] = (T)ax[q];
        if (O2) O2[e] = (T)mx[q];
      } else if (EPI == EPI_RESID) {
        O1[e] = (T)((double)B[e] - ax[q]);
      } else if (EPI == EPI_SWEEP) {
        O1[e] = (T)(xc[q] + wd * ((double)B[e] - ax[q]));
      } else {   // EPI_EIGRES
        const double res = a.lam[col] * mx[q] - ax[q];
        O1[e] = (T)res;
        s0[q] = fma(res, res, s0[q]);
        s1[q] = fma(mx[q], mx[q], s1[q]);
        s2[q] = fma(xc[q], mx[q], s2[q]);
      }
    }
  }
  if (EPI == EPI_EIGRES) {
    __shared__ double red[3][kCsrWaves][64 * kCsrQ];
#pragma unroll
    for (int q = 0; q < kCsrQ; ++q) {
      const int col = col_of<PAIR>(lane, q);   // a permutation of 0 .. 255
      red[0][wave][col] = s0[q];
      red[1][wave][col] = s1[q];
      red[2][wave][col] = s2[q];
    }
    __syncthreads();
    double* p = a.partial + (size_t)blockIdx.x * 3 * k;
    for (int c = threadIdx.x; c < k; c += 64 * kCsrWaves) {
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        double sum = 0.0;
        for (int w = 0; w < kCsrWaves; ++w) sum += red[t][w][c];
        p[t * k + c] = sum;
      }
    }
  }
}

// y (=, +=, -=) A x (mode 0, 1, 2) for a rows x cols CSR A and multi-vectors of k columns
template <typename T, bool PAIR>
__global__ __launch_bounds__(64 * kCsrWaves) void csr_apply_kernel(CsrMat A, long long rows, int k, const T* __restrict__ x,
                                                                  T* __restrict__ y, int mode, long long rpb) {
  const int lane = threadIdx.x & 63;
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const long long r0 = (long long)blockIdx.x * rpb;
  const long long r1 = (r0 + rpb < rows) ? r0 + rpb : rows;
  for (long long r = r0 + wave; r < r1; r += kCsrWaves) {
    double acc[kCsrQ];
#pragma unroll
    for (int q = 0; q < kCsrQ; ++q) acc[q] = 0.0;
    csr_row<T, PAIR>(A, r, lane, k, x, acc);
#pragma unroll
    for (int q = 0; q < kCsrQ; ++q) {
      const int col = col_of<PAIR>(lane, q);
      if (col >= k) continue;
      const long long e = r * k + col;
      if (mode == 0) y[e] = (T)acc[q];
      else if (mode == 1) y[e] = (T)((double)y[e] + acc[q]);
      else y[e] = (T)((double)y[e] - acc[q]);
    }
  }
}

// dinv[i] = 1 / A_ii (0 when row i holds no diagonal entry; setup rejects that)
__global__ void csr_diag_inv_kernel(CsrMat A, long long rows, double* __restrict__ dinv) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  double d = 0.0;
  for (int p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p)
    if (A.colind[p] == i) d += A.val[p];
  dinv[i] = (d != 0.0) ? 1.0 / d : 0.0;
}

// D (rows x rows, dense row-major) = A; one thread per row (the coarsest level only)
__global__ void csr_to_dense_kernel(CsrMat A, long long rows, double* __restrict__ D) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= rows) return;
  for (long long j = 0; j < rows; ++j) D[i * rows + j] = 0.0;
  for (int p = A.rowptr[i]; p < A.rowptr[i + 1]; ++p) D[i * rows + A.colind[p]] += A.val[p];
}

// ---- export of a grid hierarchy (dim 2 or 3), fixed slots per row
template <int DIM>
__device__ __forceinline__ void xyz_of(long long i, int m, int& x, int& y, int& z) {
  x = (int)(i % m);
  y = (int)((i / m) % m);
  z = (DIM == 3) ? (int)(i / ((long long)m * m)) : 0;
}

// rows of a level operator from its 3^DIM stencil coefficients (coef: N x 3^DIM, or a constant
// pattern when coef is null: the Q1 mass of mesh width h)
template <int DIM>
__global__ void export_stencil_kernel(int m, const double* __restrict__ coef, double hmass, int* __restrict__ rowptr,
                                      int* __restrict__ colind, double* __restrict__ val) {
  constexpr int NS = (DIM == 3) ? 27 : 9;
  long long N = (long long)m * m;
  if (DIM == 3) N *= m;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > N) return;
  if (rowptr) rowptr[i] = (int)(i * NS);
  if (i == N) return;
  int x, y, z;
  xyz_of<DIM>(i, m, x, y, z);
  for (int o = 0; o < NS; ++o) {
    const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = (DIM == 3) ? o / 9 - 1 : 0;
    bool ok = x + ox >= 0 && x + ox < m && y + oy >= 0 && y + oy < m;
    if (DIM == 3) ok = ok && z + oz >= 0 && z + oz < m;
    const long long j = i + ox + (long long)oy * m + ((DIM == 3) ? (long long)oz * m * m : 0);
    double v = 0.0;
    if (ok) {
      if (coef) {
        v = coef[i * NS + o];
      } else {
        const double c = hmass / 6.0;
        v = ((ox == 0) ? 4.0 : 1.0) * c * ((oy == 0) ? 4.0 : 1.0) * c;
        if (DIM == 3) v *= ((oz == 0) ? 4.0 : 1.0) * c;
      }
    }
    colind[i * NS + o] = ok ? (int)j : (int)i;
    val[i * NS + o] = v;
  }
}

// 1D weights of trilinear interpolation: fine index f (full-grid coordinate f + 1) and its coarse
// parents; slot s in {0, 1}: parent coordinate floor((f + 1) / 2) - 1 + s ... with weight 1 when
// the fine node sits on a coarse node (one parent), 1/2 each when it lies between two
__device__ __forceinline__ void parents1d(int f, int mc, int s, int& c, double& w) {
  const int F = f + 1;
  if ((F & 1) == 0) {
    c = F / 2 - 1;
    w = (s == 0) ? 1.0 : 0.0;
  } else {
    c = (F - 1) / 2 - 1 + s;
    w = 0.5;
  }
  if (c < 0 || c >= mc) w = 0.0;
}

// P (Nf x Nc, 2^DIM slots per row): the trilinear interpolation from mesh mc to mf = 2 mc + 1
template <int DIM>
__global__ void export_prolong_kernel(int mf, int mc, int* __restrict__ rowptr, int* __restrict__ colind,
                                      double* __restrict__ val) {
  constexpr int NSL = 1 << DIM;
  long long N = (long long)mf * mf;
  if (DIM == 3) N *= mf;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > N) return;
  if (rowptr) rowptr[i] = (int)(i * NSL);
  if (i == N) return;
  int x, y, z;
  xyz_of<DIM>(i, mf, x, y, z);
  for (int sl = 0; sl < NSL; ++sl) {
    int cx, cy, cz = 0;
    double wx, wy, wz = 1.0;
    parents1d(x, mc, sl & 1, cx, wx);
    parents1d(y, mc, (sl >> 1) & 1, cy, wy);
    if (DIM == 3) parents1d(z, mc, (sl >> 2) & 1, cz, wz);
    const double w = wx * wy * wz;
    const long long j = cx + (long long)cy * mc + ((DIM == 3) ? (long long)cz * mc * mc : 0);
    colind[i * NSL + sl] = (w != 0.0) ? (int)j : 0;
    val[i * NSL + sl] = w;
  }
}

// R = P^T (Nc x Nf, 3^DIM slots per row): coarse node c's fine neighbours 2(c+1) - 1 + d - 1,
// d in {0, 1, 2}, with weights 1/2, 1, 1/2 per axis
template <int DIM>
__global__ void export_restrict_kernel(int mf, int mc, int* __restrict__ rowptr, int* __restrict__ colind,
                                       double* __restrict__ val) {
  constexpr int NS = (DIM == 3) ? 27 : 9;
  long long N = (long long)mc * mc;
  if (DIM == 3) N *= mc;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i > N) return;
  if (rowptr) rowptr[i] = (int)(i * NS);
  if (i == N) return;
  int x, y, z;
  xyz_of<DIM>(i, mc, x, y, z);
  const double w1[3] = {0.5, 1.0, 0.5};
  for (int o = 0; o < NS; ++o) {
    const int dx = o % 3, dy = (o / 3) % 3, dz = (DIM == 3) ? o / 9 : 1;
    const int fx = 2 * (x + 1) - 1 + dx - 1, fy = 2 * (y + 1) - 1 + dy - 1, fz = 2 * (z + 1) - 1 + dz - 1;
    const bool ok = fx >= 0 && fx < mf && fy >= 0 && fy < mf && (DIM == 2 || (fz >= 0 && fz < mf));
    const long long j = fx + (long long)fy * mf + ((DIM == 3) ? (long long)fz * mf * mf : 0);
    colind[i * NS + o] = ok ? (int)j : 0;
    val[i * NS + o] = ok ? w1[dx] * w1[dy] * ((DIM == 3) ? w1[dz] : 1.0) : 0.0;
  }
}

inline unsigned blocks_of(long long n, int b) { return (unsigned)((n + b - 1) / b); }

long long csr_rows_per_block(long long rows) {
  // about 8192 blocks (32 per CU), at least one row per wave
  long long rpb = (rows + 8191) / 8192;
  if (rpb < kCsrWaves) rpb = kCsrWaves;
  return rpb;
}

}  // namespace

int csr_tiles(long long rows) { return (int)((rows + csr_rows_per_block(rows) - 1) / csr_rows_per_block(rows)); }

void launch_csr_op(const CsrOpArgs& a, Epi epi, hipStream_t s) {
  const long long rpb = csr_rows_per_block(a.rows);
  const unsigned nb = (unsigned)((a.rows + rpb - 1) / rpb);
  const dim3 blk(64 * kCsrWaves);
  const bool pair = (a.k % 2) == 0;
#define PASE_CSR(E)                                                                                  \
  if (a.fp32) {                                                                                      \
    if (pair) csr_op_kernel<float, E, true><<<nb, blk, 0, s>>>(a, rpb);                              \
    else csr_op_kernel<float, E, false><<<nb, blk, 0, s>>>(a, rpb);                                  \
  } else {                                                                                           \
    if (pair) csr_op_kernel<double, E, true><<<nb, blk, 0, s>>>(a, rpb);                             \
    else csr_op_kernel<double, E, false><<<nb, blk, 0, s>>>(a, rpb);                                 \
  }
  switch (epi) {
    case EPI_AM: PASE_CSR(EPI_AM) break;
    case EPI_RESID: PASE_CSR(EPI_RESID) break;
    case EPI_SWEEP: PASE_CSR(EPI_SWEEP) break;
    case EPI_EIGRES: PASE_CSR(EPI_EIGRES) break;
    default: set_last_error("launch_csr_op: epilogue not available on CSR operators"); break;
  }
#undef PASE_CSR
}

void launch_csr_apply(const CsrMat& A, long long rows, int k, const void* x, void* y, int mode, int fp32,
                      hipStream_t s) {
  const long long rpb = csr_rows_per_block(rows);
  const unsigned nb = (unsigned)((rows + rpb - 1) / rpb);
  const bool pair = (k % 2) == 0;
  if (fp32) {
    if (pair) csr_apply_kernel<float, true><<<nb, 64 * kCsrWaves, 0, s>>>(A, rows, k, (const float*)x, (float*)y, mode, rpb);
    else csr_apply_kernel<float, false><<<nb, 64 * kCsrWaves, 0, s>>>(A, rows, k, (const float*)x, (float*)y, mode, rpb);
  } else {
    if (pair)
      csr_apply_kernel<double, true><<<nb, 64 * kCsrWaves, 0, s>>>(A, rows, k, (const double*)x, (double*)y, mode, rpb);
    else
      csr_apply_kernel<double, false><<<nb, 64 * kCsrWaves, 0, s>>>(A, rows, k, (const double*)x, (double*)y, mode, rpb);
  }
}

void launch_csr_diag_inv(const CsrMat& A, long long rows, double* dinv, hipStream_t s) {
  csr_diag_inv_kernel<<<blocks_of(rows, 256), 256, 0, s>>>(A, rows, dinv);
}

void launch_csr_to_dense(const CsrMat& A, long long rows, double* D, hipStream_t s) {
  csr_to_dense_kernel<<<blocks_of(rows, 256), 256, 0, s>>>(A, rows, D);
}

void launch_export_stencil(int dim, int m, const double* coef, double hmass, int* rowptr, int* colind, double* val,
                           hipStream_t s) {
  const long long N = (long long)m * m * (dim == 3 ? m : 1);
  if (dim == 3) export_stencil_kernel<3><<<blocks_of(N + 1, 256), 256, 0, s>>>(m, coef, hmass, rowptr, colind, val);
  else export_stencil_kernel<2><<<blocks_of(N + 1, 256), 256, 0, s>>>(m, coef, hmass, rowptr, colind, val);
}

void launch_export_prolong(int dim, int mf, int mc, int* rowptr, int* colind, double* val, hipStream_t s) {
  const long long N = (long long)mf * mf * (dim == 3 ? mf : 1);
  if (dim == 3) export_prolong_kernel<3><<<blocks_of(N + 1, 256), 256, 0, s>>>(mf, mc, rowptr, colind, val);
  else export_prolong_kernel<2><<<blocks_of(N + 1, 256), 256, 0, s>>>(mf, mc, rowptr, colind, val);
}

void launch_export_restrict(int dim, int mf, int mc, int* rowptr, int* colind, double* val, hipStream_t s) {
  const long long N = (long long)mc * mc * (dim == 3 ? mc : 1);
  if (dim == 3) export_restrict_kernel<3><<<blocks_of(N + 1, 256), 256, 0, s>>>(mf, mc, rowptr, colind, val);
  else export_restrict_kernel<2><<<blocks_of(N + 1, 256), 256, 0, s>>>(mf, mc, rowptr, colind, val);
}

}  // namespace pase
