// Grid kernels: Q1 stencil operators over node-major multi-vectors, damped
// Jacobi, residuals, restriction / prolongation between nested levels, and the
// setup kernels that build the Galerkin coarse stencils.
//
// Operators (paper Sec. 2.1, kappa constant per element):
//   A[i, i+o] = Kpat(o) * (sum of kappa over the elements shared by nodes i and i+o)
//   M[i, i+o] = (h/6)^d * prod_a (o_a == 0 ? 4 : 1)
// with Kpat(o) = sum_a k1(o_a) prod_{b != a} m1(o_b), k1(0) = 1/h, k1(+-1) = -1/h,
// m1(0) = 2h/6, m1(+-1) = h/6: the unit-coefficient Q1 element stiffness entry
// between two vertices of one cell depends only on which coordinates differ.
// Coarse levels carry the Galerkin product P^T A P as 3^d coefficients per node.
#include "internal.hpp"

namespace pase {

namespace {

template <int DIM>
struct NSt { static constexpr int v = (DIM == 3) ? 27 : 9; };

constexpr int kMaxNb = 64;

// Blocks are dispatched round-robin over the 8 XCDs; give each XCD a
// contiguous run of tiles so neighbouring tiles share that XCD's L2.
__device__ __forceinline__ int xcd_tile(int b, int nblocks) {
  const int per = nblocks >> 3;
  return (b & 7) * per + (b >> 3);
}

template <int DIM>
__device__ __forceinline__ void offs(int o, int& ox, int& oy, int& oz) {
  ox = o % 3 - 1;
  oy = (o / 3) % 3 - 1;
  oz = (DIM == 3) ? (o / 9 - 1) : 0;
}

template <int DIM>
__device__ __forceinline__ double kpat(int o, double h) {
  int ox, oy, oz;
  offs<DIM>(o, ox, oy, oz);
  const int od[3] = {ox, oy, oz};
  const double k0 = 1.0 / h, k1 = -1.0 / h, m0 = 2.0 * h / 6.0, m1 = h / 6.0;
  double s = 0.0;
#pragma unroll
  for (int a = 0; a < DIM; ++a) {
    double t = (od[a] == 0) ? k0 : k1;
#pragma unroll
    for (int b = 0; b < DIM; ++b)
      if (b != a) t *= (od[b] == 0) ? m0 : m1;
    s += t;
  }
  return s;
}

template <int DIM>
__device__ __forceinline__ double mpat(int o, double h) {
  int ox, oy, oz;
  offs<DIM>(o, ox, oy, oz);
  const double c = h / 6.0;
  double s = ((ox == 0) ? 4.0 : 1.0) * c * ((oy == 0) ? 4.0 : 1.0) * c;
  if (DIM == 3) s *= ((oz == 0) ? 4.0 : 1.0) * c;
  return s;
}

template <int DIM>
__device__ __forceinline__ void node_xyz(long long i, int m, int& x, int& y, int& z) {
  x = (int)(i % m);
  const long long q = i / m;
  if (DIM == 3) {
    y = (int)(q % m);
    z = (int)(q / m);
  } else {
    y = (int)q;
    z = 0;
  }
}

// The 3^d A-coefficients of node (x,y,z) on the fine level, from kappa.
template <int DIM>
__device__ void kappa_coefs(const double* __restrict__ kappa, int m, double h, int x, int y, int z, double* c) {
  const int n = m + 1;
  // kappa of the 2^d cells around the node: cell (x + cx, y + cy, z + cz)
  double kc[8];
#pragma unroll
  for (int q = 0; q < (1 << DIM); ++q) {
    const int cx = q & 1, cy = (q >> 1) & 1, cz = (q >> 2) & 1;
    long long e = (long long)(x + cx) + (long long)n * (y + cy);
    if (DIM == 3) e += (long long)n * n * (z + cz);
    kc[q] = kappa ? kappa[e] : 1.0;
  }
#pragma unroll
  for (int o = 0; o < NSt<DIM>::v; ++o) {
    int ox, oy, oz;
    offs<DIM>(o, ox, oy, oz);
    double s = 0.0;
#pragma unroll
    for (int q = 0; q < (1 << DIM); ++q) {
      const int cx = q & 1, cy = (q >> 1) & 1, cz = (q >> 2) & 1;
      // cell holds both nodes iff for every axis with o != 0 the cell lies on that side
      bool ok = (ox == 0 || cx == (ox > 0)) && (oy == 0 || cy == (oy > 0));
      if (DIM == 3) ok = ok && (oz == 0 || cz == (oz > 0));
      if (ok) s += kc[q];
    }
    c[o] = kpat<DIM>(o, h) * s;
  }
}

template <int DIM>
__device__ __forceinline__ long long flat_off(int o, int m) {
  int ox, oy, oz;
  offs<DIM>(o, ox, oy, oz);
  long long f = ox + (long long)oy * m;
  if (DIM == 3) f += (long long)oz * m * m;
  return f;
}

template <int DIM, int SRC, int EPI, typename T>
__global__ __launch_bounds__(kBlock) void stencil_kernel(StencilArgs a, int slots, int nb, int tiles) {
  const T* __restrict__ X = (const T*)a.x;
  const T* __restrict__ Bv = (const T*)a.b;
  T* __restrict__ O1 = (T*)a.out1;
  T* __restrict__ O2 = (T*)a.out2;
  constexpr int NS = NSt<DIM>::v;
  __shared__ double sc[kMaxNb][NS];
  __shared__ unsigned smask[kMaxNb];
  __shared__ double sm[NS];
  __shared__ double red[3][kBlock];
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  if (tile >= tiles) return;
  const long long n0 = (long long)tile * nb;
  const int nloc = (int)((a.N - n0 < nb) ? (a.N - n0) : nb);
  const int m = a.m;
  for (int t = threadIdx.x; t < nloc; t += kBlock) {
    int x, y, z;
    node_xyz<DIM>(n0 + t, m, x, y, z);
    unsigned mask = 0;
#pragma unroll
    for (int o = 0; o < NS; ++o) {
      int ox, oy, oz;
      offs<DIM>(o, ox, oy, oz);
      bool ok = (x + ox >= 0) && (x + ox < m) && (y + oy >= 0) && (y + oy < m);
      if (DIM == 3) ok = ok && (z + oz >= 0) && (z + oz < m);
      mask |= ok ? (1u << o) : 0u;
    }
    smask[t] = mask;
    if (EPI != EPI_AM || a.out1) {
      if (SRC == (int)ASource::Kappa) {
        double c[NS];
        kappa_coefs<DIM>(a.kappa, m, a.h, x, y, z, c);
#pragma unroll
        for (int o = 0; o < NS; ++o) sc[t][o] = c[o];
      } else {
        const double* cp = a.coef + (n0 + t) * NS;
#pragma unroll
        for (int o = 0; o < NS; ++o) sc[t][o] = cp[o];
      }
    }
  }
  if (threadIdx.x < NS) sm[threadIdx.x] = mpat<DIM>(threadIdx.x, a.h);
  __syncthreads();

  const int k = a.k;
  const int col = threadIdx.x % k;
  const int slot = threadIdx.x / k;
  const bool active = slot < slots;
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
  if (active) {
    const double lamc = (EPI == EPI_EIGRES) ? a.lam[col] : 0.0;
    for (int j = slot; j < nloc; j += slots) {
      const long long node = n0 + j;
      const long long idx = node * k + col;
      const unsigned mask = smask[j];
      double ax = 0.0, mx = 0.0;
      const bool needA = (EPI != EPI_AM) || (a.out1 != nullptr);
      const bool needM = (EPI == EPI_EIGRES) || (EPI == EPI_AM && a.out2 != nullptr);
#pragma unroll
      for (int o = 0; o < NS; ++o) {
        if (mask & (1u << o)) {
          const double v = (double)X[idx + flat_off<DIM>(o, m) * k];
          if (needA) ax = fma(sc[j][o], v, ax);
          if (needM) mx = fma(sm[o], v, mx);
        }
      }
      if (EPI == EPI_AM) {
        if (O1) O1[idx] = (T)ax;
        if (O2) O2[idx] = (T)mx;
      } else if (EPI == EPI_RESID) {
        O1[idx] = (T)((double)Bv[idx] - ax);
      } else if (EPI == EPI_SWEEP) {
        O1[idx] = (T)((double)X[idx] + a.omega * a.dinv[node] * ((double)Bv[idx] - ax));
      } else {  // EPI_EIGRES
        const double r = lamc * mx - ax;
        O1[idx] = (T)r;
        acc0 = fma(r, r, acc0);
        acc1 = fma(mx, mx, acc1);
        acc2 = fma((double)X[idx], mx, acc2);
      }
    }
  }
  if (EPI == EPI_EIGRES) {
    red[0][threadIdx.x] = acc0;
    red[1][threadIdx.x] = acc1;
    red[2][threadIdx.x] = acc2;
    __syncthreads();
    if ((int)threadIdx.x < k) {
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
      for (int s = 0; s < slots; ++s) {
        s0 += red[0][s * k + threadIdx.x];
        s1 += red[1][s * k + threadIdx.x];
        s2 += red[2][s * k + threadIdx.x];
      }
      double* p = a.partial + (size_t)tile * 3 * k;
      p[threadIdx.x] = s0;
      p[k + threadIdx.x] = s1;
      p[2 * k + threadIdx.x] = s2;
    }
  }
}

// ---- flat (node, column) kernels: thread q handles node q / k, column q % k.
// 32-bit index arithmetic (the launchers fall back to the 64-bit kernels when
// N k >= 2^31); one thread per output keeps thousands of waves in flight, which
// the small coarse levels need to hide L2 latency.

__device__ __forceinline__ void flat_split(unsigned q, unsigned k, unsigned& node, unsigned& col) {
  node = q / k;
  col = q - node * k;
}

template <int DIM>
__device__ __forceinline__ void node_xyz32(unsigned node, unsigned m, int& x, int& y, int& z) {
  const unsigned q = node / m;
  x = (int)(node - q * m);
  if (DIM == 3) {
    const unsigned r = q / m;
    y = (int)(q - r * m);
    z = (int)r;
  } else {
    y = (int)q;
    z = 0;
  }
}

// A x, M x, b - A x or a damped Jacobi sweep on a level whose operator is
// given by 3^d coefficients per node (Galerkin coarse levels) or formed from
// kappa (fine level of 2D problems).
template <int DIM, int SRC, int EPI, typename T>
__global__ __launch_bounds__(kBlock) void flat_stencil_kernel(StencilArgs a) {
  constexpr int NS = NSt<DIM>::v;
  const unsigned k = (unsigned)a.k, N = (unsigned)a.N;
  const unsigned q = blockIdx.x * kBlock + threadIdx.x;
  if (q >= N * k) return;
  unsigned node, col;
  flat_split(q, k, node, col);
  const int m = a.m;
  int x, y, z;
  node_xyz32<DIM>(node, (unsigned)m, x, y, z);
  const T* __restrict__ X = (const T*)a.x;
  const bool needA = (EPI != EPI_AM) || (a.out1 != nullptr);
  const bool needM = (EPI == EPI_AM) && (a.out2 != nullptr);
  double c[NS];
  if (needA) {
    if (SRC == (int)ASource::Kappa) {
      kappa_coefs<DIM>(a.kappa, m, a.h, x, y, z, c);
    } else {
      const double* __restrict__ cp = a.coef + (size_t)node * NS;
#pragma unroll
      for (int o = 0; o < NS; ++o) c[o] = cp[o];
    }
  }
  const bool vx[3] = {x > 0, true, x + 1 < m};
  const bool vy[3] = {y > 0, true, y + 1 < m};
  const bool vz[3] = {DIM == 3 ? z > 0 : false, true, DIM == 3 ? z + 1 < m : false};
  const int sy = m * (int)k, sz = m * m * (int)k;
  const long long base = (long long)q;
  double ax = 0.0, mx = 0.0, xc = 0.0;
#pragma unroll
  for (int o = 0; o < NS; ++o) {
    const int ox = o % 3, oy = (o / 3) % 3, oz = (DIM == 3) ? o / 9 : 1;
    if (vx[ox] && vy[oy] && vz[oz]) {
      const long long off = (long long)(ox - 1) * (int)k + (long long)(oy - 1) * sy +
                            ((DIM == 3) ? (long long)(oz - 1) * sz : 0);
      const double v = (double)X[base + off];
      if (o == NS / 2) xc = v;
      if (needA) ax = fma(c[o], v, ax);
      if (needM) mx = fma(mpat<DIM>(o, a.h), v, mx);
    }
  }
  if (EPI == EPI_AM) {
    if (a.out1) ((T*)a.out1)[q] = (T)ax;
    if (a.out2) ((T*)a.out2)[q] = (T)mx;
  } else if (EPI == EPI_RESID) {
    ((T*)a.out1)[q] = (T)((double)((const T*)a.b)[q] - ax);
  } else {  // EPI_SWEEP
    ((T*)a.out1)[q] = (T)(xc + a.omega * a.dinv[node] * ((double)((const T*)a.b)[q] - ax));
  }
}

template <typename T>
__global__ void first_sweep_flat_kernel(unsigned n, unsigned k, const double* __restrict__ dinv, double omega,
                                        const T* __restrict__ b, T* __restrict__ x) {
  const unsigned i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  x[i] = (T)(omega * dinv[i / k] * (double)b[i]);
}

// 3D restriction marching along x: thread (column, coarse Y, coarse Z, run of kRestrictRun coarse
// x) forms, for each fine x-plane it meets, the weighted 3 x 3 (y, z) sum around (2Y+1, 2Z+1), and
// combines three consecutive ones with weights 1/2, 1, 1/2; the plane at 2X+2 is shared with the
// next coarse node, so a coarse value costs 18 fine loads instead of 27.
constexpr int kRestrictRun = 8;

template <typename T>
__global__ __launch_bounds__(kBlock) void restrict_march_kernel(int mf, int mc, unsigned k, const T* __restrict__ xf,
                                                               T* __restrict__ xc) {
  const unsigned nseg = (unsigned)(mc + kRestrictRun - 1) / kRestrictRun;
  const unsigned q = blockIdx.x * kBlock + threadIdx.x;
  if (q >= (unsigned)mc * (unsigned)mc * nseg * k) return;
  unsigned col, t;
  flat_split(q, k, t, col);
  const int Y = (int)(t % (unsigned)mc);
  t /= (unsigned)mc;
  const int Z = (int)(t % (unsigned)mc);
  const int seg = (int)(t / (unsigned)mc);
  const int X0 = seg * kRestrictRun, X1 = min(mc, X0 + kRestrictRun);
  const long long sy = (long long)mf * k, sz = (long long)mf * mf * k;
  const T* __restrict__ base = xf + (long long)(2 * Z + 1) * sz + (long long)(2 * Y + 1) * sy + col;
  auto plane = [&](int fx) -> double {
    const T* p = base + (long long)fx * k;
    double s = 0.0;
#pragma unroll
    for (int dz = -1; dz <= 1; ++dz)
#pragma unroll
      for (int dy = -1; dy <= 1; ++dy)
        s = fma((dz ? 0.5 : 1.0) * (dy ? 0.5 : 1.0), (double)p[dz * sz + dy * sy], s);
    return s;
  };
  double prev = plane(2 * X0);
  T* __restrict__ out = xc + ((long long)(Z * mc + Y) * mc) * k + col;
  for (int X = X0; X < X1; ++X) {
    const double mid = plane(2 * X + 1), nxt = plane(2 * X + 2);
    out[(long long)X * k] = (T)(0.5 * prev + mid + 0.5 * nxt);
    prev = nxt;
  }
}

template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) void restrict_flat_kernel(int mf, int mc, unsigned k, const T* __restrict__ xf,
                                                              T* __restrict__ xc) {
  unsigned Nc = (unsigned)mc * mc;
  if (DIM == 3) Nc *= mc;
  const unsigned q = blockIdx.x * kBlock + threadIdx.x;
  if (q >= Nc * k) return;
  unsigned node, col;
  flat_split(q, k, node, col);
  int X, Y, Z;
  node_xyz32<DIM>(node, (unsigned)mc, X, Y, Z);
  // fine node (2X+1, 2Y+1, 2Z+1) and its neighbours, weights 1 (centre) and 1/2 per offset axis;
  // all 3^d fine nodes are interior because the coarse node is
  const unsigned ctr = (unsigned)(2 * X + 1) + (unsigned)mf * ((unsigned)(2 * Y + 1) +
                       (DIM == 3 ? (unsigned)mf * (unsigned)(2 * Z + 1) : 0u));
  const long long sy = (long long)mf * k, sz = (long long)mf * mf * k;
  const T* __restrict__ p = xf + (long long)ctr * k + col;
  double s = 0.0;
#pragma unroll
  for (int oz = (DIM == 3 ? -1 : 0); oz <= (DIM == 3 ? 1 : 0); ++oz) {
    const double wz = (oz == 0) ? 1.0 : 0.5;
#pragma unroll
    for (int oy = -1; oy <= 1; ++oy) {
      const double wy = (oy == 0) ? 1.0 : 0.5;
#pragma unroll
      for (int ox = -1; ox <= 1; ++ox) {
        const double wx = (ox == 0) ? 1.0 : 0.5;
        s = fma(wx * wy * wz, (double)p[ox * (long long)k + oy * sy + oz * sz], s);
      }
    }
  }
  xc[q] = (T)s;
}

// Prolongation by coarse cells: thread (group g, column) with g = (gx, gy, gz), each in
// [-1, mc - 1], owns the fine nodes 2g+1 (on coarse node g, weight 1) and 2g+2 (between coarse
// nodes g and g+1, weights 1/2) per axis: 2^d fine nodes from the 2^d coarse corners, so every
// coarse value is read about once per cell instead of once per fine node.  Corners outside
// [0, mc) are the Dirichlet boundary (zero); fine nodes 2g+1 with g = -1 do not exist.
template <int DIM, typename T>
__global__ __launch_bounds__(kBlock) void prolong_cell_kernel(int mf, int mc, unsigned k, const T* __restrict__ xc,
                                                             T* __restrict__ xf, int mode, const T* __restrict__ b,
                                                             const double* __restrict__ dinv, double omega) {
  const unsigned ng = (unsigned)mc + 1;
  unsigned G = ng * ng;
  if (DIM == 3) G *= ng;
  const unsigned q = blockIdx.x * kBlock + threadIdx.x;
  if (q >= G * k) return;
  unsigned grp, col;
  flat_split(q, k, grp, col);
  int gx, gy, gz;
  node_xyz32<DIM>(grp, ng, gx, gy, gz);
  gx -= 1;
  gy -= 1;
  gz -= (DIM == 3) ? 1 : 0;
  // corners (unconditional loads from clamped addresses, zeroed outside the mesh)
  constexpr int NZ = (DIM == 3) ? 2 : 1;
  double v[NZ][2][2];
#pragma unroll
  for (int cz = 0; cz < NZ; ++cz)
#pragma unroll
    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
      for (int cx = 0; cx < 2; ++cx) {
        const int X = gx + cx, Y = gy + cy, Z = (DIM == 3) ? gz + cz : 0;
        const bool in = X >= 0 && X < mc && Y >= 0 && Y < mc && (DIM == 2 || (Z >= 0 && Z < mc));
        const int Xc = min(max(X, 0), mc - 1), Yc = min(max(Y, 0), mc - 1), Zc = (DIM == 3) ? min(max(Z, 0), mc - 1) : 0;
        const unsigned cn = (unsigned)Xc + (unsigned)mc * ((unsigned)Yc + (DIM == 3 ? (unsigned)mc * (unsigned)Zc : 0u));
        const double val = (double)xc[(size_t)cn * k + col];
        v[cz][cy][cx] = in ? val : 0.0;
      }
  // separable interpolation: per axis, a = corner 0 (weight 1), b = (corner 0 + corner 1) / 2
  double wx[NZ][2][2];                          // [cz][cy][a/b]
#pragma unroll
  for (int cz = 0; cz < NZ; ++cz)
#pragma unroll
    for (int cy = 0; cy < 2; ++cy) {
      wx[cz][cy][0] = v[cz][cy][0];
      wx[cz][cy][1] = 0.5 * (v[cz][cy][0] + v[cz][cy][1]);
    }
  double wy[NZ][2][2];                          // [cz][ya/yb][xa/xb]
#pragma unroll
  for (int cz = 0; cz < NZ; ++cz)
#pragma unroll
    for (int sx = 0; sx < 2; ++sx) {
      wy[cz][0][sx] = wx[cz][0][sx];
      wy[cz][1][sx] = 0.5 * (wx[cz][0][sx] + wx[cz][1][sx]);
    }
#pragma unroll
  for (int sz = 0; sz < NZ; ++sz)
#pragma unroll
    for (int sy = 0; sy < 2; ++sy)
#pragma unroll
      for (int sx = 0; sx < 2; ++sx) {
        const double val = (DIM == 3) ? (sz ? 0.5 * (wy[0][sy][sx] + wy[1][sy][sx]) : wy[0][sy][sx]) : wy[0][sy][sx];
        const int fx = 2 * gx + 1 + sx, fy = 2 * gy + 1 + sy, fz = (DIM == 3) ? 2 * gz + 1 + sz : 0;
        if (fx < 0 || fy < 0 || fz < 0) continue;                 // fine node 2g+1 with g = -1
        const unsigned fn = (unsigned)fx + (unsigned)mf * ((unsigned)fy + (DIM == 3 ? (unsigned)mf * (unsigned)fz : 0u));
        T* dst = xf + (size_t)fn * k + col;
        if (mode == 0) *dst = (T)val;
        else if (mode == 1) *dst = (T)((double)*dst + val);
        else if (mode == 2) *dst = (T)((double)*dst - val);
        else *dst = (T)fma(omega * dinv[fn], (double)b[(size_t)fn * k + col], val);
      }
}

template <typename T>
__global__ void first_sweep_kernel(long long N, int k, const double* __restrict__ dinv, double omega,
                                   const T* __restrict__ b, T* __restrict__ x) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * k) return;
  x[i] = (T)(omega * dinv[i / k] * (double)b[i]);
}

template <int DIM, typename T>
__global__ void restrict_kernel(int mf, int mc, int k, const T* __restrict__ xf, T* __restrict__ xc) {
  long long Nc = (long long)mc * mc;
  if (DIM == 3) Nc *= mc;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Nc * k) return;
  const long long node = i / k;
  const int col = (int)(i % k);
  int X, Y, Z;
  node_xyz<DIM>(node, mc, X, Y, Z);
  const int fx = 2 * X + 1, fy = 2 * Y + 1, fz = 2 * Z + 1;
  double s = 0.0;
  for (int oz = (DIM == 3 ? -1 : 0); oz <= (DIM == 3 ? 1 : 0); ++oz) {
    const double wz = (oz == 0) ? 1.0 : 0.5;
    for (int oy = -1; oy <= 1; ++oy) {
      const double wy = (oy == 0) ? 1.0 : 0.5;
      for (int ox = -1; ox <= 1; ++ox) {
        const double wx = (ox == 0) ? 1.0 : 0.5;
        long long f = (fx + ox) + (long long)mf * (fy + oy);
        if (DIM == 3) f += (long long)mf * mf * (fz + oz);
        s = fma(wx * wy * wz, (double)xf[f * k + col], s);
      }
    }
  }
  xc[i] = (T)s;
}

// Coarse indices and weights that interpolate fine coordinate f (ratio 2).
__device__ __forceinline__ int p1d(int f, int mc, int* I, double* w) {
  if (f & 1) {
    I[0] = (f - 1) >> 1;
    w[0] = 1.0;
    return 1;
  }
  int c = 0;
  const int a = (f >> 1) - 1, b = f >> 1;
  if (a >= 0) { I[c] = a; w[c] = 0.5; ++c; }
  if (b < mc) { I[c] = b; w[c] = 0.5; ++c; }
  return c;
}

template <int DIM, typename T>
__global__ void prolong_kernel(int mf, int mc, int k, const T* __restrict__ xc, T* __restrict__ xf,
                               int mode, const T* __restrict__ b, const double* __restrict__ dinv, double omega) {
  long long Nf = (long long)mf * mf;
  if (DIM == 3) Nf *= mf;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= Nf * k) return;
  const long long node = i / k;
  const int col = (int)(i % k);
  int x, y, z;
  node_xyz<DIM>(node, mf, x, y, z);
  int Ix[2], Iy[2], Iz[2] = {0, 0};
  double wx[2], wy[2], wz[2] = {1.0, 1.0};
  const int nx = p1d(x, mc, Ix, wx), ny = p1d(y, mc, Iy, wy);
  const int nz = (DIM == 3) ? p1d(z, mc, Iz, wz) : 1;
  double s = 0.0;
  for (int c = 0; c < nz; ++c)
    for (int b = 0; b < ny; ++b)
      for (int a = 0; a < nx; ++a) {
        long long J = Ix[a] + (long long)mc * Iy[b];
        if (DIM == 3) J += (long long)mc * mc * Iz[c];
        s = fma(wx[a] * wy[b] * wz[c], (double)xc[J * k + col], s);
      }
  if (mode == 0) xf[i] = (T)s;
  else if (mode == 1) xf[i] = (T)((double)xf[i] + s);
  else if (mode == 2) xf[i] = (T)((double)xf[i] - s);
  else xf[i] = (T)fma(omega * dinv[node], (double)b[i], s);
}

// node average of log kappa over the 2^3 elements around each interior node (3D)
__global__ void node_logk_kernel(int n, const double* __restrict__ kappa, double* __restrict__ out) {
  const int m = n - 1;
  const long long N = (long long)m * m * m;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int x = (int)(i % m), y = (int)((i / m) % m), z = (int)(i / ((long long)m * m));
  double s = 0.0;
  for (int cz = 0; cz < 2; ++cz)
    for (int cy = 0; cy < 2; ++cy)
      for (int cx = 0; cx < 2; ++cx) s += log(kappa[((long long)(z + cz) * n + (y + cy)) * n + (x + cx)]);
  out[i] = s / 8.0;
}

template <int DIM>
__global__ void kappa_dinv_kernel(int n, const double* __restrict__ kappa, double* __restrict__ dinv) {
  const int m = n - 1;
  long long N = (long long)m * m;
  if (DIM == 3) N *= m;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int x, y, z;
  node_xyz<DIM>(i, m, x, y, z);
  double c[NSt<DIM>::v];
  kappa_coefs<DIM>(kappa, m, 1.0 / n, x, y, z, c);
  dinv[i] = 1.0 / c[NSt<DIM>::v / 2];
}

template <int DIM>
__device__ __forceinline__ int color_of(int x, int y, int z) {
  return (x % 3) + 3 * (y % 3) + ((DIM == 3) ? 9 * (z % 3) : 0);
}

template <int DIM>
__global__ void color_probe_kernel(int m, double* __restrict__ E) {
  constexpr int NS = NSt<DIM>::v;
  long long N = (long long)m * m;
  if (DIM == 3) N *= m;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N * NS) return;
  const long long node = i / NS;
  const int c = (int)(i % NS);
  int x, y, z;
  node_xyz<DIM>(node, m, x, y, z);
  E[i] = (color_of<DIM>(x, y, z) == c) ? 1.0 : 0.0;
}

// Y = (P^T A P) E for the colour probes E: Y[I, colour(J)] = A_c[I, J] for the
// unique J of that colour within distance 1 of I.
template <int DIM>
__global__ void extract_galerkin_kernel(int m, const double* __restrict__ Y, double* __restrict__ coef,
                                        double* __restrict__ dinv) {
  constexpr int NS = NSt<DIM>::v;
  long long N = (long long)m * m;
  if (DIM == 3) N *= m;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int x, y, z;
  node_xyz<DIM>(i, m, x, y, z);
  for (int o = 0; o < NS; ++o) {
    int ox, oy, oz;
    offs<DIM>(o, ox, oy, oz);
    bool ok = (x + ox >= 0) && (x + ox < m) && (y + oy >= 0) && (y + oy < m);
    if (DIM == 3) ok = ok && (z + oz >= 0) && (z + oz < m);
    coef[i * NS + o] = ok ? Y[i * NS + color_of<DIM>(x + ox, y + oy, z + oz)] : 0.0;
  }
  dinv[i] = 1.0 / coef[i * NS + NS / 2];
}

// 1D Q1 integrals on a cell [0, h] for local vertices i, j in {0, 1}: stiffness, mass, and the
// derivative-value product int phi_i' phi_j (independent of j)
__device__ inline double q1_s(int i, int j, double h) { return (i == j ? 1.0 : -1.0) / h; }
__device__ inline double q1_m(int i, int j, double h) { return (i == j ? 2.0 : 1.0) * h / 6.0; }
__device__ inline double q1_g(int i) { return i ? 0.5 : -0.5; }

// Element matrix entry between local vertices I and J of a cube cell of side h, for the constant
// symmetric tensor T (a11, a12, a13, a22, a23, a33) and reaction phi:
// int grad phi_I . T grad phi_J + phi phi_I phi_J.  Tensor-product factors: the diagonal terms are
// s m m and its permutations, an off-diagonal pair (a, b) gives T_ab (g_I_a g_J_b + g_I_b g_J_a) m_c.
__device__ double general_entry(const double* T, double phi, const int* I, const int* J, double h) {
  double S[3], Mv[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    S[d] = q1_s(I[d], J[d], h);
    Mv[d] = q1_m(I[d], J[d], h);
  }
  double v = phi * Mv[0] * Mv[1] * Mv[2];
  v += T[0] * S[0] * Mv[1] * Mv[2] + T[3] * Mv[0] * S[1] * Mv[2] + T[5] * Mv[0] * Mv[1] * S[2];
  v += T[1] * (q1_g(I[0]) * q1_g(J[1]) + q1_g(J[0]) * q1_g(I[1])) * Mv[2];
  v += T[2] * (q1_g(I[0]) * q1_g(J[2]) + q1_g(J[0]) * q1_g(I[2])) * Mv[1];
  v += T[4] * (q1_g(I[1]) * q1_g(J[2]) + q1_g(J[1]) * q1_g(I[2])) * Mv[0];
  return v;
}

// Fine-level 27-point stencil of A = -div(T grad) + phi (3D, T and phi constant per element), one
// thread per interior node: coefficient o sums the element entries of the (up to 8) cells that
// hold both the node and its neighbour o; coefficients to nodes outside the domain are 0.
__global__ void assemble_general_kernel(int n, const double* __restrict__ tensor, const double* __restrict__ reaction,
                                        double* __restrict__ coef, double* __restrict__ dinv) {
  const int m = n - 1;
  const long long N = (long long)m * m * m;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  const int x = (int)(i % m), y = (int)((i / m) % m), z = (int)(i / ((long long)m * m));
  const double h = 1.0 / n;
  for (int o = 0; o < 27; ++o) {
    const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = o / 9 - 1;
    const bool ok = x + ox >= 0 && x + ox < m && y + oy >= 0 && y + oy < m && z + oz >= 0 && z + oz < m;
    double v = 0.0;
    if (ok) {
      for (int a = 0; a < 8; ++a) {
        const int I[3] = {a & 1, (a >> 1) & 1, (a >> 2) & 1};
        const int J[3] = {I[0] + ox, I[1] + oy, I[2] + oz};
        if (J[0] < 0 || J[0] > 1 || J[1] < 0 || J[1] > 1 || J[2] < 0 || J[2] > 1) continue;
        // the cell whose corner I is this node (full-grid node coordinate x + 1)
        const long long e = (long long)(x + 1 - I[0]) + (long long)n * (y + 1 - I[1]) +
                            (long long)n * n * (z + 1 - I[2]);
        v += general_entry(tensor + e * 6, reaction ? reaction[e] : 0.0, I, J, h);
      }
    }
    coef[i * 27 + o] = v;
  }
  dinv[i] = 1.0 / coef[i * 27 + 13];
}

template <int DIM>
__global__ void stencil_to_dense_kernel(int m, const double* __restrict__ coef, double hmass, int use_mass,
                                        double* __restrict__ D) {
  constexpr int NS = NSt<DIM>::v;
  long long N = (long long)m * m;
  if (DIM == 3) N *= m;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int x, y, z;
  node_xyz<DIM>(i, m, x, y, z);
  for (long long j = 0; j < N; ++j) D[i * N + j] = 0.0;
  for (int o = 0; o < NS; ++o) {
    int ox, oy, oz;
    offs<DIM>(o, ox, oy, oz);
    bool ok = (x + ox >= 0) && (x + ox < m) && (y + oy >= 0) && (y + oy < m);
    if (DIM == 3) ok = ok && (z + oz >= 0) && (z + oz < m);
    if (!ok) continue;
    const long long j = i + flat_off<DIM>(o, m);
    D[i * N + j] = use_mass ? mpat<DIM>(o, hmass) : coef[i * NS + o];
  }
}

inline unsigned nblk(long long n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

GridLaunch grid_launch(long long N, int k) {
  GridLaunch g;
  g.slots = kBlock / k;
  if (g.slots > kMaxNb) g.slots = kMaxNb;
  if (g.slots < 1) g.slots = 1;
  const int npass = (kMaxNb / g.slots) > 0 ? (kMaxNb / g.slots) : 1;
  g.nb = g.slots * npass;
  g.tiles = (int)((N + g.nb - 1) / g.nb);
  g.blocks = ((g.tiles + 7) / 8) * 8;
  return g;
}

template <int DIM, int SRC, typename T>
static void stencil_dispatch_epi(const StencilArgs& a, Epi epi, const GridLaunch& g, hipStream_t s) {
  switch (epi) {
    case EPI_AM:
      stencil_kernel<DIM, SRC, EPI_AM, T><<<g.blocks, kBlock, 0, s>>>(a, g.slots, g.nb, g.tiles);
      break;
    case EPI_RESID:
      stencil_kernel<DIM, SRC, EPI_RESID, T><<<g.blocks, kBlock, 0, s>>>(a, g.slots, g.nb, g.tiles);
      break;
    case EPI_SWEEP:
      stencil_kernel<DIM, SRC, EPI_SWEEP, T><<<g.blocks, kBlock, 0, s>>>(a, g.slots, g.nb, g.tiles);
      break;
    case EPI_EIGRES:
      stencil_kernel<DIM, SRC, EPI_EIGRES, T><<<g.blocks, kBlock, 0, s>>>(a, g.slots, g.nb, g.tiles);
      break;
    default:   // the fused-dot, two-sweep and single-output epilogues exist on the fine 3D path only
      break;
  }
}

constexpr long long kFlatMax = 0x7fffffffLL;   // flat kernels index (node, column) pairs in 32 bits

template <int DIM, int SRC, typename T>
static void flat_dispatch_epi(const StencilArgs& a, Epi epi, hipStream_t s) {
  const unsigned blocks = nblk(a.N * a.k);
  switch (epi) {
    case EPI_AM: flat_stencil_kernel<DIM, SRC, EPI_AM, T><<<blocks, kBlock, 0, s>>>(a); break;
    case EPI_RESID: flat_stencil_kernel<DIM, SRC, EPI_RESID, T><<<blocks, kBlock, 0, s>>>(a); break;
    case EPI_SWEEP: flat_stencil_kernel<DIM, SRC, EPI_SWEEP, T><<<blocks, kBlock, 0, s>>>(a); break;
    default: break;
  }
}

template <typename T>
static void launch_stencil_t(const StencilArgs& a, Epi epi, hipStream_t s) {
  if (epi != EPI_EIGRES && a.N * a.k <= kFlatMax) {
    if (a.dim == 3) {
      if (a.src == ASource::Kappa) flat_dispatch_epi<3, 0, T>(a, epi, s);
      else flat_dispatch_epi<3, 1, T>(a, epi, s);
    } else {
      if (a.src == ASource::Kappa) flat_dispatch_epi<2, 0, T>(a, epi, s);
      else flat_dispatch_epi<2, 1, T>(a, epi, s);
    }
    return;
  }
  const GridLaunch g = grid_launch(a.N, a.k);
  if (a.dim == 3) {
    if (a.src == ASource::Kappa) stencil_dispatch_epi<3, 0, T>(a, epi, g, s);
    else stencil_dispatch_epi<3, 1, T>(a, epi, g, s);
  } else {
    if (a.src == ASource::Kappa) stencil_dispatch_epi<2, 0, T>(a, epi, g, s);
    else stencil_dispatch_epi<2, 1, T>(a, epi, g, s);
  }
}

void launch_stencil(const StencilArgs& a, Epi epi, hipStream_t s) {
  if (a.fp32) launch_stencil_t<float>(a, epi, s);
  else launch_stencil_t<double>(a, epi, s);
}

void launch_first_sweep(int dim, long long N, int k, const double* dinv, double omega, const void* b, void* x,
                        int fp32, hipStream_t s) {
  (void)dim;
  if (N * k <= kFlatMax) {
    const unsigned n = (unsigned)(N * k);
    if (fp32)
      first_sweep_flat_kernel<float><<<nblk(N * k), kBlock, 0, s>>>(n, (unsigned)k, dinv, omega, (const float*)b,
                                                                    (float*)x);
    else
      first_sweep_flat_kernel<double><<<nblk(N * k), kBlock, 0, s>>>(n, (unsigned)k, dinv, omega, (const double*)b,
                                                                     (double*)x);
    return;
  }
  if (fp32) first_sweep_kernel<float><<<nblk(N * k), kBlock, 0, s>>>(N, k, dinv, omega, (const float*)b, (float*)x);
  else first_sweep_kernel<double><<<nblk(N * k), kBlock, 0, s>>>(N, k, dinv, omega, (const double*)b, (double*)x);
}

template <typename T>
static void launch_restrict_t(int dim, int mf, int mc, int k, const T* xf, T* xc, hipStream_t s) {
  long long Nc = (long long)mc * mc * (dim == 3 ? mc : 1);
  long long Nf = (long long)mf * mf * (dim == 3 ? mf : 1);
  if (Nf * k <= kFlatMax) {
    if (dim == 3 && mc >= 24) {                 // small levels: the gather has more parallelism
      const long long nseg = (mc + kRestrictRun - 1) / kRestrictRun;
      restrict_march_kernel<T><<<nblk((long long)mc * mc * nseg * k), kBlock, 0, s>>>(mf, mc, (unsigned)k, xf, xc);
    } else if (dim == 3) {
      restrict_flat_kernel<3, T><<<nblk(Nc * k), kBlock, 0, s>>>(mf, mc, (unsigned)k, xf, xc);
    } else {
      restrict_flat_kernel<2, T><<<nblk(Nc * k), kBlock, 0, s>>>(mf, mc, (unsigned)k, xf, xc);
    }
    return;
  }
  if (dim == 3) restrict_kernel<3, T><<<nblk(Nc * k), kBlock, 0, s>>>(mf, mc, k, xf, xc);
  else restrict_kernel<2, T><<<nblk(Nc * k), kBlock, 0, s>>>(mf, mc, k, xf, xc);
}

void launch_restrict(int dim, int mf, int mc, int k, const void* xf, void* xc, int fp32, hipStream_t s) {
  if (fp32) launch_restrict_t<float>(dim, mf, mc, k, (const float*)xf, (float*)xc, s);
  else launch_restrict_t<double>(dim, mf, mc, k, (const double*)xf, (double*)xc, s);
}

// mode 0: xf = P xc, 1: xf += P xc, 2: xf -= P xc, 3: xf = omega D^{-1} b + P xc
template <typename T>
static void launch_prolong_t(int dim, int mf, int mc, int k, const T* xc, T* xf, int mode, const T* b,
                             const double* dinv, double omega, hipStream_t s) {
  long long Nf = (long long)mf * mf * (dim == 3 ? mf : 1);
  const long long G = (long long)(mc + 1) * (mc + 1) * (dim == 3 ? (mc + 1) : 1);
  if (Nf * k <= kFlatMax && G * k <= kFlatMax) {
    if (dim == 3)
      prolong_cell_kernel<3, T><<<nblk(G * k), kBlock, 0, s>>>(mf, mc, (unsigned)k, xc, xf, mode, b, dinv, omega);
    else
      prolong_cell_kernel<2, T><<<nblk(G * k), kBlock, 0, s>>>(mf, mc, (unsigned)k, xc, xf, mode, b, dinv, omega);
    return;
  }
  if (dim == 3) prolong_kernel<3, T><<<nblk(Nf * k), kBlock, 0, s>>>(mf, mc, k, xc, xf, mode, b, dinv, omega);
  else prolong_kernel<2, T><<<nblk(Nf * k), kBlock, 0, s>>>(mf, mc, k, xc, xf, mode, b, dinv, omega);
}

void launch_prolong(int dim, int mf, int mc, int k, const void* xc, void* xf, int mode, int fp32, hipStream_t s) {
  if (fp32) launch_prolong_t<float>(dim, mf, mc, k, (const float*)xc, (float*)xf, mode, nullptr, nullptr, 0.0, s);
  else launch_prolong_t<double>(dim, mf, mc, k, (const double*)xc, (double*)xf, mode, nullptr, nullptr, 0.0, s);
}

void launch_prolong_first(int dim, int mf, int mc, int k, const void* xc, void* xf, const void* b,
                          const double* dinv, double omega, int fp32, hipStream_t s) {
  if (fp32)
    launch_prolong_t<float>(dim, mf, mc, k, (const float*)xc, (float*)xf, 3, (const float*)b, dinv, omega, s);
  else
    launch_prolong_t<double>(dim, mf, mc, k, (const double*)xc, (double*)xf, 3, (const double*)b, dinv, omega, s);
}

template <int DIM>
__global__ void kappa_coefs_kernel(int n, const double* __restrict__ kappa, double* __restrict__ coef) {
  constexpr int NS = NSt<DIM>::v;
  const int m = n - 1;
  long long N = (long long)m * m;
  if (DIM == 3) N *= m;
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  int x, y, z;
  node_xyz<DIM>(i, m, x, y, z);
  double c[NS];
  kappa_coefs<DIM>(kappa, m, 1.0 / n, x, y, z, c);
  for (int o = 0; o < NS; ++o) coef[i * NS + o] = c[o];
}

void launch_kappa_coefs(int dim, int n, const double* kappa, double* coef, hipStream_t s) {
  const long long N = (long long)(n - 1) * (n - 1) * (dim == 3 ? (n - 1) : 1);
  if (dim == 3) kappa_coefs_kernel<3><<<nblk(N), kBlock, 0, s>>>(n, kappa, coef);
  else kappa_coefs_kernel<2><<<nblk(N), kBlock, 0, s>>>(n, kappa, coef);
}

void launch_kappa_dinv(int dim, int n, const double* kappa, double* dinv, hipStream_t s) {
  const long long N = (long long)(n - 1) * (n - 1) * (dim == 3 ? (n - 1) : 1);
  if (dim == 3) kappa_dinv_kernel<3><<<nblk(N), kBlock, 0, s>>>(n, kappa, dinv);
  else kappa_dinv_kernel<2><<<nblk(N), kBlock, 0, s>>>(n, kappa, dinv);
}

void launch_node_logk(int n, const double* kappa, double* out, hipStream_t s) {
  const long long N = (long long)(n - 1) * (n - 1) * (n - 1);
  node_logk_kernel<<<nblk(N), kBlock, 0, s>>>(n, kappa, out);
}

void launch_color_probe(int dim, int m, double* E, hipStream_t s) {
  const long long N = (long long)m * m * (dim == 3 ? m : 1);
  if (dim == 3) color_probe_kernel<3><<<nblk(N * 27), kBlock, 0, s>>>(m, E);
  else color_probe_kernel<2><<<nblk(N * 9), kBlock, 0, s>>>(m, E);
}

void launch_extract_galerkin(int dim, int m, const double* Y, double* coef, double* dinv, hipStream_t s) {
  const long long N = (long long)m * m * (dim == 3 ? m : 1);
  if (dim == 3) extract_galerkin_kernel<3><<<nblk(N), kBlock, 0, s>>>(m, Y, coef, dinv);
  else extract_galerkin_kernel<2><<<nblk(N), kBlock, 0, s>>>(m, Y, coef, dinv);
}

void launch_assemble_general(int n, const double* tensor, const double* reaction, double* coef, double* dinv,
                             hipStream_t s) {
  const long long N = (long long)(n - 1) * (n - 1) * (n - 1);
  assemble_general_kernel<<<nblk(N), kBlock, 0, s>>>(n, tensor, reaction, coef, dinv);
}

void launch_stencil_to_dense(int dim, int m, const double* coef, double hmass, int use_mass, double* D,
                             hipStream_t s) {
  const long long N = (long long)m * m * (dim == 3 ? m : 1);
  if (dim == 3) stencil_to_dense_kernel<3><<<nblk(N), kBlock, 0, s>>>(m, coef, hmass, use_mass, D);
  else stencil_to_dense_kernel<2><<<nblk(N), kBlock, 0, s>>>(m, coef, hmass, use_mass, D);
}

}  // namespace pase
