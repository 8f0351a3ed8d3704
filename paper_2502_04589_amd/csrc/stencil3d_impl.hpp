// Kernel and launch templates of the fine-level 3D Q1 operator (instantiated for
// float64 in stencil3d.hip and for float32 in stencil3d_f32.hip).
//
// Fine-level 3D Q1 operator over node-major multi-vectors, LDS-staged.
//
// A block owns an 8 x 8 tile of nodes in (x, y), a chunk of KC columns and a
// run of z-planes.  It marches up in z keeping three node planes of the
// multi-vector (with a one-node halo in x and y) in an LDS ring, so each input
// value is read from HBM once per block (plus the halo), and every output
// (node, column) takes its 27 neighbours from LDS.  The A-coefficients of a
// node come from the kappa of its 8 surrounding cells (two element layers,
// held in registers), or (ASM) from an assembled 27-coefficient row per node (the
// tensor-coefficient problem):
//   A[i, i+o] = Kpat(o) * (sum of kappa over the cells shared by nodes i and i+o),
//   M[i, i+o] = (h/6)^3 prod_a (o_a == 0 ? 4 : 1).
// Thread (node, column) mapping puts columns fastest, so global loads and
// stores of a node's KC columns are contiguous.
#pragma once

#include <type_traits>

#include "internal.hpp"

namespace pase {

namespace {


// Write-only target of the stores of lanes that have no output (nodes past the grid, columns past
// k, the step past the end of an odd z-run): every lane then issues the same memory operations,
// and no branch around a store leaves the compiler unsure which loads are still in flight.
__device__ double4 fine3_sink[1];

// 8 x 4 tiles with 8 vectors per node when k is a multiple of 8 vectors (whole 128-byte lines of a
// node row per block) or at least 64 columns in whole vectors (the last column chunk ragged): the
// rule that the column-sum partial rows follow as well (fine3_spatial_blocks)
__host__ __device__ inline bool fine3_wide_tile(int k, bool fp32) {
  const int vw = (fp32 && k % 4 == 0) ? 4 : 2;
  return k % vw == 0 && (k % (8 * vw) == 0 || k >= 64);
}

__device__ __forceinline__ int xcd_block(int b, int nblocks) {
  const int per = nblocks >> 3;
  return (b & 7) * per + (b >> 3);
}

// Sum of kappa over the cells of one layer that a node shares with its neighbour at (ox, oy):
// along an axis with offset -1 only the lower cell, +1 only the upper cell, 0 both.  c[cy][cx] are
// the node's 4 cells in that layer.
template <int OX, int OY>
__device__ __forceinline__ double cell_sum(const double (&c)[2][2]) {
  constexpr int x0 = (OX > 0) ? 1 : 0, y0 = (OY > 0) ? 1 : 0;
  if constexpr (OX != 0 && OY != 0) return c[y0][x0];
  else if constexpr (OX != 0) return c[0][x0] + c[1][x0];
  else if constexpr (OY != 0) return c[y0][0] + c[y0][1];
  else return (c[0][0] + c[0][1]) + (c[1][0] + c[1][1]);
}

template <int OX, int OY, int OZ>
__device__ __forceinline__ double kpat(double k0, double k1, double m0, double m1) {
  const double kx = (OX == 0) ? k0 : k1, ky = (OY == 0) ? k0 : k1, kz = (OZ == 0) ? k0 : k1;
  const double mx = (OX == 0) ? m0 : m1, my = (OY == 0) ? m0 : m1, mz = (OZ == 0) ? m0 : m1;
  return kx * my * mz + mx * ky * mz + mx * my * kz;
}

// vector of a thread's VW consecutive columns: double2 (16 bytes), float2 (8 bytes, k even)
// or float4 (16 bytes, k a multiple of 4)
template <typename T, int W> struct Vec;
template <> struct Vec<double, 2> { typedef double2 type; };
template <> struct Vec<float, 2> { typedef float2 type; };
template <> struct Vec<float, 4> { typedef float4 type; };

template <typename T, int W>
__device__ __forceinline__ double vget(const typename Vec<T, W>::type& v, int i) {
  if constexpr (W == 2) return i == 0 ? (double)v.x : (double)v.y;
  else return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}
template <typename T, int W>
__device__ __forceinline__ void vset(typename Vec<T, W>::type& v, int i, double x) {
  if constexpr (W == 2) { if (i == 0) v.x = (T)x; else v.y = (T)x; }
  else { if (i == 0) v.x = (float)x; else if (i == 1) v.y = (float)x; else if (i == 2) v.z = (float)x; else v.w = (float)x; }
}

constexpr int kSlots = 4;             // LDS ring: planes z-1, z, z+1 and the one being filled

template <typename T, int W, int BX, int BY, int NQ>
struct Fine3SmemV {
  typedef typename Vec<T, W>::type V;
  union {
    V xs[kSlots][BY + 2][BX + 2][NQ];
    double red[3][BX * BY * NQ * W];
  };
};

// NQ threads per node, each with a VW-column vector: a block covers KC = NQ VW columns of its
// tile (NQ = 5 when it splits k into whole chunks and 4 does not, e.g. k = 50 with VW = 2)
template <typename T, int VW, int EPI, bool CONSTK, bool VEC, int BX, int BY, int NQ, bool ASM>
__global__ __launch_bounds__(BX * BY * NQ) void fine3v_kernel(Fine3Args a) {
  constexpr int TX = BX, TY = BY;
  constexpr int kThreadsV = BX * BY * NQ;   // (node, column vector) pairs of a tile
  typedef typename Vec<T, VW>::type V;
  constexpr int KC = NQ * VW;                // columns per block
  __shared__ Fine3SmemV<T, VW, BX, BY, NQ> sm;
  const int m = a.m, n = m + 1, k = a.k;
  const int ntx = (m + TX - 1) / TX;
  const int nty = (m + TY - 1) / TY;
  const int nch = (k + KC - 1) / KC;
  const int nzc = a.nzc;
  const int total = ntx * nty * nzc * nch;
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  if (lb >= total) return;
  // column chunk innermost: the chunks of one tile run together on one XCD and share
  // its L2 lines (a node's columns are contiguous; a 128-byte line spans two chunks)
  int q = lb;
  const int c0 = (q % nch) * KC; q /= nch;
  const int txi = q % ntx; q /= ntx;
  const int tyi = q % nty; q /= nty;
  const int zc = q;
  const int tx0 = txi * TX, ty0 = tyi * TY;
  const int zlen = (m + nzc - 1) / nzc;
  const int z0 = zc * zlen;
  const int z1 = (z0 + zlen < m) ? z0 + zlen : m;
  const int tid = threadIdx.x;
  const int qv = tid % NQ;                   // column vector within the chunk
  const int node = tid / NQ;
  const int lx = node % TX, ly = node / TX;
  const int gx = tx0 + lx, gy = ty0 + ly;
  const int colv = c0 + qv * VW;             // first column of this thread
  const bool nodeok = (gx < m) && (gy < m);
  const T* __restrict__ X = (const T*)a.x;

  // halo plane: (TX+2)(TY+2) nodes x NQ vectors; thread owns entries tid and tid + kThreadsV.
  // Loads are branch-free: entries outside the domain (or the column range) read a zero
  // vector, so loaded registers stay in flight until they are stashed.
  constexpr int HV = (TX + 2) * (TY + 2) * NQ;
  static_assert(HV <= 2 * kThreadsV, "two halo entries per thread");
  const V* __restrict__ zerov = (const V*)a.zero;
  // per-thread halo entry geometry (independent of z)
  int hoff[2];
  bool hin[2];
  int hslot[2];
  int hnode[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    const int e = tid + u * kThreadsV;
    const int cq = e % NQ;
    const int hn = e / NQ;
    const int hx = hn % (TX + 2), hy = hn / (TX + 2);
    const int x = tx0 + hx - 1, y = ty0 + hy - 1;
    hin[u] = e < HV && x >= 0 && x < m && y >= 0 && y < m && c0 + cq * VW < k;
    hoff[u] = (y * m + x) * k + c0 + cq * VW;     // offset within a plane
    hslot[u] = (e < HV) ? e : -1;
    hnode[u] = hin[u] ? y * m + x : 0;            // node within a plane
  }
  const long long plane = (long long)m * m * k;
  auto ld1 = [&](int z, int u) -> V {
    const bool ok = hin[u] && z >= 0 && z < m;
    if constexpr (VEC) {
      const V* p = ok ? (const V*)(X + z * plane + hoff[u]) : zerov;
      return *p;
    } else {
      V v;
#pragma unroll
      for (int i = 0; i < VW; ++i) {
        const int cq = ((tid + u * kThreadsV) % NQ);
        const bool oki = ok && (c0 + cq * VW + i < k);
        const T* p = oki ? X + z * plane + hoff[u] + i : (const T*)zerov;
        vset<T, VW>(v, i, (double)*p);
      }
      return v;
    }
  };
  // the ring is indexed from the shared array itself (not through a table of pointers), so the
  // stash is an LDS store, not a generic store that would also wait on the global loads in flight
  constexpr int kPlaneV = (BY + 2) * (BX + 2) * NQ;
  auto st1 = [&](int slot, int u, const V& v) {
    if (hslot[u] >= 0) (&sm.xs[0][0][0][0])[slot * kPlaneV + hslot[u]] = v;
  };
  // kappa form: the tile's (BX+1) x (BY+1) cells of a layer are staged in an LDS ring beside the
  // planes (layer L in the slot of plane L), one cell per thread, loaded a step ahead with the
  // plane, so no step waits on a load that it issued itself
  constexpr bool kKapL = !CONSTK && !ASM;
  constexpr int kCells = (BX + 1) * (BY + 1);
  static_assert(kCells <= kThreadsV, "one cell per thread");
  __shared__ double ksm[kKapL ? kSlots * kCells : 1];
  auto kld = [&](int L) -> double {
    if constexpr (kKapL) {
      const int ex = tx0 + tid % (BX + 1), ey = ty0 + tid / (BX + 1);
      const bool ok = tid < kCells && ex < n && ey < n && L >= 0 && L < n;
      const double* p = ok ? a.kappa + ((long long)L * n + ey) * n + ex : (const double*)a.zero;
      return *p;
    } else {
      return 0.0;
    }
  };
  auto kst = [&](int slot, double v) {
    if (kKapL && tid < kCells) ksm[slot * kCells + tid] = v;
  };
  // EPI_SWEEP2V: the staged planes hold x1 = omega D^{-1} b; the diagonal is loaded with the plane
  // (kept in flight beside it) and applied when the plane is stashed
  constexpr bool kFirst2 = (EPI == EPI_SWEEP2V || EPI == EPI_RESID1V);
  const long long nplane = (long long)m * m;
  auto ldd = [&](int z, int u) -> double {
    if constexpr (kFirst2) {
      const bool ok = hin[u] && z >= 0 && z < m;
      return ok ? a.dinv[z * nplane + hnode[u]] : 0.0;
    } else {
      return 0.0;
    }
  };
  auto st1s = [&](int slot, int u, const V& v, double d) {
    if constexpr (kFirst2) {
      const double w = a.omega * d;
      V r;
#pragma unroll
      for (int i = 0; i < VW; ++i) vset<T, VW>(r, i, w * vget<T, VW>(v, i));
      st1(slot, u, r);
    } else {
      st1(slot, u, v);
    }
  };
  const long long cbase = ((long long)gy * m + gx) * k + colv;
  constexpr bool kSweep = (EPI == EPI_SWEEP || EPI == EPI_SWEEPDOT || EPI == EPI_SWEEP2V);
  constexpr bool kSums1 = (EPI == EPI_AMDOT || EPI == EPI_SWEEPDOT);   // one column sum
  // EPI_SWEEP2V needs no b: its staged x1 = omega D^{-1} b already holds it (see its epilogue)
  constexpr bool kLoadB = (EPI == EPI_RESID || EPI == EPI_SWEEP || EPI == EPI_SWEEPDOT);
  const bool bneed = kLoadB && nodeok && colv < k;
  auto bload = [&](int z) -> V {
    const bool ok = bneed && z < z1;
    const T* B = (const T*)a.b;
    if constexpr (VEC) {
      const V* p = ok ? (const V*)(B + z * plane + cbase) : zerov;
      return *p;
    } else {
      V v;
#pragma unroll
      for (int i = 0; i < VW; ++i) {
        const bool oki = ok && colv + i < k;
        const T* p = oki ? B + z * plane + cbase + i : (const T*)zerov;
        vset<T, VW>(v, i, (double)*p);
      }
      return v;
    }
  };
  auto stvec = [&](T* base, long long off, const V& v, bool ok) {
    if constexpr (VEC) {
      *(ok ? (V*)(base + off) : (V*)fine3_sink) = v;
    } else {
#pragma unroll
      for (int i = 0; i < VW; ++i)
        *((ok && colv + i < k) ? base + off + i : (T*)fine3_sink) = (T)vget<T, VW>(v, i);
    }
  };
  const double h = a.h;
  const double k0 = 1.0 / h, k1 = -1.0 / h, m0 = 2.0 * h / 6.0, m1 = h / 6.0;
  const double mc = h / 6.0, mc3 = mc * mc * mc;
  // EPI_AM writes both A x and M x; EPI_A and EPI_M one of them
  constexpr bool needA = (EPI != EPI_M);
  constexpr bool needM = (EPI == EPI_EIGRES) || (EPI == EPI_AM) || (EPI == EPI_M);

  // prologue: planes z0-1, z0, z0+1 into slots 0, 1, 2 (kappa layers z0, z0+1, z0+2 into slots
  // 1, 2, 3); b(z0), plane z0+2 and kappa layer z0+3 in flight
  {
#pragma unroll
    for (int p = 0; p < 3; ++p) {
      const V t0 = ld1(z0 - 1 + p, 0), t1 = ld1(z0 - 1 + p, 1);
      const double e0 = ldd(z0 - 1 + p, 0), e1 = ldd(z0 - 1 + p, 1);
      st1s(p, 0, t0, e0);
      st1s(p, 1, t1, e1);
    }
  }
  V bA = bload(z0), bB = bA;
  V pA0 = ld1(z0 + 2, 0), pA1 = ld1(z0 + 2, 1);
  V pB0 = pA0, pB1 = pA1;
  double dA[2] = {ldd(z0 + 2, 0), ldd(z0 + 2, 1)};
  double dB[2] = {dA[0], dA[1]};
  if (kKapL) {
    const double l0 = kld(z0), l1 = kld(z0 + 1), l2 = kld(z0 + 2);
    kst(1, l0);
    kst(2, l1);
    kst(3, l2);
  }
  double kA = kld(z0 + 3), kB = kA;
  __syncthreads();
  // kappa form: the node's cells in layers p (kl) and p+1 (ku) of the plane p being added
  double kl[2][2] = {{0.0, 0.0}, {0.0, 0.0}}, ku[2][2] = {{0.0, 0.0}, {0.0, 0.0}};
  auto kread = [&](int slot, double (&c)[2][2]) {
#pragma unroll
    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
      for (int cx = 0; cx < 2; ++cx) c[cy][cx] = ksm[slot * kCells + (ly + cy) * (BX + 1) + lx + cx];
  };
  double acc0[VW], acc1[VW], acc2[VW];
#pragma unroll
  for (int i = 0; i < VW; ++i) acc0[i] = acc1[i] = acc2[i] = 0.0;
  double lamc[VW];
#pragma unroll
  for (int i = 0; i < VW; ++i) lamc[i] = (EPI == EPI_EIGRES && colv + i < k) ? a.lam[colv + i] : 0.0;

  // Output plane z: planes z-1, z, z+1 sit in slots sb, sb+1, sb+2 (mod 4) with sb = (z - z0) & 3;
  // PS0/PS1 hold plane z+2 (in flight since the previous step) and are stashed into slot sb+3;
  // PL0/PL1 receive plane z+3; BV is b(z) and BN receives b(z+1).  kappa runs a step further
  // ahead (layer L in the slot of plane L): layer z+2 is read, KS (layer z+3) stashed into slot
  // sb, KL receives layer z+4.
#define PASE_STEP(z, PL0, PL1, PS0, PS1, BV, BN, DL, DS, KL, KS)                                       \
  {                                                                                                     \
    const int sb = ((z) - z0) & 3;                                                                      \
    if (kLoadB) BN = bload((z) + 1);                                                                    \
    PL0 = ld1((z) + 3, 0);                                                                              \
    PL1 = ld1((z) + 3, 1);                                                                              \
    if (kFirst2) {                                                                                      \
      DL[0] = ldd((z) + 3, 0);                                                                          \
      DL[1] = ldd((z) + 3, 1);                                                                          \
    }                                                                                                   \
    if (kKapL) {                                                                                        \
      KL = kld((z) + 4);                                                                                \
      _Pragma("unroll") for (int cy = 0; cy < 2; ++cy) _Pragma("unroll") for (int cx = 0; cx < 2; ++cx) \
        kl[cy][cx] = ku[cy][cx];                                                                        \
      kread((sb + 3) & 3, ku);                                                                          \
    }                                                                                                   \
    compute_plane((z), sb, BV, nodeok && colv < k && (z) < z1);                                         \
    st1s((sb + 3) & 3, 0, PS0, DS[0]);                                                                  \
    st1s((sb + 3) & 3, 1, PS1, DS[1]);                                                                  \
    kst(sb, KS);                                                                                        \
    __syncthreads();                                                                                    \
  }
  // Constant coefficient (residual, sweep and eigen-residual epilogues): reuse along z.  A plane
  // is read once (9 taps) when it becomes the
  // newest, and each tap goes into the running sums of the three outputs it touches (its
  // coefficient depends only on whether the z offset is zero): ra/rm[0] = output z (completed by
  // plane z+1), [1] = output z+1, [2] = output z+2.  cen[0] is x at output z, cen[1] at z+1.
  double ra[3][VW], rm[3][VW], cen[2][VW];
#pragma unroll
  for (int i = 0; i < VW; ++i) {
    ra[0][i] = ra[1][i] = ra[2][i] = 0.0;
    rm[0][i] = rm[1][i] = rm[2][i] = 0.0;
    cen[0][i] = cen[1][i] = 0.0;
  }
  // MODE 0: plane z0-1 (only output z0, offset -1); 1: plane z0 (outputs z0 and z0+1, centre of
  // z0); 2: plane z+1 in step z (outputs z, z+1, z+2, centre of z+1)
  auto plane9 = [&](int slot, int mode) {
#define PASE_TAP9(OX, OY)                                                                            \
  {                                                                                                  \
    const V v = sm.xs[slot][ly + 1 + (OY)][lx + 1 + (OX)][qv];                                       \
    constexpr double sxy = (double)(((OX) == 0 ? 2 : 1) * ((OY) == 0 ? 2 : 1));                      \
    const double cz = needA ? kpat<OX, OY, 0>(k0, k1, m0, m1) * (2.0 * sxy) : 0.0;                   \
    const double cn = needA ? kpat<OX, OY, 1>(k0, k1, m0, m1) * sxy : 0.0;                           \
    constexpr double mxy = (double)(((OX) == 0 ? 4 : 1) * ((OY) == 0 ? 4 : 1));                      \
    const double mz = mxy * 4.0 * mc3, mn = mxy * mc3;                                               \
    _Pragma("unroll") for (int i = 0; i < VW; ++i) {                                                 \
      const double xv = vget<T, VW>(v, i);                                                           \
      if (mode == 0) {                                                                               \
        if (needA) ra[0][i] = fma(cn, xv, ra[0][i]);                                                 \
        if (needM) rm[0][i] = fma(mn, xv, rm[0][i]);                                                 \
      } else if (mode == 1) {                                                                        \
        if ((OX) == 0 && (OY) == 0) cen[0][i] = xv;                                                  \
        if (needA) { ra[0][i] = fma(cz, xv, ra[0][i]); ra[1][i] = fma(cn, xv, ra[1][i]); }           \
        if (needM) { rm[0][i] = fma(mz, xv, rm[0][i]); rm[1][i] = fma(mn, xv, rm[1][i]); }           \
      } else {                                                                                       \
        if ((OX) == 0 && (OY) == 0) cen[1][i] = xv;                                                  \
        if (needA) {                                                                                 \
          ra[0][i] = fma(cn, xv, ra[0][i]);                                                          \
          ra[1][i] = fma(cz, xv, ra[1][i]);                                                          \
          ra[2][i] = fma(cn, xv, ra[2][i]);                                                          \
        }                                                                                            \
        if (needM) {                                                                                 \
          rm[0][i] = fma(mn, xv, rm[0][i]);                                                          \
          rm[1][i] = fma(mz, xv, rm[1][i]);                                                          \
          rm[2][i] = fma(mn, xv, rm[2][i]);                                                          \
        }                                                                                            \
      }                                                                                              \
    }                                                                                                \
  }
    PASE_TAP9(-1, -1) PASE_TAP9(0, -1) PASE_TAP9(1, -1)
    PASE_TAP9(-1, 0)  PASE_TAP9(0, 0)  PASE_TAP9(1, 0)
    PASE_TAP9(-1, 1)  PASE_TAP9(0, 1)  PASE_TAP9(1, 1)
#undef PASE_TAP9
  };
  // kappa form, the same running sums.  The Q1 stiffness of a cube of side h couples a node with
  // itself by h/3, with a neighbour across a face by 0, across an edge or a corner by -h/12 (times
  // the kappa of the cells they share), so A x = (h/3) K8 x_i - (h/12) sum_j S_ij x_j over the 20
  // edge and corner neighbours, with K8 the node's 8 cells and S_ij the kappa of the cells shared
  // with j; ra holds the sums of S_ij x_j, rm the M sums in units of (h/6)^3, dco the K8 of the
  // outputs z and z+1.  A tap (ox, oy) of plane p meets output p-1 in its upper layer (p, kl),
  // output p in both, output p+1 in its lower layer (p+1, ku); in plane p only the 4 corner taps
  // are edge neighbours of output p.  M: the plane's 9 taps weighted (4 or 1 per axis) once, then
  // 1, 4, 1 for the outputs p-1, p, p+1.
  double dco[2] = {0.0, 0.0};
  auto plane9k = [&](int slot, int mode) {
    double pm[VW];
#pragma unroll
    for (int i = 0; i < VW; ++i) pm[i] = 0.0;
#define PASE_TAPK(OX, OY)                                                                            \
  {                                                                                                  \
    const V v = sm.xs[slot][ly + 1 + (OY)][lx + 1 + (OX)][qv];                                       \
    constexpr bool kCen = (OX) == 0 && (OY) == 0;                                                    \
    constexpr bool kCorner = (OX) != 0 && (OY) != 0;                                                 \
    constexpr double mxy = (double)(((OX) == 0 ? 4 : 1) * ((OY) == 0 ? 4 : 1));                      \
    const double su = cell_sum<OX, OY>(ku);                                                          \
    const double sl = (mode == 0) ? 0.0 : cell_sum<OX, OY>(kl);                                      \
    const double slu = sl + su;                                                                      \
    _Pragma("unroll") for (int i = 0; i < VW; ++i) {                                                 \
      const double xv = vget<T, VW>(v, i);                                                           \
      if (needM) pm[i] = fma(mxy, xv, pm[i]);                                                        \
      if constexpr (kCen) {                                                                          \
        if (mode == 1) cen[0][i] = xv;                                                               \
        else if (mode == 2) cen[1][i] = xv;                                                          \
      } else if (mode == 0) {                                                                        \
        ra[0][i] = fma(su, xv, ra[0][i]);                                                            \
      } else if (mode == 1) {                                                                        \
        if (kCorner) ra[0][i] = fma(slu, xv, ra[0][i]);                                              \
        ra[1][i] = fma(su, xv, ra[1][i]);                                                            \
      } else {                                                                                       \
        ra[0][i] = fma(sl, xv, ra[0][i]);                                                            \
        if (kCorner) ra[1][i] = fma(slu, xv, ra[1][i]);                                              \
        ra[2][i] = fma(su, xv, ra[2][i]);                                                            \
      }                                                                                              \
    }                                                                                                \
  }
    PASE_TAPK(-1, -1) PASE_TAPK(0, -1) PASE_TAPK(1, -1)
    PASE_TAPK(-1, 0)  PASE_TAPK(0, 0)  PASE_TAPK(1, 0)
    PASE_TAPK(-1, 1)  PASE_TAPK(0, 1)  PASE_TAPK(1, 1)
#undef PASE_TAPK
    if (needM) {
#pragma unroll
      for (int i = 0; i < VW; ++i) {
        if (mode == 0) {
          rm[0][i] += pm[i];
        } else if (mode == 1) {
          rm[0][i] = fma(4.0, pm[i], rm[0][i]);
          rm[1][i] += pm[i];
        } else {
          rm[0][i] += pm[i];
          rm[1][i] = fma(4.0, pm[i], rm[1][i]);
          rm[2][i] += pm[i];
        }
      }
    }
    if (mode >= 1) dco[mode - 1] = cell_sum<0, 0>(kl) + cell_sum<0, 0>(ku);
  };
  // every lane computes (its LDS reads stay inside the tile and its halo); ok says whether the
  // lane owns an output: the others store to the sink and add nothing to the column sums
  auto compute_plane = [&](int z, int sb, const V& bv, bool ok) {
    double ax[VW], mx[VW], center[VW];
#pragma unroll
    for (int i = 0; i < VW; ++i) ax[i] = mx[i] = center[i] = 0.0;
    double dcoef = 1.0;
    double cf[ASM ? 27 : 1];
    if constexpr (ASM) {
      if (needA) {
        const long long row = ok ? ((long long)z * m + gy) * m + gx : 0;
        const double* __restrict__ cp = a.coef + row * 27;
#pragma unroll
        for (int o = 0; o < 27; ++o) cf[o] = cp[o];
      }
    }
    if constexpr (CONSTK && EPI != EPI_AM) {
      plane9((sb + 2) & 3, 2);
#pragma unroll
      for (int i = 0; i < VW; ++i) {
        ax[i] = ra[0][i];
        mx[i] = rm[0][i];
        center[i] = cen[0][i];
        ra[0][i] = ra[1][i];
        ra[1][i] = ra[2][i];
        ra[2][i] = 0.0;
        rm[0][i] = rm[1][i];
        rm[1][i] = rm[2][i];
        rm[2][i] = 0.0;
        cen[0][i] = cen[1][i];
      }
      dcoef = kpat<0, 0, 0>(k0, k1, m0, m1) * 8.0;
    } else if constexpr (kKapL) {
      plane9k((sb + 2) & 3, 2);
      const double hd = h / 3.0, ho = -h / 12.0;
      dcoef = hd * dco[0];
#pragma unroll
      for (int i = 0; i < VW; ++i) {
        ax[i] = fma(dcoef, cen[0][i], ho * ra[0][i]);
        mx[i] = mc3 * rm[0][i];
        center[i] = cen[0][i];
        ra[0][i] = ra[1][i];
        ra[1][i] = ra[2][i];
        ra[2][i] = 0.0;
        rm[0][i] = rm[1][i];
        rm[1][i] = rm[2][i];
        rm[2][i] = 0.0;
        cen[0][i] = cen[1][i];
      }
      dco[0] = dco[1];
    } else {
#define PASE_TAP(OX, OY, OZ)                                                                       \
  {                                                                                                \
    const V v = sm.xs[(sb + 1 + (OZ)) & 3][ly + 1 + (OY)][lx + 1 + (OX)][qv];                      \
    double coef = 0.0, mp = 0.0;                                                                   \
    if (needA) {                                                                                   \
      if constexpr (ASM) {                                                                         \
        coef = cf[((OX) + 1) + 3 * ((OY) + 1) + 9 * ((OZ) + 1)];                                   \
      } else {                                                                                     \
        const double s = (double)(((OX) == 0 ? 2 : 1) * ((OY) == 0 ? 2 : 1) * ((OZ) == 0 ? 2 : 1)); \
        coef = kpat<OX, OY, OZ>(k0, k1, m0, m1) * s;                                               \
      }                                                                                            \
      if ((OX) == 0 && (OY) == 0 && (OZ) == 0) dcoef = coef;                                       \
    }                                                                                              \
    if (needM) mp = (double)(((OX) == 0 ? 4 : 1) * ((OY) == 0 ? 4 : 1) * ((OZ) == 0 ? 4 : 1)) * mc3; \
    _Pragma("unroll") for (int i = 0; i < VW; ++i) {                                               \
      const double xv = vget<T, VW>(v, i);                                                             \
      if ((OX) == 0 && (OY) == 0 && (OZ) == 0) center[i] = xv;                                     \
      if (needA) ax[i] = fma(coef, xv, ax[i]);                                                     \
      if (needM) mx[i] = fma(mp, xv, mx[i]);                                                       \
    }                                                                                              \
  }
    PASE_TAP(-1, -1, -1) PASE_TAP(0, -1, -1) PASE_TAP(1, -1, -1)
    PASE_TAP(-1, 0, -1)  PASE_TAP(0, 0, -1)  PASE_TAP(1, 0, -1)
    PASE_TAP(-1, 1, -1)  PASE_TAP(0, 1, -1)  PASE_TAP(1, 1, -1)
    PASE_TAP(-1, -1, 0)  PASE_TAP(0, -1, 0)  PASE_TAP(1, -1, 0)
    PASE_TAP(-1, 0, 0)   PASE_TAP(0, 0, 0)   PASE_TAP(1, 0, 0)
    PASE_TAP(-1, 1, 0)   PASE_TAP(0, 1, 0)   PASE_TAP(1, 1, 0)
    PASE_TAP(-1, -1, 1)  PASE_TAP(0, -1, 1)  PASE_TAP(1, -1, 1)
    PASE_TAP(-1, 0, 1)   PASE_TAP(0, 0, 1)   PASE_TAP(1, 0, 1)
    PASE_TAP(-1, 1, 1)   PASE_TAP(0, 1, 1)   PASE_TAP(1, 1, 1)
#undef PASE_TAP
    }
    const long long off = (long long)z * plane + cbase;
    V o1, o2;
    if (EPI == EPI_AM) {
#pragma unroll
      for (int i = 0; i < VW; ++i) { vset<T, VW>(o1, i, ax[i]); vset<T, VW>(o2, i, mx[i]); }
      stvec((T*)a.out1, off, o1, ok);
      stvec((T*)a.out2, off, o2, ok);
    } else if (EPI == EPI_A) {
#pragma unroll
      for (int i = 0; i < VW; ++i) vset<T, VW>(o1, i, ax[i]);
      stvec((T*)a.out1, off, o1, ok);
    } else if (EPI == EPI_M) {
#pragma unroll
      for (int i = 0; i < VW; ++i) vset<T, VW>(o2, i, mx[i]);
      stvec((T*)a.out2, off, o2, ok);
    } else if (EPI == EPI_RESID) {
#pragma unroll
      for (int i = 0; i < VW; ++i) vset<T, VW>(o1, i, vget<T, VW>(bv, i) - ax[i]);
      stvec((T*)a.out1, off, o1, ok);
    } else if (EPI == EPI_SWEEP2) {
      // the staged planes hold b: x1 = c b, A x1 = c (A b), out = x1 + c (b - A x1)
      const double c = a.omega / dcoef;
#pragma unroll
      for (int i = 0; i < VW; ++i) vset<T, VW>(o1, i, c * center[i] + c * (center[i] - c * ax[i]));
      stvec((T*)a.out1, off, o1, ok);
    } else if (EPI == EPI_RESID1V) {
      // b - A x1 with b = x1 a_ii / omega at the node (x1 = omega D^{-1} b as staged)
      const double c = dcoef / a.omega;
#pragma unroll
      for (int i = 0; i < VW; ++i) vset<T, VW>(o1, i, fma(c, center[i], -ax[i]));
      stvec((T*)a.out1, off, o1, ok);
    } else if (EPI == EPI_SWEEP2V) {
      // second sweep from x1 = omega D^{-1} b: x1 + omega D^{-1} (b - A x1) = 2 x1 - omega D^{-1} A x1
      const double wd = a.omega / dcoef;
#pragma unroll
      for (int i = 0; i < VW; ++i) vset<T, VW>(o1, i, fma(-wd, ax[i], 2.0 * center[i]));
      stvec((T*)a.out1, off, o1, ok);
    } else if (kSweep) {
      const double wd = a.omega / dcoef;
#pragma unroll
      for (int i = 0; i < VW; ++i) vset<T, VW>(o1, i, center[i] + wd * (vget<T, VW>(bv, i) - ax[i]));
      stvec((T*)a.out1, off, o1, ok);
      if (EPI == EPI_SWEEPDOT && ok) {
#pragma unroll
        for (int i = 0; i < VW; ++i) acc0[i] = fma(vget<T, VW>(bv, i), vget<T, VW>(o1, i), acc0[i]);
      }
    } else if (EPI == EPI_AMDOT) {
#pragma unroll
      for (int i = 0; i < VW; ++i) vset<T, VW>(o1, i, ax[i]);
      stvec((T*)a.out1, off, o1, ok);
      if (ok) {
#pragma unroll
        for (int i = 0; i < VW; ++i) acc0[i] = fma(center[i], vget<T, VW>(o1, i), acc0[i]);
      }
    } else {
#pragma unroll
      for (int i = 0; i < VW; ++i) {
        const double r = lamc[i] * mx[i] - ax[i];
        vset<T, VW>(o1, i, r);
        if (ok) {
          acc0[i] = fma(r, r, acc0[i]);
          acc1[i] = fma(mx[i], mx[i], acc1[i]);
          acc2[i] = fma(center[i], mx[i], acc2[i]);
        }
      }
      stvec((T*)a.out1, off, o1, ok);
    }
  };
  if (CONSTK && EPI != EPI_AM && nodeok && colv < k) {
    plane9(0, 0);       // plane z0 - 1
    plane9(1, 1);       // plane z0
  }
  if (kKapL) {
    kread(1, ku);       // layer z0
    plane9k(0, 0);      // plane z0 - 1
#pragma unroll
    for (int cy = 0; cy < 2; ++cy)
#pragma unroll
      for (int cx = 0; cx < 2; ++cx) kl[cy][cx] = ku[cy][cx];
    kread(2, ku);       // layer z0 + 1
    plane9k(1, 1);      // plane z0
  }
  // two steps per trip, the in-flight registers alternating; the second step of the last trip of
  // an odd run lies past z1 and only loads, and stores to the sink, so every trip is the same code
  // and the waits for the loads in flight stay exact
  for (int z = z0; z < z1; z += 2) {
    PASE_STEP(z, pB0, pB1, pA0, pA1, bA, bB, dB, dA, kB, kA)
    PASE_STEP(z + 1, pA0, pA1, pB0, pB1, bB, bA, dA, dB, kA, kB)
  }
#undef PASE_STEP
  if (kSums1) {
    // one column sum per column: partial[spatial block][column]
    __syncthreads();
#pragma unroll
    for (int i = 0; i < VW; ++i) sm.red[0][tid * VW + i] = acc0[i];
    __syncthreads();
    if (tid < KC && c0 + tid < k) {
      const int tq = tid / VW, ti = tid % VW;
      double s0 = 0.0;
      for (int nd = 0; nd < TX * TY; ++nd) s0 += sm.red[0][(nd * NQ + tq) * VW + ti];
      const int sbk = (zc * nty + tyi) * ntx + txi;
      a.partial[(size_t)sbk * k + c0 + tid] = s0;
    }
  }
  if (EPI == EPI_EIGRES) {
    __syncthreads();
#pragma unroll
    for (int i = 0; i < VW; ++i) {
      sm.red[0][tid * VW + i] = acc0[i];
      sm.red[1][tid * VW + i] = acc1[i];
      sm.red[2][tid * VW + i] = acc2[i];
    }
    __syncthreads();
    // thread t < KC owns column c0 + t: entries (node, qv = t / VW, i = t % VW)
    if (tid < KC && c0 + tid < k) {
      const int tq = tid / VW, ti = tid % VW;
      double s0 = 0.0, s1 = 0.0, s2 = 0.0;
      for (int nd = 0; nd < TX * TY; ++nd) {
        const int src = (nd * NQ + tq) * VW + ti;
        s0 += sm.red[0][src];
        s1 += sm.red[1][src];
        s2 += sm.red[2][src];
      }
      const int sbk = (zc * nty + tyi) * ntx + txi;
      double* p = a.partial + (size_t)sbk * 3 * k;
      p[c0 + tid] = s0;
      p[k + c0 + tid] = s1;
      p[2 * k + c0 + tid] = s2;
    }
  }
}

template <typename T, int VW, int EPI, bool CONSTK, bool VEC, bool ASM>
void launchv_tile(const Fine3Args& a, hipStream_t s) {
  auto go = [&](auto bq) {
    constexpr int BX = 8, NQ = decltype(bq)::value, BY = (NQ == 8) ? 4 : 8;
    constexpr int KC = NQ * VW;
    const int ntx = (a.m + BX - 1) / BX, nty = (a.m + BY - 1) / BY, nch = (a.k + KC - 1) / KC;
    const int total = ntx * nty * a.nzc * nch;
    const int blocks = ((total + 7) / 8) * 8;
    fine3v_kernel<T, VW, EPI, CONSTK, VEC, BX, BY, NQ, ASM><<<blocks, BX * BY * NQ, 0, s>>>(a);
  };
  // 8 x 4 nodes with 8 threads per node when a block's columns are whole 128-byte lines of the
  // node rows (k a multiple of 8 VW): its halo loads are then full lines, which measured 16 % faster
  // than 8 x 8 nodes with 4 threads (half lines, the other half read by the next column chunk)
  if (fine3_wide_tile(a.k, sizeof(T) == 4)) {
    go(std::integral_constant<int, 8>());
    return;
  }
  // else 8 x 8 nodes, column chunks of 5 vectors when that wastes fewer padded columns than chunks
  // of 4 (not for the A+M and eigen-residual epilogues, whose register use makes the larger block
  // slower)
  const int w4 = ((a.k + 4 * VW - 1) / (4 * VW)) * 4 * VW - a.k;
  const int w5 = ((a.k + 5 * VW - 1) / (5 * VW)) * 5 * VW - a.k;
  if constexpr (EPI != EPI_AM && EPI != EPI_EIGRES) {
    if (w5 < w4) {
      go(std::integral_constant<int, 5>());
      return;
    }
  }
  go(std::integral_constant<int, 4>());
}

template <typename T, int VW, int EPI>
void launchv_w(const Fine3Args& a, hipStream_t s) {
  const bool vec = (a.k % VW) == 0;
  // M does not depend on the coefficient: the constant-coefficient path
  if constexpr (EPI != EPI_M && EPI != EPI_SWEEP2) {
    if (a.coef) {
      if (vec) launchv_tile<T, VW, EPI, false, true, true>(a, s);
      else launchv_tile<T, VW, EPI, false, false, true>(a, s);
      return;
    }
  }
  if constexpr (EPI == EPI_SWEEP2V || EPI == EPI_RESID1V) {
    // variable coefficient only (the caller passes coef or kappa)
    if (vec) launchv_tile<T, VW, EPI, false, true, false>(a, s);
    else launchv_tile<T, VW, EPI, false, false, false>(a, s);
    return;
  }
  if (a.kappa && EPI != EPI_M) {
    if (vec) launchv_tile<T, VW, EPI, false, true, false>(a, s);
    else launchv_tile<T, VW, EPI, false, false, false>(a, s);
  } else {
    if (vec) launchv_tile<T, VW, EPI, true, true, false>(a, s);
    else launchv_tile<T, VW, EPI, true, false, false>(a, s);
  }
}

// double: double2 vectors; float: float4 when k is a multiple of 4, else float2
template <typename T, int EPI>
void launchv(const Fine3Args& a, hipStream_t s) {
  if constexpr (sizeof(T) == 8) {
    launchv_w<T, 2, EPI>(a, s);
  } else {
    if (a.k % 4 == 0) launchv_w<T, 4, EPI>(a, s);
    else launchv_w<T, 2, EPI>(a, s);
  }
}

}  // namespace

}  // namespace pase
