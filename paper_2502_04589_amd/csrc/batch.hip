// Selection of the batch scheme (Sec. "Batch scheme for computing plenty of eigenpairs", eq.
// largest_component): of the nsel composite pairs nearest the shift, the k whose eigenvectors
// have the largest component in span(u_hat).  The driver is in pase.hip.
#include "internal.hpp"

namespace pase {
namespace {

constexpr int kSelMax = 256;

// Y (k x nsel row-major) holds the coordinates of the eigenvectors in an orthonormal basis of
// span(u_hat), so score_j = sum_i Y[i][j]^2.  The k largest scores (ties to the lower index) are
// written to sel in ascending index order, i.e. ascending eigenvalue.  A non-finite score sets
// *flag; sel still holds k valid indices.
__global__ __launch_bounds__(kSelMax) void batch_select_kernel(int k, int nsel, const double* __restrict__ Y,
                                                               int* __restrict__ sel, int* __restrict__ flag) {
  __shared__ double sc[kSelMax];
  __shared__ int keep[kSelMax];
  const int t = threadIdx.x;
  if (t < k) sel[t] = t;
  if (t < nsel) {
    double s = 0.0;
    for (int i = 0; i < k; ++i) {
      const double y = Y[(size_t)i * nsel + t];
      s = fma(y, y, s);
    }
    sc[t] = s;
    if (!isfinite(s)) *flag = 1;
  }
  __syncthreads();
  if (t < nsel) {
    int rank = 0;
    const double st = sc[t];
    for (int l = 0; l < nsel; ++l) rank += (sc[l] > st) || (sc[l] == st && l < t);
    keep[t] = rank < k;
  }
  __syncthreads();
  if (t < nsel && keep[t]) {
    int pos = 0;
    for (int l = 0; l < t; ++l) pos += keep[l];
    if (pos < k) sel[pos] = t;
  }
}

}  // namespace

int batch_select_max() { return kSelMax; }

void launch_batch_select(int k, int nsel, const double* Y, int* sel, int* flag, hipStream_t s) {
  batch_select_kernel<<<1, kSelMax, 0, s>>>(k, nsel, Y, sel, flag);
}

}  // namespace pase
