// Handle-free Gram product G = X^T Y that allocates nothing: the per-block
// partial sums of the MFMA Gram live in a fixed device array of the library
// instead of a caller workspace, for callers that cannot allocate device memory
// (code under HIP graph capture, tight serving loops).
#include <mutex>
#include <string>

#include "internal.hpp"

using namespace pase;

namespace {

constexpr size_t kScratchBytes = (size_t)16 << 20;   // per device, held until the process ends
constexpr int kMaxK = 128;
constexpr int kMaxDevices = 64;

// Partial sums of the Gram kernel: every block writes all k x k entries of its own slot, so
// nothing needs clearing between calls.
static __device__ __align__(256) double scratch[kScratchBytes / sizeof(double)];

std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};          // device address of `scratch` on each device

// the message goes where pase_last_error(NULL) reads it
pase_status fail(pase_status s, const std::string& msg) {
  set_last_error(msg);
  return s;
}

// Address of this device's copy of the scratch array, looked up once per device with that
// device current (each device holds its own copy at its own address).
pase_status scratch_ptr(double** out) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return fail(PASE_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) return fail(PASE_E_UNSUPPORTED, "device index beyond the supported range");
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(PASE_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[dev] = p;
  }
  *out = (double*)g_scratch[dev];
  return PASE_OK;
}

}  // namespace

extern "C" {

pase_status pase_gram_noalloc(long long N, int k, const double* X, const double* Y, double* G, void* stream) {
  if (!X || !Y || !G) return fail(PASE_E_ARG, "X, Y and G must be non-null device pointers");
  if (N < 1) return fail(PASE_E_ARG, "N must be positive");
  if (k < 1 || k > kMaxK) return fail(PASE_E_ARG, "k must be in [1, 128]");
  double* part = nullptr;
  const pase_status st = scratch_ptr(&part);
  if (st != PASE_OK) return st;
  // as many row blocks as the handle path takes, capped by what the scratch array holds
  const long long cap = (long long)(kScratchBytes / (sizeof(double) * (size_t)k * (size_t)k));
  int tiles = gram_tiles(N, k);
  if (tiles > cap) tiles = (int)cap;
  hipStream_t s = (hipStream_t)stream;
  launch_gram(N, k, X, Y, part, tiles, G, s);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return fail(PASE_E_HIP, std::string("Gram launch: ") + hipGetErrorString(e));
  return PASE_OK;
}

}  // extern "C"
