// Entry point without device allocation: ddps_residual_norms_noalloc.
//
// Same computation and kernels as ddps_residual_norms (r = f - A x and its
// norms for k <= 8 columns), with the reduction's partial sums in a fixed
// device array of this file instead of memory allocated by the call, for
// callers that must not allocate device memory.  The array, `scratch`, is a
// file-scope __device__ variable: every GPU the library runs on holds its own
// copy until the process ends.  Host code never passes `scratch` itself to a
// kernel (on the host the name is only a stand-in for the symbol); the device
// address of each GPU's copy is looked up once per device with
// hipGetSymbolAddress, with that device current, and that address is what the
// kernels receive.
#include <mutex>

#include "../../include/ddps.h"
#include "ddps_internal.h"

namespace {

using namespace ddps;

// [kVecGrid][kMaxRhs][4] partial sums, then [kMaxRhs][4] reduced values:
// 262,400 bytes.  Every entry a call reads was written earlier in the same
// call, so nothing needs clearing between calls.
constexpr size_t kPartDoubles = (size_t)kVecGrid * kMaxRhs * 4;
constexpr size_t kScratchDoubles = kPartDoubles + 4 * kMaxRhs;
static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
double* g_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch` (looked up on the
// first call on that device); nullptr on failure.
double* scratch_of_current_device(hipError_t* err) {
  int dev = -1;
  *err = hipGetDevice(&dev);
  if (*err != hipSuccess) return nullptr;
  if (dev < 0 || dev >= kMaxDevices) {
    *err = hipErrorInvalidDevice;
    return nullptr;
  }
  std::lock_guard<std::mutex> lock(g_mutex);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (*err != hipSuccess || !p) {
      if (*err == hipSuccess) *err = hipErrorInvalidSymbol;
      return nullptr;
    }
    g_ptr[dev] = (double*)p;
  }
  return g_ptr[dev];
}

}  // namespace

extern "C" int ddps_residual_norms_noalloc(int64_t n, int32_t k, const int64_t* row_ptr, const int32_t* col,
                                           const double* val, const double* X, int64_t ldx, const double* F,
                                           int64_t ldf, double* R, int64_t ldr, double* norms, void* stream) {
  // k beyond the array's capacity (kMaxRhs columns of partial sums) is refused
  if (n <= 0 || k < 1 || k > kMaxRhs || !row_ptr || !col || !val || !X || !F || !norms || ldx < n || ldf < n ||
      (R && ldr < n))
    return DDPS_E_ARG;
  hipError_t e = hipSuccess;
  double* base = scratch_of_current_device(&e);
  if (!base) return DDPS_E_HIP;
  hipStream_t s = (hipStream_t)stream;
  double* part = base;
  double* out = base + kPartDoubles;
  residual_norms_cols(n, k, row_ptr, col, val, X, ldx, F, ldf, R, ldr, part, out, s);
  e = hipGetLastError();
  if (e == hipSuccess) e = hipMemcpyAsync(norms, out, sizeof(double) * 4 * k, hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return DDPS_E_HIP;
  for (int j = 0; j < k; ++j) {
    norms[4 * j + 1] = std::sqrt(norms[4 * j + 1]);
    norms[4 * j + 3] = std::sqrt(norms[4 * j + 3]);
  }
  return DDPS_OK;
}
