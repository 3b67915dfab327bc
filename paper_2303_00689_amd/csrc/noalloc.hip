// xlbomd_spectral_bounds_noalloc: the spectral bounds of xlbomd_spectral_bounds
// for callers that cannot allocate device memory.  No handle; the scratch of
// the kernels (Lanczos vectors, the product vector, per-row Gershgorin
// intervals, the reduced scalars) lives in one file-scope device array of a
// fixed size, shared by every call on a device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "../../include/xlbomd.h"
#include "common.h"
#include "small_eig.h"

namespace {

constexpr int NA_K = 32;                  // Lanczos steps, as xlbomd_spectral_bounds
constexpr int NA_MAX_N = XLBOMD_SPECTRAL_BOUNDS_NOALLOC_MAX_N;
// layout in doubles: Q ((K + 1) x n) | w (n) | row intervals (2 n) | Gershgorin (2) | alpha, beta (2 K)
constexpr size_t NA_OFF_W = (size_t)(NA_K + 1) * NA_MAX_N;
constexpr size_t NA_OFF_ROWS = NA_OFF_W + NA_MAX_N;
constexpr size_t NA_OFF_G = NA_OFF_ROWS + 2 * (size_t)NA_MAX_N;
constexpr size_t NA_OFF_AB = NA_OFF_G + 2;
constexpr size_t NA_DOUBLES = NA_OFF_AB + 2 * NA_K;

// The array's name is a host-side stand-in in host code: kernels get the
// device address from hipGetSymbolAddress (per device), never the name.
static __device__ __align__(256) double scratch[NA_DOUBLES];

constexpr int NA_MAX_DEV = 64;
std::mutex na_mutex;
double *na_ptr[NA_MAX_DEV] = {};

// device address of this device's copy of the scratch array (looked up once
// per device, with that device current)
hipError_t scratch_ptr(double **out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= NA_MAX_DEV) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(na_mutex);
  if (!na_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    na_ptr[dev] = static_cast<double *>(p);
  }
  *out = na_ptr[dev];
  return hipSuccess;
}

}  // namespace

extern "C" xlbomd_status xlbomd_spectral_bounds_noalloc(const double *F, int n, void *stream, double *lohi) {
  if (!F || !lohi || n < 1 || n > NA_MAX_N) return XLBOMD_E_ARG;
  double *base = nullptr;
  if (scratch_ptr(&base) != hipSuccess) return XLBOMD_E_HIP;
  hipStream_t s = static_cast<hipStream_t>(stream);
  double *Q = base, *w = base + NA_OFF_W, *rows = base + NA_OFF_ROWS, *gdev = base + NA_OFF_G,
         *ab = base + NA_OFF_AB;
  // every value read below is written by this call first: the start vector,
  // each Lanczos vector, w, the row intervals and the reduced scalars
  xl::gershgorin(n, F, gdev, rows, s);
  xl::lanczos_start(n, Q, s);
  const int K = std::min(NA_K, n);
  xl::lanczos(n, K, F, Q, w, ab, s);
  if (hipGetLastError() != hipSuccess) return XLBOMD_E_HIP;
  double g[2], abh[2 * NA_K];
  if (hipMemcpyAsync(g, gdev, sizeof(g), hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipMemcpyAsync(abh, ab, sizeof(double) * 2 * K, hipMemcpyDeviceToHost, s) != hipSuccess ||
      hipStreamSynchronize(s) != hipSuccess)
    return XLBOMD_E_HIP;
  if (!xl::bounds_from_lanczos(g, abh, K, n, lohi)) return XLBOMD_E_NONFINITE;
  return XLBOMD_OK;
}
