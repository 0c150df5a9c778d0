// gmresir_errors_noalloc: the error report of gmresir_errors (normwise and
// componentwise backward errors from a double-double residual, forward
// error) without a handle and without allocating: every scratch vector and
// reduction word lives in one file-scope device array per GPU, and the three
// results are written to device memory in stream order (no host round trip,
// so the call can sit inside a captured HIP graph).
//
// `scratch` is a device symbol: in host code its name is only a stand-in, so
// the host takes its device address with hipGetSymbolAddress once per device
// (on the first call made with that device current) and passes that address
// to the kernels.  All calls on one device share the array: calls that
// overlap on one device (other streams, other threads) race on it.
#include <hip/hip_runtime.h>

#include <array>
#include <cstdint>
#include <mutex>

#include "../../include/gmresir.h"
#include "kernels.h"

namespace {

// largest order accepted (the library's own limit)
constexpr int64_t kMaxN = 16384;
// layout (doubles): b copy [kMaxN], x copy [kMaxN], r / x_true copy [kMaxN],
// then 8 reduction words
constexpr size_t kScratchDoubles = 3 * (size_t)kMaxN + 8;

static __device__ __align__(256) double scratch[kScratchDoubles];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
std::array<double*, kMaxDevices> g_ptr{};  // device address of scratch, per device

// the device address of this device's scratch array (set up on first use)
int scratch_ptr(double** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    gir::set_last_error(hipGetErrorString(e));
    return GMRESIR_EHIP;
  }
  if (dev < 0 || dev >= kMaxDevices) {
    gir::set_last_error("device index beyond the scratch table");
    return GMRESIR_EINVAL;
  }
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      gir::set_last_error(e != hipSuccess ? hipGetErrorString(e)
                                          : "hipGetSymbolAddress returned null");
      return GMRESIR_EHIP;
    }
    g_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_ptr[dev];
  return 0;
}

}  // namespace

extern "C" int gmresir_errors_noalloc(const double* A, int64_t n, int64_t lda, const double* b,
                                      const double* x, const double* x_true, double* out,
                                      void* stream) {
  if (!A || !b || !x || !out || n <= 0 || lda < n) {
    gir::set_last_error("invalid arguments (null pointer, n <= 0 or lda < n)");
    return GMRESIR_EINVAL;
  }
  if (n > kMaxN) {
    gir::set_last_error("n exceeds the static scratch limit of 16384");
    return GMRESIR_EINVAL;
  }
  // the residual kernel reads the rows of A as 16-byte pairs
  if ((reinterpret_cast<uintptr_t>(A) & 15) != 0 || (lda & 1) != 0) {
    gir::set_last_error("A must be 16-byte aligned with an even leading dimension");
    return GMRESIR_EINVAL;
  }
  double* base = nullptr;
  const int rc = scratch_ptr(&base);
  if (rc) return rc;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  double* bs = base;
  double* xs = base + kMaxN;
  double* rs = base + 2 * kMaxN;
  unsigned long long* w = reinterpret_cast<unsigned long long*>(base + 3 * kMaxN);
  // every reduction word is cleared by the kernel that raises it (no memset
  // node), so a previous call's contents do not matter
  const int ni = (int)n;
  gir::launch_copy_i32(reinterpret_cast<int*>(bs), reinterpret_cast<const int*>(b), 2 * n, s);
  gir::launch_copy_i32(reinterpret_cast<int*>(xs), reinterpret_cast<const int*>(x), 2 * n, s);
  gir::launch_maxabs(bs, ni, w + 2, s);
  gir::launch_rowsum_max(A, n, lda, w + 3, s);
  gir::launch_residual_dd(A, lda, ni, bs, xs, rs, w, s);
  if (x_true) {
    gir::launch_copy_i32(reinterpret_cast<int*>(rs), reinterpret_cast<const int*>(x_true),
                         2 * n, s);
    gir::launch_ferr(xs, rs, ni, w + 5, s);
  }
  gir::launch_errors_finish(w, x_true ? 1 : 0, out, s);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    gir::set_last_error(hipGetErrorString(e));
    return GMRESIR_EHIP;
  }
  return 0;
}
