// rs_gradient_noalloc: the gradient pass of rs_gradient with its per-block FP64
// partial sums in a fixed file-scope device array, so that the call allocates no
// device memory (for callers under HIP graph capture or in loops that may not call
// hipMalloc).  The kernels are those of rs_gradient; only where the partial sums
// live differs.
#include <mutex>
#include <string>

#include "rs_internal.hpp"

namespace rs {

// 8 Mi doubles (64 MiB): every built (d, k) fits with at least 256 partial-sum
// blocks (d <= 8192, k <= 4).  Each device holds its own copy for the life of
// the process.
constexpr int64_t kNoAllocDoubles = (int64_t)8 << 20;
static __device__ __align__(256) double scratch[kNoAllocDoubles];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
double* g_noalloc_ptr[kMaxDevices] = {};  // per device: the address of its copy of scratch

// The device address of the current device's copy of scratch, looked up once per
// device (with that device current).  The host-side name of the array is only a
// stand-in for it and is never passed to a kernel.
rs_status noalloc_scratch(double** out) {
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
    return set_error(RS_ERR_HIP, "rs_gradient_noalloc: no current device");
  std::lock_guard<std::mutex> g(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return set_error(RS_ERR_HIP, (std::string("rs_gradient_noalloc: hipGetSymbolAddress: ") +
                                    hipGetErrorString(e)).c_str());
    g_noalloc_ptr[dev] = static_cast<double*>(p);
  }
  *out = g_noalloc_ptr[dev];
  return RS_OK;
}

}  // namespace
}  // namespace rs

using namespace rs;

extern "C" {

rs_status rs_gradient_noalloc(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda,
                              const void* b, double nu2, const double* X, int64_t k, double* G,
                              hipStream_t stream) {
  if (!A || !b || !X || !G) return set_error(RS_ERR_ARG, "rs_gradient_noalloc: null argument");
  if (a_t != RS_F32 && a_t != RS_F64)
    return set_error(RS_ERR_ARG, "rs_gradient_noalloc: A must be F32 or F64");
  if (n < 1 || d < 1) return set_error(RS_ERR_SHAPE, "rs_gradient_noalloc: empty matrix");
  const int64_t es = a_t == RS_F64 ? 8 : 4;
  if (lda < d || (lda * es) % 16 != 0)
    return set_error(RS_ERR_ARG, "rs_gradient_noalloc: lda must be >= d and a multiple of 16 bytes");
  if (reinterpret_cast<uintptr_t>(A) % 16 != 0)
    return set_error(RS_ERR_ARG, "rs_gradient_noalloc: A must be 16-byte aligned");
  if (k < 1 || k > 4) return set_error(RS_ERR_ARG, "rs_gradient_noalloc: k must be in 1..4");
  const int64_t kd = k * d;
  if (kd > kNoAllocDoubles)
    return set_error(RS_ERR_SHAPE, "rs_gradient_noalloc: k * d above the fixed scratch (8 Mi doubles)");
  double* part = nullptr;
  const rs_status st = noalloc_scratch(&part);
  if (st != RS_OK) return st;
  // the grid of rs_gradient, capped by what the fixed scratch holds; each block
  // overwrites its own partial, so nothing needs clearing between calls
  const int grid = (int)std::min<int64_t>(grad_partial_blocks_max(n), kNoAllocDoubles / kd);
  if (a_t == RS_F32)
    return gradient_launch<float>(reinterpret_cast<const float*>(A), n, d, lda,
                                  reinterpret_cast<const float*>(b), nu2, X, (int)k, G, part, grid,
                                  nullptr, stream, nullptr, false);
  return gradient_launch<double>(reinterpret_cast<const double*>(A), n, d, lda,
                                 reinterpret_cast<const double*>(b), nu2, X, (int)k, G, part, grid,
                                 nullptr, stream, nullptr, false);
}

}  // extern "C"
