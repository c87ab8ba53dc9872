// Low-precision storage of the sketch SA for the precision form.
//
// FP8 (OCP E4M3, largest finite 448): each column j gets a power-of-two scale
// s_j = 2^ceil(log2(max_k |SA[k][j]| / 448)) (1 for an all-zero column) so the
// column's largest entry maps into [224, 448]; SA[k][j] ~= fp8(SA[k][j] / s_j) * s_j
// with round-to-nearest-even.  The stored values define the sketch used by the
// factor: its Gram is formed from the dequantized entries, so H_S stays an exact
// (S'A)^T (S'A) + nu^2 I for the rounded sketch and the outer iteration still
// converges to x*.
#include "rs_internal.hpp"

namespace rs {

// colmax[j] = max_k |X[k][j]| (as float bits; all values are >= 0).
__global__ __launch_bounds__(256) void k_colmax(const float* __restrict__ X, int64_t m, int64_t d,
                                                int64_t ldx, uint32_t* __restrict__ colmax) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j >= d) return;
  const int64_t k0 = (int64_t)blockIdx.y * 256;
  const int64_t k1 = k0 + 256 < m ? k0 + 256 : m;
  float mx = 0.0f;
  for (int64_t k = k0; k < k1; ++k) mx = fmaxf(mx, fabsf(X[k * ldx + j]));
  atomicMax(&colmax[j], __float_as_uint(mx));
}

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    p[i] = v;
}

__device__ __forceinline__ float pow2_scale(float mx) {
  if (!(mx > 0.0f)) return 1.0f;
  int e;
  frexpf(mx / 448.0f, &e);            // mx/448 = f * 2^e, f in [0.5, 1)
  float s = ldexpf(1.0f, e);           // smallest power of two >= mx/448 (up to one step)
  if (mx / (s * 0.5f) <= 448.0f) s *= 0.5f;
  return s;
}

__global__ __launch_bounds__(256) void k_scales(const uint32_t* __restrict__ colmax, int64_t d,
                                                float* __restrict__ scale) {
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (j < d) scale[j] = pow2_scale(__uint_as_float(colmax[j]));
}

__global__ __launch_bounds__(256) void k_quant_fp8(const float* __restrict__ X, int64_t m,
                                                   int64_t d, int64_t ldx,
                                                   const float* __restrict__ scale,
                                                   uint8_t* __restrict__ Q, int64_t ldq) {
  const int64_t total = m * d;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int64_t k = e / d, j = e % d;
    Q[k * ldq + j] = f32_to_e4m3(X[k * ldx + j] / scale[j]);
  }
}

rs_status quantize_fp8(const float* X, int64_t m, int64_t d, int64_t ldx, uint32_t* colmax,
                       float* scale, uint8_t* Q, int64_t ldq, hipStream_t s) {
  hipLaunchKernelGGL(k_fill_u32, dim3((unsigned)std::min<int64_t>((d + 255) / 256, 1024)),
                     dim3(256), 0, s, colmax, d, 0u);
  hipLaunchKernelGGL(k_colmax, dim3((unsigned)((d + 255) / 256), (unsigned)((m + 255) / 256)),
                     dim3(256), 0, s, X, m, d, ldx, colmax);
  hipLaunchKernelGGL(k_scales, dim3((unsigned)((d + 255) / 256)), dim3(256), 0, s, colmax, d, scale);
  const int64_t total = m * d;
  hipLaunchKernelGGL(k_quant_fp8, dim3((unsigned)std::min<int64_t>((total + 255) / 256, 65536)),
                     dim3(256), 0, s, X, m, d, ldx, scale, Q, ldq);
  return check_launch("fp8 quantize");
}

}  // namespace rs
