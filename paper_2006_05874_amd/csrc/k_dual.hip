// The underdetermined case (appendix, the dual problem): Algorithm 1 runs on the
// dual, whose data matrix is A^T.  These kernels form that matrix once, widen b
// for the dual gradient A A^T z - b + nu^2 z, and map the dual solution back to
// the primal one, x = A^T z.
#include "rs_internal.hpp"

namespace rs {

// M = A^T (d x n, leading dimension ldm >= n; columns n..ldm-1 of M set to 0).
// 64 x 64 tiles through LDS (one padding column against bank conflicts): rows of
// A are read and rows of M written as 64 consecutive elements per wave.
template <typename T>
__global__ __launch_bounds__(256) void k_transpose(const T* __restrict__ A, int64_t n, int64_t d,
                                                   int64_t lda, T* __restrict__ M, int64_t ldm) {
  __shared__ T tile[64][65];
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  const int64_t c0 = (int64_t)blockIdx.x * 64;  // columns of A = rows of M
  const int64_t r0 = (int64_t)blockIdx.y * 64;  // rows of A = columns of M
  for (int r = ty; r < 64; r += 4) {
    const int64_t row = r0 + r, col = c0 + tx;
    tile[r][tx] = (row < n && col < d) ? A[row * lda + col] : T(0);
  }
  __syncthreads();
  for (int r = ty; r < 64; r += 4) {
    const int64_t mrow = c0 + r, mcol = r0 + tx;
    if (mrow < d && mcol < ldm) M[mrow * ldm + mcol] = tile[tx][r];
  }
}

// c = b in FP64.
template <typename T>
__global__ __launch_bounds__(256) void k_widen(const T* __restrict__ b, int64_t n,
                                               double* __restrict__ c) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    c[i] = (double)b[i];
}

// x = M z (M rows x cols, leading dimension ldm): one wave per row, lanes stride
// the row, FP64 accumulation, a fixed-order butterfly over the wave.
template <typename T>
__global__ __launch_bounds__(256) void k_rowdot(const T* __restrict__ M, int64_t rows, int64_t cols,
                                                int64_t ldm, const double* __restrict__ z,
                                                double* __restrict__ x) {
  const int lane = threadIdx.x & 63;
  const int64_t row = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= rows) return;
  const T* m = M + row * ldm;
  double acc = 0.0;
  for (int64_t j = lane; j < cols; j += 64) acc += (double)m[j] * z[j];
  for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, 64);
  if (lane == 0) x[row] = acc;
}

rs_status dual_transpose(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda, void* M,
                         int64_t ldm, hipStream_t s) {
  const dim3 grid((unsigned)((d + 63) / 64), (unsigned)((ldm + 63) / 64));
  if (grid.y > 65535u) return set_error(RS_ERR_SHAPE, "dual: n too large for the transpose");
  if (a_t == RS_F32)
    hipLaunchKernelGGL(k_transpose<float>, grid, dim3(256), 0, s,
                       reinterpret_cast<const float*>(A), n, d, lda, reinterpret_cast<float*>(M),
                       ldm);
  else
    hipLaunchKernelGGL(k_transpose<double>, grid, dim3(256), 0, s,
                       reinterpret_cast<const double*>(A), n, d, lda, reinterpret_cast<double*>(M),
                       ldm);
  return check_launch("dual transpose");
}

rs_status dual_widen(const void* b, rs_dtype a_t, int64_t n, double* c, hipStream_t s) {
  const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
  if (a_t == RS_F32)
    hipLaunchKernelGGL(k_widen<float>, dim3(g), dim3(256), 0, s, reinterpret_cast<const float*>(b),
                       n, c);
  else
    hipLaunchKernelGGL(k_widen<double>, dim3(g), dim3(256), 0, s,
                       reinterpret_cast<const double*>(b), n, c);
  return check_launch("dual widen");
}

rs_status dual_rowdot(const void* M, rs_dtype a_t, int64_t rows, int64_t cols, int64_t ldm,
                      const double* z, double* x, hipStream_t s) {
  const unsigned g = (unsigned)((rows + 3) / 4);
  if (a_t == RS_F32)
    hipLaunchKernelGGL(k_rowdot<float>, dim3(g), dim3(256), 0, s,
                       reinterpret_cast<const float*>(M), rows, cols, ldm, z, x);
  else
    hipLaunchKernelGGL(k_rowdot<double>, dim3(g), dim3(256), 0, s,
                       reinterpret_cast<const double*>(M), rows, cols, ldm, z, x);
  return check_launch("dual map");
}

}  // namespace rs
