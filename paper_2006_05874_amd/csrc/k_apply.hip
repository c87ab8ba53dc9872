// gtilde = H_S^-1 g and the sketched Newton decrement r = 1/2 g^T gtilde
// (Lemma 1), for k right-hand sides, against the explicit FP64 inverse built by
// the factor.  One wave per RPW rows of Hinv: lanes stride the columns (512-byte
// coalesced reads), each g value loaded once per wave is used for RPW rows.
#include "rs_internal.hpp"

namespace rs {

template <int K, int RPW>
__global__ __launch_bounds__(256) void k_symv(const double* __restrict__ H, int64_t ldh, int64_t d,
                                              const double* __restrict__ G,
                                              double* __restrict__ Y, double* __restrict__ rpart,
                                              const int* __restrict__ status) {
  if (status && *status != 0) return;
  __shared__ double rr[4][K];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + w) * RPW;
  double acc[RPW][K];
#pragma unroll
  for (int i = 0; i < RPW; ++i)
#pragma unroll
    for (int c = 0; c < K; ++c) acc[i][c] = 0.0;
  for (int64_t j = lane; j < d; j += 64) {
    double gv[K];
#pragma unroll
    for (int c = 0; c < K; ++c) gv[c] = G[c * d + j];
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int64_t row = r0 + i;
      if (row < d) {
        const double h = H[row * ldh + j];
#pragma unroll
        for (int c = 0; c < K; ++c) acc[i][c] = fma(h, gv[c], acc[i][c]);
      }
    }
  }
  double rloc[K];
#pragma unroll
  for (int c = 0; c < K; ++c) rloc[c] = 0.0;
#pragma unroll
  for (int i = 0; i < RPW; ++i) {
    const int64_t row = r0 + i;
#pragma unroll
    for (int c = 0; c < K; ++c) {
      const double y = wave_sum(acc[i][c]);
      if (row < d) {
        if (lane == 0) Y[c * d + row] = y;
        rloc[c] += y * G[c * d + row];
      }
    }
  }
  if (lane == 0)
#pragma unroll
    for (int c = 0; c < K; ++c) rr[w][c] = rloc[c];
  __syncthreads();
  if (threadIdx.x < K) {
    double s = 0.0;
    for (int ww = 0; ww < 4; ++ww) s += rr[ww][threadIdx.x];
    rpart[(int64_t)blockIdx.x * K + threadIdx.x] = s;
  }
}

// r[c] = 1/2 sum_b rpart[b][c] (fixed order).
__global__ void k_rsum(const double* __restrict__ rpart, int nblk, int K, double* __restrict__ r) {
  if (threadIdx.x < (unsigned)K) {
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += rpart[(int64_t)b * K + threadIdx.x];
    r[threadIdx.x] = 0.5 * s;
  }
}

constexpr int kApplyRPW = 2;

int apply_blocks(int64_t d) { return (int)((d + 4 * kApplyRPW - 1) / (4 * kApplyRPW)); }

rs_status apply_launch(const double* Hinv, int64_t ldh, int64_t d, const double* G, int k,
                       double* Y, double* rpart, const int* status, hipStream_t s) {
  const unsigned nb = (unsigned)apply_blocks(d);
  switch (k) {
    case 1: hipLaunchKernelGGL((k_symv<1, kApplyRPW>), dim3(nb), dim3(256), 0, s, Hinv, ldh, d, G, Y, rpart, status); break;
    case 2: hipLaunchKernelGGL((k_symv<2, kApplyRPW>), dim3(nb), dim3(256), 0, s, Hinv, ldh, d, G, Y, rpart, status); break;
    case 3: hipLaunchKernelGGL((k_symv<3, kApplyRPW>), dim3(nb), dim3(256), 0, s, Hinv, ldh, d, G, Y, rpart, status); break;
    case 4: hipLaunchKernelGGL((k_symv<4, kApplyRPW>), dim3(nb), dim3(256), 0, s, Hinv, ldh, d, G, Y, rpart, status); break;
    default: return set_error(RS_ERR_ARG, "apply: k must be in 1..4");
  }
  return check_launch("apply");
}

rs_status rsum_launch(const double* rpart, int nblk, int k, double* r, hipStream_t s) {
  hipLaunchKernelGGL(k_rsum, dim3(1), dim3(64), 0, s, rpart, nblk, k, r);
  return check_launch("rsum");
}

}  // namespace rs
