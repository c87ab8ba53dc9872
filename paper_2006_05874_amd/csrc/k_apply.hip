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
  symv_rows<K, RPW>(H, ldh, d, G, Y, rpart + (int64_t)blockIdx.x * K);
}

// r[c] = 1/2 sum_b rpart[b][c] (fixed order).
template <int K>
__global__ __launch_bounds__(256) void k_rsum(const double* __restrict__ rpart, int nblk,
                                              double* __restrict__ r) {
  __shared__ double sh[256 * K];
  __shared__ double out[K];
  block_sum_cols<K, 256>(rpart, nblk, sh, out);
  if (threadIdx.x < K) r[threadIdx.x] = 0.5 * out[threadIdx.x];
}

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
  switch (k) {
    case 1: hipLaunchKernelGGL(k_rsum<1>, dim3(1), dim3(256), 0, s, rpart, nblk, r); break;
    case 2: hipLaunchKernelGGL(k_rsum<2>, dim3(1), dim3(256), 0, s, rpart, nblk, r); break;
    case 3: hipLaunchKernelGGL(k_rsum<3>, dim3(1), dim3(256), 0, s, rpart, nblk, r); break;
    case 4: hipLaunchKernelGGL(k_rsum<4>, dim3(1), dim3(256), 0, s, rpart, nblk, r); break;
    default: return set_error(RS_ERR_ARG, "rsum: k must be in 1..4");
  }
  return check_launch("rsum");
}

}  // namespace rs
