// gtilde = H_S^-1 g and the sketched Newton decrement r = 1/2 g^T gtilde
// (Lemma 1), for k right-hand sides: against the explicit FP64 inverse of the
// d x d factor (m >= d), or through the whitened sketch C (m < d, below).  One wave per RPW rows of Hinv: lanes stride the columns (512-byte
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

// ---------------------------------------------------------------- Woodbury form
// With C = L^-1 SA (m x d, the whitened sketch of the factor; L L^T = nu^2 I +
// SA SA^T), H_S^-1 g = (g - C^T (C g)) / nu^2 (Woodbury identity, proof of
// Theorem 7): two passes over C, O(m d) per apply, no d x d inverse.  Everything
// in FP64; sums in a fixed order.
// Y[c][i] = (C G)[i][c]: one wave per row of C, lanes stride the columns.
template <int K>
__global__ __launch_bounds__(256) void k_wy(const double* __restrict__ C, int64_t ldc, int64_t m,
                                            int64_t d, const double* __restrict__ G,
                                            double* __restrict__ Y, const int* __restrict__ status) {
  if (status && *status != 0) return;
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (i >= m) return;
  double acc[K];
#pragma unroll
  for (int c = 0; c < K; ++c) acc[c] = 0.0;
  for (int64_t j = lane; j < d; j += 64) {
    const double cij = C[i * ldc + j];
#pragma unroll
    for (int c = 0; c < K; ++c) acc[c] = fma(cij, G[c * d + j], acc[c]);
  }
#pragma unroll
  for (int c = 0; c < K; ++c) {
    const double y = wave_sum(acc[c]);
    if (lane == 0) Y[c * m + i] = y;
  }
}

// P[s][c][j] = sum over rows i of split s of C[i][j] Y[c][i]: block (256 columns,
// split s), one column per thread, rows in order.
template <int K>
__global__ __launch_bounds__(256) void k_wct(const double* __restrict__ C, int64_t ldc, int64_t m,
                                             int64_t d, const double* __restrict__ Y,
                                             int64_t rows_per_split, int64_t ldp,
                                             double* __restrict__ P, const int* __restrict__ status) {
  if (status && *status != 0) return;
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int64_t i0 = (int64_t)blockIdx.y * rows_per_split;
  const int64_t i1 = i0 + rows_per_split < m ? i0 + rows_per_split : m;
  const int64_t jc = j < d ? j : 0;
  double acc[K];
#pragma unroll
  for (int c = 0; c < K; ++c) acc[c] = 0.0;
  for (int64_t i = i0; i < i1; ++i) {
    const double cij = C[i * ldc + jc];
#pragma unroll
    for (int c = 0; c < K; ++c) acc[c] = fma(cij, Y[c * m + i], acc[c]);
  }
  if (j < d)
#pragma unroll
    for (int c = 0; c < K; ++c) P[((int64_t)blockIdx.y * K + c) * ldp + j] = acc[c];
}

// gtilde = (G - sum_s P[s]) / nu^2 and the block partials of g^T gtilde into
// rpart[b][c] (block b of 256 columns); block 0 zeroes the partial slots past the
// grid up to nrp, so the decision kernels read the same layout as after k_symv.
template <int K>
__global__ __launch_bounds__(256) void k_wfin(const double* __restrict__ P, int ns, int64_t ldp,
                                              int64_t d, const double* __restrict__ G,
                                              double inv_nu2, double* __restrict__ GT,
                                              double* __restrict__ rpart, int nrp,
                                              const int* __restrict__ status) {
  if (status && *status != 0) return;
  __shared__ double sh[256 * K];
  __shared__ double out[K];
  const int64_t j = (int64_t)blockIdx.x * 256 + threadIdx.x;
  double loc[K];
#pragma unroll
  for (int c = 0; c < K; ++c) {
    loc[c] = 0.0;
    if (j < d) {
      double q = 0.0;
      for (int z = 0; z < ns; ++z) q += P[((int64_t)z * K + c) * ldp + j];
      const double g = G[c * d + j];
      const double gt = (g - q) * inv_nu2;
      GT[c * d + j] = gt;
      loc[c] = g * gt;
    }
    sh[c * 256 + threadIdx.x] = loc[c];
  }
  __syncthreads();
  if (threadIdx.x < K) {
    double s = 0.0;
    for (int u = 0; u < 256; ++u) s += sh[threadIdx.x * 256 + u];
    out[threadIdx.x] = s;
    rpart[(int64_t)blockIdx.x * K + threadIdx.x] = s;
  }
  if (blockIdx.x == 0)
    for (int64_t e = (int64_t)gridDim.x * K + threadIdx.x; e < (int64_t)nrp * K; e += 256)
      rpart[e] = 0.0;
}

int wapply_splits(int64_t m, int64_t d) {
  const int64_t cb = (d + 255) / 256;
  int64_t ns = (2 * device_cus() + cb - 1) / cb;
  ns = std::max<int64_t>(1, std::min<int64_t>(ns, (m + 63) / 64));
  return (int)std::min<int64_t>(ns, 64);
}

size_t wapply_scratch_doubles(int64_t m, int64_t d) {
  const int64_t dp = (d + 63) / 64 * 64;
  return (size_t)4 * m + (size_t)wapply_splits(m, d) * 4 * dp;
}

rs_status wapply_launch(const double* C, int64_t ldc, int64_t m, int64_t d, double nu2,
                        const double* G, int k, double* GT, double* rpart, int nrp,
                        double* scratch, const int* status, hipStream_t s) {
  if (k < 1 || k > 4) return set_error(RS_ERR_ARG, "apply: k must be in 1..4");
  if ((d + 255) / 256 > nrp) return set_error(RS_ERR_ARG, "apply: partial count too small");
  const int ns = wapply_splits(m, d);
  const int64_t rps = (m + ns - 1) / ns;
  const int64_t dp = (d + 63) / 64 * 64;
  double* Y = scratch;
  double* P = scratch + 4 * m;
  const dim3 gy((unsigned)((m + 3) / 4)), gc((unsigned)((d + 255) / 256), (unsigned)ns),
      gf((unsigned)((d + 255) / 256));
  const double inv = 1.0 / nu2;
#define RS_WAPPLY(KK)                                                                           \
  hipLaunchKernelGGL(k_wy<KK>, gy, dim3(256), 0, s, C, ldc, m, d, G, Y, status);              \
  hipLaunchKernelGGL(k_wct<KK>, gc, dim3(256), 0, s, C, ldc, m, d, Y, rps, dp, P, status);    \
  hipLaunchKernelGGL(k_wfin<KK>, gf, dim3(256), 0, s, P, ns, dp, d, G, inv, GT, rpart, nrp,   \
                     status);
  switch (k) {
    case 1: RS_WAPPLY(1) break;
    case 2: RS_WAPPLY(2) break;
    case 3: RS_WAPPLY(3) break;
    case 4: RS_WAPPLY(4) break;
  }
#undef RS_WAPPLY
  return check_launch("woodbury apply");
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
