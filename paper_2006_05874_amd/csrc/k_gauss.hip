// Gaussian embedding SA = S A, S[k][j] = z_{k n + j} / sqrt(m) (Section 1: i.i.d.
// N(0, 1/m) entries).  S is never stored: each block draws the 64 x 16 slice of
// S it needs from Philox4x32-10 + Box-Muller into LDS, stages the matching
// 16 x 128 slice of A, and accumulates a 64 x 128 tile of SA on the matrix
// cores (FP32 MFMA 16x16x4 for FP32 data, FP64 MFMA 16x16x4 for FP64 data).
// Forming SA costs 2 m n d flops (the O(mnd) of Section 1).
#include "rs_internal.hpp"

namespace rs {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
__device__ __forceinline__ T gauss_at(uint64_t seed, uint32_t sid, uint64_t idx);
template <>
__device__ __forceinline__ float gauss_at<float>(uint64_t seed, uint32_t sid, uint64_t idx) {
  return gauss_f32(seed, sid, idx);
}
template <>
__device__ __forceinline__ double gauss_at<double>(uint64_t seed, uint32_t sid, uint64_t idx) {
  return gauss_f64(seed, sid, idx);
}

// Output tile 64 x TD: every S slice drawn by a block serves TD columns of SA, so a
// wider tile draws S fewer times (d / TD per slice).  FP32: 256 (512 halves the
// occupancy and is slower); FP64: 128 (its accumulators are twice as large).
template <typename T>
struct GaussTile {
  static constexpr int TD = sizeof(T) == 4 ? 256 : 128;
};

// Rows k_off .. m-1 of SA (earlier rows untouched).  With split > 0 the block
// sums only A's rows [z * split, (z+1) * split) (z = blockIdx.z) and writes its
// unscaled partial to P[z] (rows k - k_off, leading dimension d) instead.
template <typename T, typename OutT>
__global__ __launch_bounds__(256) void k_gauss_sketch(const T* __restrict__ A, int64_t n, int64_t d,
                                                      int64_t lda, int64_t m, uint64_t seed,
                                                      uint32_t sid, double scale,
                                                      OutT* __restrict__ SA, int64_t ldsa,
                                                      int64_t k_off, int64_t split,
                                                      T* __restrict__ P) {
  constexpr int TM = 64, TD = GaussTile<T>::TD, KC = 16;
  constexpr int NB = TD / 32;  // 16-column tiles per wave (a wave owns 32 x TD / 2)
  __shared__ T Ss[KC][TM + 1];  // Ss[j][k] = S[k0 + k][j0 + j]
  __shared__ T As[KC][TD + 1];  // As[j][c] = A[j0 + j][c0 + c]
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;
  const int wr = w >> 1, wc = w & 1;  // wave quadrant: 32 rows x TD / 2 cols
  const int64_t k0 = k_off + (int64_t)blockIdx.y * TM;
  const int64_t c0 = (int64_t)blockIdx.x * TD;
  using Acc4 = typename std::conditional<sizeof(T) == 4, f32x4, f64x4>::type;
  Acc4 acc[2][NB];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = Acc4{0, 0, 0, 0};

  const int64_t jlo = split > 0 ? (int64_t)blockIdx.z * split : 0;
  const int64_t jhi = split > 0 ? (jlo + split < n ? jlo + split : n) : n;
  for (int64_t j0 = jlo; j0 < jhi; j0 += KC) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {  // S slice: 64 x 16 = 1024 draws
      const int idx = t * 4 + e;
      const int kk = idx / KC, jj = idx % KC;
      const int64_t k = k0 + kk, j = j0 + jj;
      T v = 0;
      if (k < m && j < jhi) v = gauss_at<T>(seed, sid, (uint64_t)k * (uint64_t)n + (uint64_t)j);
      Ss[jj][kk] = v;
    }
#pragma unroll
    for (int e = 0; e < KC * TD / 256; ++e) {  // A slice: 16 x TD
      const int idx = t * (KC * TD / 256) + e;
      const int jj = idx / TD, cc = idx % TD;
      const int64_t j = j0 + jj, c = c0 + cc;
      As[jj][cc] = (j < jhi && c < d) ? A[j * lda + c] : (T)0;
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < KC / 4; ++k4) {
      const int kr = k4 * 4 + (lane >> 4);
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const T av = Ss[kr][wr * 32 + a * 16 + (lane & 15)];
#pragma unroll
        for (int b = 0; b < NB; ++b) {
          const T bv = As[kr][wc * (TD / 2) + b * 16 + (lane & 15)];
          if constexpr (sizeof(T) == 4)
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[a][b], 0, 0, 0);
          else
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[a][b], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t k = k0 + wr * 32 + a * 16 + mfma16_row<T>(lane, r);
        const int64_t c = c0 + wc * (TD / 2) + b * 16 + (lane & 15);
        if (k < m && c < d) {
          if (split > 0) {
            P[((int64_t)blockIdx.z * (m - k_off) + (k - k_off)) * d + c] = acc[a][b][r];
          } else {
            const double v = (double)acc[a][b][r] * scale;
            if constexpr (sizeof(OutT) == 2)
              SA[k * ldsa + c] = f32_to_bf16_rne((float)v);
            else
              SA[k * ldsa + c] = (OutT)v;
          }
        }
      }
}

// The precision form's product for FP32 A and a BF16 sketch: S and A are rounded
// to BF16 (nearest even) as they are staged and multiplied on the BF16 matrix
// cores (v_mfma_f32_16x16x32_bf16, FP32 accumulation): SA = bf16(S) bf16(A) / sqrt(m).
// Block tile 64 x 256 of SA, 32 rows of A per step.  LDS holds the S slice
// row-major (Ss[k][j], the A operand: 8 consecutive j per lane) and the A slice
// transposed (As[c][j], the B operand), so every operand read is one 16-byte load.
// Thread (rg, cg) loads rows 8 rg .. 8 rg + 7 of A's columns 4 cg .. 4 cg + 3 (each
// load a 1 KB coalesced row segment across the wave) and writes each column's 8
// rows as one 16-byte LDS store.  Split and output as in k_gauss_sketch.
typedef __bf16 gbf16x8 __attribute__((ext_vector_type(8)));
constexpr int kGbKC = 32;          // rows of A per step
constexpr int kGbPad = kGbKC + 8;  // LDS row pitch (bf16 elements)

template <typename OutT>
__global__ __launch_bounds__(256) void k_gauss_sketch_bf16(
    const float* __restrict__ A, int64_t n, int64_t d, int64_t lda, int64_t m, uint64_t seed,
    uint32_t sid, double scale, OutT* __restrict__ SA, int64_t ldsa, int64_t k_off, int64_t split,
    float* __restrict__ P) {
  constexpr int TM = 64, TD = 256, KC = kGbKC, NB = TD / 32;
  __shared__ __attribute__((aligned(16))) uint16_t Ss[TM][kGbPad];
  __shared__ __attribute__((aligned(16))) uint16_t As[TD][kGbPad];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;
  const int wr = w >> 1, wc = w & 1;  // wave quadrant: 32 rows x 128 cols
  const int64_t k0 = k_off + (int64_t)blockIdx.y * TM;
  const int64_t c0 = (int64_t)blockIdx.x * TD;
  f32x4 acc[2][NB];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b) acc[a][b] = f32x4{0, 0, 0, 0};
  const int64_t jlo = split > 0 ? (int64_t)blockIdx.z * split : 0;
  const int64_t jhi = split > 0 ? (jlo + split < n ? jlo + split : n) : n;
  const int rg = t >> 6, cg = t & 63;  // A staging: 4 row groups of 8 x 64 column groups of 4
  const int64_t ca = c0 + 4 * cg;
  const int64_t car = ca < d ? ca : 0;
  for (int64_t j0 = jlo; j0 < jhi; j0 += KC) {
    // S slice: 64 x 32 = 2048 draws, 8 per thread (row kk, columns jj .. jj + 7)
    {
      const int kk = t >> 2, jj = (t & 3) * 8;
      const int64_t k = k0 + kk;
      uint16_t h[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t j = j0 + jj + e;
        float v = 0.0f;
        if (k < m && j < jhi) v = gauss_f32(seed, sid, (uint64_t)k * (uint64_t)n + (uint64_t)j);
        h[e] = f32_to_bf16_rne(v);
      }
      *reinterpret_cast<uint4*>(&Ss[kk][jj]) = *reinterpret_cast<const uint4*>(h);
    }
    // A slice: rows j0 + 8 rg + e, columns ca .. ca + 3 (zero past jhi and d)
    {
      float4 r[8];
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t j = j0 + 8 * rg + e;
        const int64_t jr = j < jhi ? j : jlo;
        r[e] = *reinterpret_cast<const float4*>(A + jr * lda + car);
        if (j >= jhi) r[e] = make_float4(0.f, 0.f, 0.f, 0.f);
      }
#pragma unroll
      for (int cc = 0; cc < 4; ++cc) {
        uint16_t h[8];
#pragma unroll
        for (int e = 0; e < 8; ++e) h[e] = ca + cc < d ? f32_to_bf16_rne(get(r[e], cc)) : (uint16_t)0;
        *reinterpret_cast<uint4*>(&As[4 * cg + cc][8 * rg]) = *reinterpret_cast<const uint4*>(h);
      }
    }
    __syncthreads();
    const int kof = 8 * (lane >> 4);
#pragma unroll
    for (int a = 0; a < 2; ++a) {
      const gbf16x8 av = *reinterpret_cast<const gbf16x8*>(&Ss[wr * 32 + a * 16 + (lane & 15)][kof]);
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const gbf16x8 bv =
            *reinterpret_cast<const gbf16x8*>(&As[wc * (TD / 2) + b * 16 + (lane & 15)][kof]);
        acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[a][b], 0, 0, 0);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t k = k0 + wr * 32 + a * 16 + mfma16_row<float>(lane, r);
        const int64_t c = c0 + wc * (TD / 2) + b * 16 + (lane & 15);
        if (k < m && c < d) {
          if (split > 0) {
            P[((int64_t)blockIdx.z * (m - k_off) + (k - k_off)) * d + c] = acc[a][b][r];
          } else {
            const double v = (double)acc[a][b][r] * scale;
            if constexpr (sizeof(OutT) == 2)
              SA[k * ldsa + c] = f32_to_bf16_rne((float)v);
            else
              SA[k * ldsa + c] = (OutT)v;
          }
        }
      }
}

// SA[k] = scale * sum_z P[z][k - k_off] (fixed order, FP64) for rows k_off .. m-1.
template <typename T, typename OutT>
__global__ __launch_bounds__(256) void k_gauss_reduce(const T* __restrict__ P, int nz,
                                                      int64_t rows, int64_t d, int64_t k_off,
                                                      double scale, OutT* __restrict__ SA,
                                                      int64_t ldsa) {
  const int64_t r = blockIdx.x;
  for (int64_t c = threadIdx.x; c < d; c += 256) {
    double v = 0.0;
    for (int z = 0; z < nz; ++z) v += (double)P[((int64_t)z * rows + r) * d + c];
    v *= scale;
    if constexpr (sizeof(OutT) == 2)
      SA[(k_off + r) * ldsa + c] = f32_to_bf16_rne((float)v);
    else
      SA[(k_off + r) * ldsa + c] = (OutT)v;
  }
}

// Splits of the summed dimension (A's rows) so that the launch fills the chip
// when m is small; the partials go through P (gauss_split_bytes of scratch).
static int gauss_splits(int64_t n, int64_t d, int64_t rows, int td) {
  const int64_t tiles = ((d + td - 1) / td) * ((rows + 63) / 64);
  int64_t z = (2 * device_cus() + tiles - 1) / tiles;
  z = std::max<int64_t>(1, std::min<int64_t>(z, (n + 1023) / 1024));
  return (int)std::min<int64_t>(z, 64);
}

size_t gauss_split_bytes(int64_t n, int64_t d, int64_t rows, rs_dtype a_t) {
  const int z = gauss_splits(n, d, rows, a_t == RS_F64 ? GaussTile<double>::TD
                                                      : GaussTile<float>::TD);
  return z > 1 ? (size_t)z * rows * d * (a_t == RS_F64 ? 8 : 4) : 0;
}

template <typename T, typename OutT>
static void gauss_go(const T* A, int64_t n, int64_t d, int64_t lda, int64_t m, uint64_t seed,
                     uint32_t sid, double scale, OutT* SA, int64_t ldsa, int64_t k_off,
                     void* part, size_t part_bytes, hipStream_t s) {
  const int64_t rows = m - k_off;
  constexpr int TD = GaussTile<T>::TD;
  const int z = gauss_splits(n, d, rows, TD);
  const size_t need = (size_t)z * rows * d * sizeof(T);
  if (z > 1 && part && part_bytes >= need) {
    const int64_t split = ((n + z - 1) / z + 15) / 16 * 16;
    const unsigned nz = (unsigned)((n + split - 1) / split);
    const dim3 grid((unsigned)((d + TD - 1) / TD), (unsigned)((rows + 63) / 64), nz);
    hipLaunchKernelGGL((k_gauss_sketch<T, OutT>), grid, dim3(256), 0, s, A, n, d, lda, m, seed,
                       sid, scale, SA, ldsa, k_off, split, reinterpret_cast<T*>(part));
    hipLaunchKernelGGL((k_gauss_reduce<T, OutT>), dim3((unsigned)rows), dim3(256), 0, s,
                       reinterpret_cast<const T*>(part), (int)nz, rows, d, k_off, scale, SA, ldsa);
  } else {
    const dim3 grid((unsigned)((d + TD - 1) / TD), (unsigned)((rows + 63) / 64));
    hipLaunchKernelGGL((k_gauss_sketch<T, OutT>), grid, dim3(256), 0, s, A, n, d, lda, m, seed,
                       sid, scale, SA, ldsa, k_off, (int64_t)0, (T*)nullptr);
  }
}

// The BF16 form: the same tiling (64 x 256 tiles, the split over A's rows and its
// FP64 reduction) with the BF16 matrix-core kernel.
static void gauss_go_bf16(const float* A, int64_t n, int64_t d, int64_t lda, int64_t m,
                          uint64_t seed, uint32_t sid, double scale, uint16_t* SA, int64_t ldsa,
                          int64_t k_off, void* part, size_t part_bytes, hipStream_t s) {
  const int64_t rows = m - k_off;
  constexpr int TD = 256;
  const int z = gauss_splits(n, d, rows, TD);
  const size_t need = (size_t)z * rows * d * sizeof(float);
  if (z > 1 && part && part_bytes >= need) {
    const int64_t split = ((n + z - 1) / z + kGbKC - 1) / kGbKC * kGbKC;
    const unsigned nz = (unsigned)((n + split - 1) / split);
    const dim3 grid((unsigned)((d + TD - 1) / TD), (unsigned)((rows + 63) / 64), nz);
    hipLaunchKernelGGL((k_gauss_sketch_bf16<uint16_t>), grid, dim3(256), 0, s, A, n, d, lda, m,
                       seed, sid, scale, SA, ldsa, k_off, split, reinterpret_cast<float*>(part));
    hipLaunchKernelGGL((k_gauss_reduce<float, uint16_t>), dim3((unsigned)rows), dim3(256), 0, s,
                       reinterpret_cast<const float*>(part), (int)nz, rows, d, k_off, scale, SA,
                       ldsa);
  } else {
    const dim3 grid((unsigned)((d + TD - 1) / TD), (unsigned)((rows + 63) / 64));
    hipLaunchKernelGGL((k_gauss_sketch_bf16<uint16_t>), grid, dim3(256), 0, s, A, n, d, lda, m,
                       seed, sid, scale, SA, ldsa, k_off, (int64_t)0, (float*)nullptr);
  }
}

rs_status gauss_launch(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda, int64_t m,
                       uint64_t seed, uint32_t sid, void* SA, rs_dtype sa_t, int64_t ldsa,
                       hipStream_t s, int64_t k_off, double scale_override, void* part,
                       size_t part_bytes) {
  if (k_off >= m) return RS_OK;
  const double scale = scale_override > 0.0 ? scale_override : 1.0 / std::sqrt((double)m);
  if (a_t == RS_F64) {
    if (sa_t != RS_F64) return set_error(RS_ERR_UNSUPPORTED, "gaussian: F64 A needs F64 SA");
    gauss_go<double, double>(reinterpret_cast<const double*>(A), n, d, lda, m, seed, sid, scale,
                             reinterpret_cast<double*>(SA), ldsa, k_off, part, part_bytes, s);
  } else if (sa_t == RS_F32) {
    gauss_go<float, float>(reinterpret_cast<const float*>(A), n, d, lda, m, seed, sid, scale,
                           reinterpret_cast<float*>(SA), ldsa, k_off, part, part_bytes, s);
  } else if (sa_t == RS_BF16) {
    gauss_go_bf16(reinterpret_cast<const float*>(A), n, d, lda, m, seed, sid, scale,
                  reinterpret_cast<uint16_t*>(SA), ldsa, k_off, part, part_bytes, s);
  } else {
    return set_error(RS_ERR_UNSUPPORTED, "gaussian: SA dtype not supported");
  }
  return check_launch("gaussian sketch");
}

// SA = scale * G for the cached unscaled rows G (m x d, leading dimension d) of
// the nested Gaussian sketch: the same product and rounding as the sketch
// kernel's output stage.
template <typename T, typename OutT>
__global__ __launch_bounds__(256) void k_gauss_scale(const T* __restrict__ G, int64_t d,
                                                     double scale, OutT* __restrict__ SA,
                                                     int64_t ldsa) {
  const int64_t k = blockIdx.x;
  for (int64_t c = threadIdx.x; c < d; c += 256) {
    const double v = (double)G[k * d + c] * scale;
    if constexpr (sizeof(OutT) == 2)
      SA[k * ldsa + c] = f32_to_bf16_rne((float)v);
    else
      SA[k * ldsa + c] = (OutT)v;
  }
}

rs_status gauss_scale_rows(const void* G, rs_dtype g_t, int64_t m, int64_t d, double scale,
                           void* SA, rs_dtype sa_t, int64_t ldsa, hipStream_t s) {
  const dim3 g((unsigned)m);
  if (g_t == RS_F64) {
    if (sa_t != RS_F64) return set_error(RS_ERR_UNSUPPORTED, "gaussian: F64 A needs F64 SA");
    hipLaunchKernelGGL((k_gauss_scale<double, double>), g, dim3(256), 0, s,
                       reinterpret_cast<const double*>(G), d, scale,
                       reinterpret_cast<double*>(SA), ldsa);
  } else if (sa_t == RS_F32) {
    hipLaunchKernelGGL((k_gauss_scale<float, float>), g, dim3(256), 0, s,
                       reinterpret_cast<const float*>(G), d, scale, reinterpret_cast<float*>(SA),
                       ldsa);
  } else if (sa_t == RS_BF16) {
    hipLaunchKernelGGL((k_gauss_scale<float, uint16_t>), g, dim3(256), 0, s,
                       reinterpret_cast<const float*>(G), d, scale,
                       reinterpret_cast<uint16_t*>(SA), ldsa);
  } else {
    return set_error(RS_ERR_UNSUPPORTED, "gaussian: SA dtype not supported");
  }
  return check_launch("gaussian scale");
}

}  // namespace rs
