// Device-side helpers shared by the librs kernels (gfx950, wave64).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rs {

// ------------------------------------------------------------ Philox4x32-10
// Counter-based generator of Salmon, Moraes, Dror and Shaw (SC'11): ten rounds,
// each multiplying counter words 0 and 2 by two 32-bit constants, mixing the
// high halves with the other words and the key, and bumping the key by the Weyl
// constants between rounds.
constexpr uint32_t kPhiloxM0 = 0xD2511F53u;
constexpr uint32_t kPhiloxM1 = 0xCD9E8D57u;
constexpr uint32_t kPhiloxW0 = 0x9E3779B9u;
constexpr uint32_t kPhiloxW1 = 0xBB67AE85u;

constexpr uint32_t kStreamSigns = 4;
constexpr uint32_t kStreamRowKeys = 5;
constexpr uint32_t kStreamGauss = 6;
constexpr uint32_t kStreamProbe = 7;
constexpr uint32_t kStreamCount = 8;

__device__ __forceinline__ uint4 philox(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint32_t lo0 = kPhiloxM0 * c.x;
    const uint32_t hi0 = __umulhi(kPhiloxM0, c.x);
    const uint32_t lo1 = kPhiloxM1 * c.z;
    const uint32_t hi1 = __umulhi(kPhiloxM1, c.z);
    c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
    k0 += kPhiloxW0;
    k1 += kPhiloxW1;
  }
  return c;
}

// Block for counter (idx, stream, sketch_id) under key = seed.
__device__ __forceinline__ uint4 draw(uint64_t seed, uint32_t stream, uint32_t sketch_id,
                                      uint64_t idx) {
  return philox(make_uint4((uint32_t)idx, (uint32_t)(idx >> 32), stream, sketch_id),
                (uint32_t)seed, (uint32_t)(seed >> 32));
}

__device__ __forceinline__ uint64_t row_key(uint64_t seed, uint32_t sid, uint64_t i) {
  const uint4 w = draw(seed, kStreamRowKeys, sid, i);
  return ((uint64_t)w.y << 32) | (uint64_t)w.x;
}

__device__ __forceinline__ int sign_of(uint64_t seed, uint32_t sid, uint64_t i) {
  const uint4 w = draw(seed, kStreamSigns, sid, i);
  return 1 - 2 * (int)(w.x & 1u);
}

// Box-Muller standard normal, FP32 uniforms ((w >> 9) + 1/2) 2^-23.
__device__ __forceinline__ float gauss_f32(uint64_t seed, uint32_t sid, uint64_t idx) {
  const uint4 w = draw(seed, kStreamGauss, sid, idx);
  const float u1 = ((float)(w.x >> 9) + 0.5f) * 1.1920928955078125e-07f;
  const float u2 = ((float)(w.y >> 9) + 0.5f) * 1.1920928955078125e-07f;
  return sqrtf(-2.0f * logf(u1)) * cosf(6.2831853071795864769f * u2);
}

// Box-Muller standard normal, FP64 uniforms with 52 random bits each.
__device__ __forceinline__ double gauss_f64(uint64_t seed, uint32_t sid, uint64_t idx) {
  const uint4 w = draw(seed, kStreamGauss, sid, idx);
  const double u1 = ((double)(w.x >> 6) * 67108864.0 + (double)(w.y >> 6) + 0.5) *
                    2.220446049250313080847e-16;
  const double u2 = ((double)(w.z >> 6) * 67108864.0 + (double)(w.w >> 6) + 0.5) *
                    2.220446049250313080847e-16;
  return sqrt(-2.0 * log(u1)) * cos(6.283185307179586476925 * u2);
}

// ------------------------------------------------------------ reductions
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Butterfly sum over aligned groups of W lanes (W a power of two <= 64); every
// lane of a group ends with the same bits.
template <int W, typename T>
__device__ __forceinline__ T group_sum(T v) {
#pragma unroll
  for (int off = W / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// Value of v in lane src (src uniform across the wave), through the scalar
// unit: two v_readlane_b32 instead of a cross-lane permute.
__device__ __forceinline__ double lane_value(double v, int src) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)b, src);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), src);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Fixed-order sum over a block of nthreads threads of per-thread values for K
// columns: each thread first adds its strided share of src[b * K + c] (b <
// count), then a tree in LDS.  Result in out[c] (shared) for every c < K.
template <int K, int NT>
__device__ __forceinline__ void block_sum_cols(const double* __restrict__ src, int count,
                                               double* sh /* NT * K */, double* out) {
  const int t = threadIdx.x;
  double v[K];
#pragma unroll
  for (int c = 0; c < K; ++c) v[c] = 0.0;
  for (int b = t; b < count; b += NT)
#pragma unroll
    for (int c = 0; c < K; ++c) v[c] += src[(int64_t)b * K + c];
#pragma unroll
  for (int c = 0; c < K; ++c) sh[c * NT + t] = v[c];
  __syncthreads();
  for (int off = NT / 2; off > 0; off >>= 1) {
    if (t < off)
#pragma unroll
      for (int c = 0; c < K; ++c) sh[c * NT + t] += sh[c * NT + t + off];
    __syncthreads();
  }
  if (t < K) out[t] = sh[t * NT];
  __syncthreads();
}

// Rows r0.. of Y = H G (K columns) for one block: each wave takes RPW rows, lanes
// read 16-byte pairs of H (128 columns per wave per step, ldh even and H 16-byte
// aligned); the block's share of g^T Y goes to rpart[c].
template <int K, int RPW>
__device__ __forceinline__ void symv_rows(const double* __restrict__ H, int64_t ldh, int64_t d,
                                          const double* __restrict__ G, double* __restrict__ Y,
                                          double* __restrict__ rpart) {
  __shared__ double rr[4][K];
  const int lane = threadIdx.x & 63;
  const int w = threadIdx.x >> 6;
  const int64_t r0 = ((int64_t)blockIdx.x * 4 + w) * RPW;
  double acc[RPW][K];
#pragma unroll
  for (int i = 0; i < RPW; ++i)
#pragma unroll
    for (int c = 0; c < K; ++c) acc[i][c] = 0.0;
  for (int64_t j0 = 0; j0 < d; j0 += 128) {
    const int64_t j = j0 + 2 * lane;
    const bool ok0 = j < d, ok1 = j + 1 < d;
    const int64_t jc = ok0 ? j : 0;
    double g0[K], g1[K];
#pragma unroll
    for (int c = 0; c < K; ++c) {
      const double a0 = G[c * d + jc];
      const double a1 = G[c * d + (ok1 ? j + 1 : 0)];
      g0[c] = ok0 ? a0 : 0.0;
      g1[c] = ok1 ? a1 : 0.0;
    }
#pragma unroll
    for (int i = 0; i < RPW; ++i) {
      const int64_t row = r0 + i < d ? r0 + i : 0;
      const double2 h = *reinterpret_cast<const double2*>(H + row * ldh + jc);
#pragma unroll
      for (int c = 0; c < K; ++c) acc[i][c] = fma(h.x, g0[c], fma(h.y, g1[c], acc[i][c]));
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
    rpart[threadIdx.x] = s;
  }
}

// ------------------------------------------------------------ conversions
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float bf16_to_f32(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

// OCP FP8 E4M3 (bias 7, max 448, no infinities), round to nearest even,
// saturating to +-448.
__device__ __forceinline__ uint8_t f32_to_e4m3(float f) {
  uint32_t u = __float_as_uint(f);
  const uint32_t sign = (u >> 24) & 0x80u;
  float a = fabsf(f);
  if (!(a == a)) return (uint8_t)(sign | 0x7f);
  if (a >= 448.0f) return (uint8_t)(sign | 0x7e);
  if (a < 0.0009765625f) {  // below 2^-10: subnormal range step 2^-9
    int q = (int)rintf(a * 512.0f);
    return (uint8_t)(sign | (uint32_t)q);
  }
  int e;
  float mfrac = frexpf(a, &e);  // a = mfrac * 2^e, mfrac in [0.5, 1)
  int E = e - 1 + 7;            // biased exponent of a = 1.xxx * 2^(e-1)
  if (E <= 0) {                 // subnormal: value = q * 2^-9
    int q = (int)rintf(a * 512.0f);
    if (q >= 8) return (uint8_t)(sign | 0x08u);
    return (uint8_t)(sign | (uint32_t)q);
  }
  float scaled = mfrac * 16.0f;  // in [8, 16): 1.mmm * 8
  int q = (int)rintf(scaled);    // 8..16
  if (q == 16) { q = 8; E += 1; }
  if (E > 15 || (E == 15 && (q - 8) > 6)) return (uint8_t)(sign | 0x7e);
  return (uint8_t)(sign | ((uint32_t)E << 3) | (uint32_t)(q - 8));
}
__device__ __forceinline__ float e4m3_to_f32(uint8_t v) {
  const float s = (v & 0x80u) ? -1.0f : 1.0f;
  const int E = (v >> 3) & 0xf;
  const int M = v & 7;
  if (E == 0) return s * (float)M * 0.001953125f;
  return s * ldexpf(1.0f + (float)M * 0.125f, E - 7);
}

// Row of the 16x16 MFMA result held in accumulator slot r of `lane`.
// 16x16x4 FP32 (and the FP32-accumulating BF16 forms): rows 4*(lane/16) + r.
// 16x16x4 FP64: rows lane/16 + 4*r (checked by a lane-layout probe on gfx950).
template <typename TAcc>
__device__ __forceinline__ int mfma16_row(int lane, int r) {
  return sizeof(TAcc) == 4 ? 4 * (lane >> 4) + r : (lane >> 4) + 4 * r;
}

template <typename T> struct VecOf;
template <> struct VecOf<float> { using type = float4; static constexpr int n = 4; };
template <> struct VecOf<double> { using type = double2; static constexpr int n = 2; };

__device__ __forceinline__ float get(const float4& v, int i) {
  return i == 0 ? v.x : (i == 1 ? v.y : (i == 2 ? v.z : v.w));
}
__device__ __forceinline__ double get(const double2& v, int i) { return i == 0 ? v.x : v.y; }
__device__ __forceinline__ void set(float4& v, int i, float x) {
  if (i == 0) v.x = x; else if (i == 1) v.y = x; else if (i == 2) v.z = x; else v.w = x;
}
__device__ __forceinline__ void set(double2& v, int i, double x) {
  if (i == 0) v.x = x; else v.y = x;
}

}  // namespace rs
