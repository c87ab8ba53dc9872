// Fused gradient G = A^T (A X - b) + nu^2 X for k right-hand sides, one read of A.
//
// The per-iteration cost of the method is this product (proof of Theorem 7: the
// matrix-vector products A x_t and A^T (A x_t - b)).  It is bound by HBM: each
// pass streams n*d*sizeof(T) bytes and does 4 n d k flops.
//
// Layout: TPR threads cover one row of A with NV 16-byte vectors each (columns
// (lt + TPR*v)*VEC ..), so a row is read with fully coalesced 16-byte loads.  A
// 256-thread block holds 256/TPR row groups; each group takes R rows at a time.
// Row dots are reduced inside the group (shuffles, plus LDS when TPR > 64); the
// A^T r products of the R rows are summed in T and then added to FP64
// accumulators.  Each block writes one FP64 partial of length k*d; a second
// kernel adds the partials in a fixed order (deterministic) and nu^2 X.
#include <map>
#include <mutex>
#include <tuple>
#include <type_traits>
#include <vector>

#include "rs_internal.hpp"

namespace rs {

// wave_sum's butterfly (xor 32, 16, 8, 4, 2, 1, in that order) with the four
// in-row stages as DPP moves instead of LDS permutes.  xor 8 is row_ror:8 and xor
// 2, xor 1 are quad permutes (the same partners); row_ror:4 takes lane p +- 4 in
// place of p ^ 4, and after the xor-8 stage lanes 8 apart hold the same bits, so
// the operands, and every lane's result, are wave_sum's bit for bit.
__device__ __forceinline__ float wave_sum_dpp(float v) {
  v += __shfl_xor(v, 32, 64);
  v += __shfl_xor(v, 16, 64);
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x128,
                                                              0xF, 0xF, false));  // row_ror:8
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x124,
                                                              0xF, 0xF, false));  // row_ror:4
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x4E,
                                                              0xF, 0xF, false));  // [2,3,0,1]
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xB1,
                                                              0xF, 0xF, false));  // [1,0,3,2]
  return v;
}

// S wave sums at once (S a power of two, at least 4) with wave_sum's pairings: the
// xor-32 and xor-16 stages are transposed (a lane keeps half of its values and hands
// the other half to its partner, which keeps the mirror half), so they take S/2 + S/4
// permutes instead of 2 S; the in-row stages then run on the S/4 values left, as in
// wave_sum_dpp.  Every sum adds the same lane pairs in the same order as wave_sum,
// so its bits are wave_sum's.  On return v[u] (u < S/4) of lane L holds the sum of
// value (L >> 4) * (S/4) + u, the same bits in all 16 lanes of L's row.
template <int S>
__device__ __forceinline__ void wave_sums_t(float (&v)[S]) {
  static_assert(S >= 4 && (S & (S - 1)) == 0, "S: a power of two >= 4");
  const int lane = threadIdx.x & 63;
  const bool h5 = (lane & 32) != 0, h4 = (lane & 16) != 0;
  float a[S / 2];
#pragma unroll
  for (int u = 0; u < S / 2; ++u) {
    const float send = h5 ? v[u] : v[u + S / 2];
    const float keep = h5 ? v[u + S / 2] : v[u];
    a[u] = keep + __shfl_xor(send, 32, 64);
  }
#pragma unroll
  for (int u = 0; u < S / 4; ++u) {
    const float send = h4 ? a[u] : a[u + S / 4];
    const float keep = h4 ? a[u + S / 4] : a[u];
    float c = keep + __shfl_xor(send, 16, 64);
    c += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, c),
                                                                0x128, 0xF, 0xF, false));
    c += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, c),
                                                                0x124, 0xF, 0xF, false));
    c += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, c),
                                                                0x4E, 0xF, 0xF, false));
    c += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, c),
                                                                0xB1, 0xF, 0xF, false));
    v[u] = c;
  }
}

// group_sum<W> (W = 16 or 32) with its in-row stages as DPP moves, as in
// wave_sum_dpp: the same lane pairs, the same bits in every lane of the group.
template <int W>
__device__ __forceinline__ float group_sum_dpp(float v) {
  static_assert(W == 16 || W == 32, "W: 16 or 32");
  if constexpr (W == 32) v += __shfl_xor(v, 16, 64);
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x128,
                                                              0xF, 0xF, false));  // row_ror:8
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x124,
                                                              0xF, 0xF, false));  // row_ror:4
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x4E,
                                                              0xF, 0xF, false));  // [2,3,0,1]
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0xB1,
                                                              0xF, 0xF, false));  // [1,0,3,2]
  return v;
}

template <typename T, int TPR, int NV, int K, int R>
__global__ __launch_bounds__(256) void k_grad_partial(const T* __restrict__ A, int64_t n, int64_t d,
                                                      int64_t lda, const T* __restrict__ b,
                                                      const double* __restrict__ X,
                                                      int64_t rows_per_block, int iters,
                                                      double* __restrict__ partial,
                                                      const int* __restrict__ status,
                                                      int* __restrict__ ran) {
  if (status && *status != 0) return;
  if (ran && blockIdx.x == 0 && threadIdx.x == 0) *ran = 1;
  using V = typename VecOf<T>::type;
  constexpr int VEC = VecOf<T>::n;
  constexpr int GPB = 256 / TPR;          // row groups per block
  constexpr int WPG = TPR > 64 ? TPR / 64 : 1;  // waves per group
  __shared__ double red_acc[256 * NV * VEC > 4096 ? 4096 : 256 * NV * VEC];
  __shared__ T red_dot[2][GPB][WPG][R * K];

  const int tid = threadIdx.x;
  const int grp = tid / TPR;
  const int lt = tid % TPR;
  const int64_t row0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t row1 = row0 + rows_per_block < n ? row0 + rows_per_block : n;

  // x in registers (T precision); loads are unconditional from clamped
  // in-bounds addresses and masked afterwards, so they all stay in flight
  T xv[K][NV][VEC];
  bool colok[NV][VEC];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const int64_t c = (int64_t)(lt + TPR * v) * VEC + e;
      colok[v][e] = c < d;
      const int64_t cc = c < d ? c : 0;
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const T xval = (T)X[k * d + cc];
        xv[k][v][e] = colok[v][e] ? xval : (T)0;
      }
    }
  }
  double acc[K][NV][VEC];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[k][v][e] = 0.0;

  for (int it = 0; it < iters; ++it) {
    const int64_t base = row0 + ((int64_t)it * GPB + grp) * R;
    V a[R][NV];
    T bv[R];
    bool rok[R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int64_t row = base + i;
      rok[i] = row < row1;
      const int64_t rowc = row < n ? row : n - 1;
      bv[i] = b[rowc];
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int64_t c = (int64_t)(lt + TPR * v) * VEC;
        const int64_t cc = c < d ? c : 0;
        a[i][v] = *reinterpret_cast<const V*>(A + rowc * lda + cc);
      }
    }
    // mask rows past the block and columns past d (a vector may straddle d)
#pragma unroll
    for (int i = 0; i < R; ++i) {
      bv[i] = rok[i] ? bv[i] : (T)0;
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const T val = get(a[i][v], e);
          set(a[i][v], e, (rok[i] && colok[v][e]) ? val : (T)0);
        }
    }

    T s[R][K];
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        T t = 0;
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
          for (int e = 0; e < VEC; ++e) t = fma(get(a[i][v], e), xv[k][v][e], t);
        s[i][k] = t;
      }
    // reduce the row dots over the TPR threads of the group.  FP32: DPP for the
    // in-row stages, and where the R K dots of a wave form a power of two of at
    // least 4 they are reduced together (wave_sums_t); the lane pairs are those of
    // group_sum / wave_sum, so the bits are too
    constexpr int S = R * K;
    constexpr bool kF32 = std::is_same<T, float>::value;
    // (k <= 2: with four right-hand sides the wider shapes have no registers to spare)
    constexpr bool kTrans = kF32 && K <= 2 && S >= 4 && (S & (S - 1)) == 0;
    if constexpr (TPR <= 64) {
      if constexpr (kF32 && TPR == 64 && kTrans) {
        float dots[S];
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
          for (int k = 0; k < K; ++k) dots[i * K + k] = s[i][k];
        wave_sums_t<S>(dots);
        // lane 16 h holds dots h S/4 .. h S/4 + S/4 - 1: every lane takes all of them
#pragma unroll
        for (int q = 0; q < S; ++q)
          s[q / K][q % K] = __builtin_bit_cast(
              float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, dots[q % (S / 4)]),
                                               (q / (S / 4)) * 16));
      } else if constexpr (kF32 && TPR == 64) {
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
          for (int k = 0; k < K; ++k) s[i][k] = wave_sum_dpp(s[i][k]);
      } else if constexpr (kF32 && (TPR == 16 || TPR == 32)) {
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
          for (int k = 0; k < K; ++k) s[i][k] = group_sum_dpp<TPR>(s[i][k]);
      } else {
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
          for (int k = 0; k < K; ++k) s[i][k] = group_sum<TPR>(s[i][k]);
      }
    } else {
      const int w = lt / 64;
      const int buf = it & 1;
      if constexpr (kTrans) {
        float dots[S];
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
          for (int k = 0; k < K; ++k) dots[i * K + k] = s[i][k];
        wave_sums_t<S>(dots);
        if ((lt & 15) == 0) {
#pragma unroll
          for (int u = 0; u < S / 4; ++u) red_dot[buf][grp][w][((lt & 63) >> 4) * (S / 4) + u] = dots[u];
        }
      } else {
#pragma unroll
        for (int i = 0; i < R; ++i)
#pragma unroll
          for (int k = 0; k < K; ++k) {
            T t;
            if constexpr (kF32) t = wave_sum_dpp(s[i][k]);
            else t = wave_sum(s[i][k]);
            if ((lt & 63) == 0) red_dot[buf][grp][w][i * K + k] = t;
          }
      }
      __syncthreads();
#pragma unroll
      for (int i = 0; i < R; ++i)
#pragma unroll
        for (int k = 0; k < K; ++k) {
          T t = 0;
#pragma unroll
          for (int ww = 0; ww < WPG; ++ww) t += red_dot[buf][grp][ww][i * K + k];
          s[i][k] = t;
        }
    }
    // A^T r for the R rows: T sums, then FP64 accumulation
#pragma unroll
    for (int k = 0; k < K; ++k) {
      T res[R];
#pragma unroll
      for (int i = 0; i < R; ++i) res[i] = s[i][k] - bv[i];
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          T t = 0;
#pragma unroll
          for (int i = 0; i < R; ++i) t = fma(get(a[i][v], e), res[i], t);
          acc[k][v][e] += (double)t;
        }
    }
  }

  // combine the row groups of the block in a fixed order, one RHS at a time
  constexpr int COLS = TPR * NV * VEC;  // columns covered by one group
  for (int k = 0; k < K; ++k) {
    if constexpr (GPB == 1) {
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const int64_t c = (int64_t)(lt + TPR * v) * VEC + e;
          if (c < d) partial[((int64_t)blockIdx.x * K + k) * d + c] = acc[k][v][e];
        }
    } else {
      // red_acc holds GPB * COLS doubles when that fits 4096, else groups pass
      // through it in rounds
      constexpr int GR = (GPB * COLS <= 4096) ? GPB : (4096 / COLS);
      double sum[NV][VEC];
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int e = 0; e < VEC; ++e) sum[v][e] = 0.0;
      for (int g0 = 0; g0 < GPB; g0 += GR) {
        __syncthreads();
        if (grp >= g0 && grp < g0 + GR) {
#pragma unroll
          for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int e = 0; e < VEC; ++e)
              red_acc[(grp - g0) * COLS + (lt + TPR * v) * VEC + e] = acc[k][v][e];
        }
        __syncthreads();
        if (grp == 0) {
#pragma unroll
          for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int e = 0; e < VEC; ++e)
              for (int gg = 0; gg < GR && g0 + gg < GPB; ++gg)
                sum[v][e] += red_acc[gg * COLS + (lt + TPR * v) * VEC + e];
        }
      }
      if (grp == 0) {
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
          for (int e = 0; e < VEC; ++e) {
            const int64_t c = (int64_t)(lt + TPR * v) * VEC + e;
            if (c < d) partial[((int64_t)blockIdx.x * K + k) * d + c] = sum[v][e];
          }
      }
    }
  }
}

// Wide rows (FP32, up to 512 * NV * 4 columns): one row group per block of 512
// threads, thread lt holding the 16-byte vectors lt + 512 v (v < NV) of every row,
// R rows per step.  The rows of step s + 1 are loaded into a second register set
// while step s is reduced and accumulated, so the pass keeps a step of A in flight
// at all times.  Loads go through a buffer descriptor over the block's rows (row
// offset as the scalar offset, column offset as the 32-bit lane offset).  Row dots
// are reduced over the 8 waves through LDS (two buffers, one barrier per step); the
// A^T r products of a step's R rows are summed in FP32 and added to FP64
// accumulators, as in k_grad_partial.
template <int K, int NV, int R>
__global__ __launch_bounds__(512) void k_grad_wide(const float* __restrict__ A, int64_t n,
                                                   int64_t d, int64_t lda,
                                                   const float* __restrict__ b,
                                                   const double* __restrict__ X,
                                                   int64_t rows_per_block, int iters,
                                                   double* __restrict__ partial,
                                                   const int* __restrict__ status,
                                                   int* __restrict__ ran) {
  if (status && *status != 0) return;
  if (ran && blockIdx.x == 0 && threadIdx.x == 0) *ran = 1;
  constexpr int NW = 8;  // waves per block
  __shared__ float red[2][NW][R * K];
  const int lt = threadIdx.x;
  const int w = lt >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t row1 = row0 + rows_per_block < n ? row0 + rows_per_block : n;
  if (row0 >= row1) {  // an empty block still writes its (zero) partial
    for (int k = 0; k < K; ++k)
      for (int v = 0; v < NV; ++v)
        for (int e = 0; e < 4; ++e) {
          const int64_t c = (int64_t)(lt + 512 * v) * 4 + e;
          if (c < d) partial[((int64_t)blockIdx.x * K + k) * d + c] = 0.0;
        }
    return;
  }
  // x in registers; columns past d get x = 0 and their A values are zeroed
  float xv[K][NV][4];
  uint32_t coff[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int64_t c0 = (int64_t)(lt + 512 * v) * 4;
    coff[v] = (uint32_t)((c0 < d ? c0 : 0) * 4);
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int64_t c = c0 + e;
#pragma unroll
      for (int k = 0; k < K; ++k) xv[k][v][e] = c < d ? (float)X[k * d + c] : 0.0f;
    }
  }
  double acc[K][NV][4];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[k][v][e] = 0.0;
  const uint32_t rowb = (uint32_t)(lda * 4);
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(A + row0 * lda), (short)0, (int)(rowb * (uint32_t)(row1 - row0)),
      0x00020000);
  const int64_t nrows = row1 - row0;
  // rows of a step past the block's range repeat its last row (uniform) and count 0
  auto load = [&](float4 (&a)[R][NV], int step) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      int64_t r = (int64_t)step * R + i;
      r = r < nrows ? r : nrows - 1;
#pragma unroll
      for (int v = 0; v < NV; ++v)
        a[i][v] = __builtin_bit_cast(
            float4, __builtin_amdgcn_raw_buffer_load_b128(rs, coff[v], (uint32_t)r * rowb, 0));
    }
  };
  // MASK: zero A values past d (padding columns may hold anything); a d that fills
  // every thread's columns runs the loop without the selects
  auto process = [&](float4 (&a)[R][NV], int step, auto mask) {
    const int buf = step & 1;
    if constexpr (decltype(mask)::value) {
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const bool ok = (int64_t)(lt + 512 * v) * 4 + e < d;
#pragma unroll
          for (int i = 0; i < R; ++i) set(a[i][v], e, ok ? get(a[i][v], e) : 0.0f);
        }
    }
    float dots[R * K];  // dot i * K + k
#pragma unroll
    for (int i = 0; i < R; ++i)
#pragma unroll
      for (int k = 0; k < K; ++k) {
        float t = 0.0f;
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
          for (int e = 0; e < 4; ++e) t = fmaf(get(a[i][v], e), xv[k][v][e], t);
        dots[i * K + k] = t;
      }
    if constexpr (R * K >= 4 && (R * K & (R * K - 1)) == 0) {
      wave_sums_t<R * K>(dots);
      if ((lt & 15) == 0) {
#pragma unroll
        for (int u = 0; u < R * K / 4; ++u)
          red[buf][w][((lt & 63) >> 4) * (R * K / 4) + u] = dots[u];
      }
    } else {
#pragma unroll
      for (int q = 0; q < R * K; ++q) {
        const float t = wave_sum_dpp(dots[q]);
        if ((lt & 63) == 0) red[buf][w][q] = t;
      }
    }
    __syncthreads();
    // lane q < R K of each wave adds the NW wave partials of dot q in wave order;
    // readlane hands the sums to the whole wave
    float mine = 0.0f;
    if ((lt & 63) < R * K) {
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) mine += red[buf][ww][lt & 63];
    }
    float res[K][R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int64_t r = (int64_t)step * R + i;
      const bool live = r < nrows;
      const float bi = b[row0 + (live ? r : 0)];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const float t = __builtin_bit_cast(
            float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, mine), i * K + k));
        res[k][i] = live ? t - bi : 0.0f;
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          float t = 0.0f;
#pragma unroll
          for (int i = 0; i < R; ++i) t = fmaf(get(a[i][v], e), res[k][i], t);
          acc[k][v][e] += (double)t;
        }
  };
  auto run = [&](auto mask) {
    float4 a0[R][NV], a1[R][NV];
    load(a0, 0);
    for (int it = 0; it < iters; it += 2) {
      if (it + 1 < iters) load(a1, it + 1);
      process(a0, it, mask);
      if (it + 1 >= iters) break;
      if (it + 2 < iters) load(a0, it + 2);
      process(a1, it + 1, mask);
    }
  };
  if (d >= (int64_t)2048 * NV)
    run(std::false_type{});
  else
    run(std::true_type{});
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int64_t c = (int64_t)(lt + 512 * v) * 4 + e;
        if (c < d) partial[((int64_t)blockIdx.x * K + k) * d + c] = acc[k][v][e];
      }
}

// Two problems that share A and b (two nu, or two starts), each with two columns:
// one read of A serves both.  Each job's columns get exactly the arithmetic of
// k_grad_wide<2, NV, R> on the same grid (the same products in the same order, wave
// and block sums, FP64 accumulation), so its partial sums are those of its own pass.
// Four columns of x in registers would not fit beside the FP64 sums, so x sits in
// LDS: thread lt keeps its columns there and reads back only its own entries (no
// barrier needed for them).  A job whose status flag is raised gets no partial sums
// written (its finish returns at once too); both raised: the block returns.
template <int NV, int R>
__global__ __launch_bounds__(512) void k_grad_wide_two(
    const float* __restrict__ A, int64_t n, int64_t d, int64_t lda, const float* __restrict__ b,
    const double* __restrict__ X0, const double* __restrict__ X1, int64_t rows_per_block,
    int iters, double* __restrict__ partial0, double* __restrict__ partial1,
    const int* __restrict__ status0, const int* __restrict__ status1, int* __restrict__ ran) {
  constexpr int K = 4;  // job 0: columns 0, 1; job 1: columns 2, 3
  const bool live0 = !status0 || *status0 == 0;
  const bool live1 = !status1 || *status1 == 0;
  if (!live0 && !live1) return;
  if (ran && blockIdx.x == 0 && threadIdx.x == 0) *ran = 1;
  constexpr int NW = 8;
  __shared__ float red[2][NW][R * K];
  __shared__ float4 xs[K][NV][512];
  const int lt = threadIdx.x;
  const int w = lt >> 6;
  const int64_t row0 = (int64_t)blockIdx.x * rows_per_block;
  const int64_t row1 = row0 + rows_per_block < n ? row0 + rows_per_block : n;
  auto put = [&](int k, int v, int e, double val) {
    const int64_t c = (int64_t)(lt + 512 * v) * 4 + e;
    if (c >= d) return;
    if (k < 2) {
      if (live0) partial0[((int64_t)blockIdx.x * 2 + k) * d + c] = val;
    } else if (live1) {
      partial1[((int64_t)blockIdx.x * 2 + (k - 2)) * d + c] = val;
    }
  };
  if (row0 >= row1) {
    for (int k = 0; k < K; ++k)
      for (int v = 0; v < NV; ++v)
        for (int e = 0; e < 4; ++e) put(k, v, e, 0.0);
    return;
  }
  uint32_t coff[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int64_t c0 = (int64_t)(lt + 512 * v) * 4;
    coff[v] = (uint32_t)((c0 < d ? c0 : 0) * 4);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const double* X = k < 2 ? X0 + (int64_t)k * d : X1 + (int64_t)(k - 2) * d;
      float4 xv;
#pragma unroll
      for (int e = 0; e < 4; ++e) set(xv, e, c0 + e < d ? (float)X[c0 + e] : 0.0f);
      xs[k][v][lt] = xv;
    }
  }
  double acc[K][NV][4];
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[k][v][e] = 0.0;
  const uint32_t rowb = (uint32_t)(lda * 4);
  const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(A + row0 * lda), (short)0, (int)(rowb * (uint32_t)(row1 - row0)),
      0x00020000);
  const int64_t nrows = row1 - row0;
  auto load = [&](float4 (&a)[R][NV], int step) {
#pragma unroll
    for (int i = 0; i < R; ++i) {
      int64_t r = (int64_t)step * R + i;
      r = r < nrows ? r : nrows - 1;
#pragma unroll
      for (int v = 0; v < NV; ++v)
        a[i][v] = __builtin_bit_cast(
            float4, __builtin_amdgcn_raw_buffer_load_b128(rs, coff[v], (uint32_t)r * rowb, 0));
    }
  };
  // MASK: some of the thread's columns lie past d (zeroed); a d that fills every
  // thread's columns runs the loop without the selects
  auto process = [&](float4 (&a)[R][NV], int step, auto mask) {
    const int buf = step & 1;
    if constexpr (decltype(mask)::value) {
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const bool ok = (int64_t)(lt + 512 * v) * 4 + e < d;
#pragma unroll
          for (int i = 0; i < R; ++i) set(a[i][v], e, ok ? get(a[i][v], e) : 0.0f);
        }
    }
    float dots[R * K];  // dot i * K + k
#pragma unroll
    for (int k = 0; k < K; ++k) {
      float4 xk[NV];
#pragma unroll
      for (int v = 0; v < NV; ++v) xk[v] = xs[k][v][lt];
#pragma unroll
      for (int i = 0; i < R; ++i) {
        float t = 0.0f;
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
          for (int e = 0; e < 4; ++e) t = fmaf(get(a[i][v], e), get(xk[v], e), t);
        dots[i * K + k] = t;
      }
    }
    wave_sums_t<R * K>(dots);
    if ((lt & 15) == 0) {
#pragma unroll
      for (int u = 0; u < R * K / 4; ++u) red[buf][w][((lt & 63) >> 4) * (R * K / 4) + u] = dots[u];
    }
    __syncthreads();
    // lane q < R K of each wave adds the NW wave partials of dot q (in wave order,
    // as every lane does in k_grad_wide); readlane hands the sums to the whole wave
    float mine = 0.0f;
    if ((lt & 63) < R * K) {
#pragma unroll
      for (int ww = 0; ww < NW; ++ww) mine += red[buf][ww][lt & 63];
    }
    float res[K][R];
#pragma unroll
    for (int i = 0; i < R; ++i) {
      const int64_t r = (int64_t)step * R + i;
      const bool live = r < nrows;
      const float bi = b[row0 + (live ? r : 0)];
#pragma unroll
      for (int k = 0; k < K; ++k) {
        const float t = __builtin_bit_cast(
            float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, mine), i * K + k));
        res[k][i] = live ? t - bi : 0.0f;
      }
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
#pragma unroll
      for (int v = 0; v < NV; ++v)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          float t = 0.0f;
#pragma unroll
          for (int i = 0; i < R; ++i) t = fmaf(get(a[i][v], e), res[k][i], t);
          acc[k][v][e] += (double)t;
        }
  };
  auto run = [&](auto mask) {
    float4 a0[R][NV], a1[R][NV];
    load(a0, 0);
    for (int it = 0; it < iters; it += 2) {
      if (it + 1 < iters) load(a1, it + 1);
      process(a0, it, mask);
      if (it + 1 >= iters) break;
      if (it + 2 < iters) load(a0, it + 2);
      process(a1, it + 1, mask);
    }
  };
  if (d >= (int64_t)2048 * NV)
    run(std::false_type{});
  else
    run(std::true_type{});
#pragma unroll
  for (int k = 0; k < K; ++k)
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int e = 0; e < 4; ++e) put(k, v, e, acc[k][v][e]);
}

// G[k][j] = sum over blocks of partial[b][k][j] (fixed order) + nu2 X[k][j] - sub[j]
// (sub null: 0; the dual problem's gradient carries -b there).
// Block: 8 columns x 32 block-strides; LDS tree over the 32 strides.
__global__ __launch_bounds__(256) void k_grad_finish(const double* __restrict__ partial, int nblk,
                                                     int64_t kd, double nu2,
                                                     const double* __restrict__ X,
                                                     double* __restrict__ G,
                                                     const int* __restrict__ status,
                                                     const double* __restrict__ sub, int64_t d) {
  if (status && *status != 0) return;
  __shared__ double s[32][8];
  const int cl = threadIdx.x & 7;
  const int rs_ = threadIdx.x >> 3;
  const int64_t c = (int64_t)blockIdx.x * 8 + cl;
  double t = 0.0;
  if (c < kd)
    for (int b = rs_; b < nblk; b += 32) t += partial[(int64_t)b * kd + c];
  s[rs_][cl] = t;
  __syncthreads();
  if (threadIdx.x < 8) {
    double u = 0.0;
    for (int r = 0; r < 32; ++r) u += s[r][threadIdx.x];
    const int64_t cc = (int64_t)blockIdx.x * 8 + threadIdx.x;
    if (cc < kd) G[cc] = sub ? u + nu2 * X[cc] - sub[cc % d] : u + nu2 * X[cc];
  }
}

namespace {

struct GradShape {
  int tpr, nv, r;  // threads per row, vectors per thread, rows per group and step (0: default)
};

template <typename T>
GradShape pick_shape(int64_t d) {
  constexpr int VEC = VecOf<T>::n;
  const int64_t chunks = (d + VEC - 1) / VEC;  // 16-byte vectors per row
  if (chunks <= 16) return {16, 1, 0};
  if (chunks <= 64) return {64, 1, 0};
  if (chunks <= 128) return {64, 2, 0};
  if (chunks <= 256) return {64, 4, 0};
  if (chunks <= 512) return {128, 4, 0};
  if (chunks <= 1024) return {256, 4, 0};
  if (chunks <= 2048) return {256, 8, 0};
  return {0, 0, 0};
}

constexpr int default_rows(int nv) { return nv >= 8 ? 2 : (nv >= 4 ? 4 : 8); }

template <typename T, int TPR, int NV, int K, int R>
void launch_partial(const T* A, int64_t n, int64_t d, int64_t lda, const T* b, const double* X,
                    double* partial, int grid, int64_t rpb, const int* status, hipStream_t s,
                    bool prof) {
  constexpr int GPB = 256 / TPR;
  const int iters = (int)((rpb + GPB * R - 1) / (GPB * R));
  const ProfSlot ps = prof ? prof_begin() : ProfSlot();
  launch_timed(k_grad_partial<T, TPR, NV, K, R>, dim3(grid), dim3(256), s, ps.begin, ps.end, A, n,
               d, lda, b, X, rpb, iters, partial, status, ps.ran);
}

template <int K, int NV, int R>
void launch_wide(const float* A, int64_t n, int64_t d, int64_t lda, const float* b,
                 const double* X, double* partial, int grid, int64_t rpb, const int* status,
                 hipStream_t s, bool prof) {
  const int iters = (int)((rpb + R - 1) / R);
  const ProfSlot ps = prof ? prof_begin() : ProfSlot();
  launch_timed(k_grad_wide<K, NV, R>, dim3(grid), dim3(512), s, ps.begin, ps.end, A, n, d, lda,
               b, X, rpb, iters, partial, status, ps.ran);
}

template <typename T, int K>
bool dispatch_k(GradShape sh, const T* A, int64_t n, int64_t d, int64_t lda, const T* b,
                const double* X, double* partial, int grid, int64_t rpb, const int* status,
                hipStream_t s, bool prof = true) {
#define RS_GCASE(TP, NVV, RR)                                                                \
  if (sh.tpr == TP && sh.nv == NVV && (sh.r == RR || (sh.r == 0 && RR == default_rows(NVV)))) { \
    launch_partial<T, TP, NVV, K, RR>(A, n, d, lda, b, X, partial, grid, rpb, status, s, prof); \
    return true;                                                                             \
  }
  RS_GCASE(16, 1, 8) RS_GCASE(64, 1, 8) RS_GCASE(64, 2, 8) RS_GCASE(64, 4, 4) RS_GCASE(128, 4, 4)
  RS_GCASE(256, 4, 4) RS_GCASE(256, 8, 2)
  // deeper row batches (more loads in flight per step), offered to the autotuner
  RS_GCASE(64, 4, 8) RS_GCASE(128, 4, 8) RS_GCASE(256, 4, 8) RS_GCASE(256, 8, 4)
#undef RS_GCASE
  // 512 threads per row (FP32 only; the block's rows addressed with 32-bit offsets)
  if constexpr (sizeof(T) == 4) {
    if (sh.tpr == 512 && rpb * lda * 4 < ((int64_t)1 << 31)) {
#define RS_WCASE(NVV, RR)                                                                   \
  if (sh.nv == NVV && sh.r == RR) {                                                        \
    launch_wide<K, NVV, RR>(A, n, d, lda, b, X, partial, grid, rpb, status, s, prof);       \
    return true;                                                                           \
  }
      RS_WCASE(4, 2) RS_WCASE(2, 4)
#undef RS_WCASE
    }
  }
  return false;
}

}  // namespace

int grad_partial_blocks(int64_t n) {
  const int64_t target = (int64_t)device_cus() * 2;
  int64_t g = n / 64;
  if (g < 1) g = 1;
  return (int)(g < target ? g : target);
}

int grad_partial_blocks_max(int64_t n) {
  const int64_t target = (int64_t)device_cus() * 4;
  int64_t g = n / 64;
  if (g < 1) g = 1;
  return (int)(g < target ? g : target);
}

// ---------------------------------------------------------------- plans and autotuning
// A plan is the (threads per row, vectors per thread) shape and the grid of the
// partial-sum kernel.  Without tuning the shape follows d and the grid is two
// blocks per CU; rs_gradient_autotune times every instantiated shape that covers d
// (up to 4x the row) at 1, 2 and 4 blocks per CU on the caller's problem and keeps
// the fastest for (type, n rounded up to a power of two, d, k).
namespace {

using PlanKey = std::tuple<int, int64_t, int64_t, int>;
std::mutex g_plan_mu;
std::map<PlanKey, GradPlan> g_plans;

int64_t pow2_ceil(int64_t v) {
  int64_t p = 1;
  while (p < v) p <<= 1;
  return p;
}

const GradShape kShapes[] = {{16, 1, 8},  {64, 1, 8},  {64, 2, 8},  {64, 4, 4},
                             {128, 4, 4}, {256, 4, 4}, {256, 8, 2}, {64, 4, 8},
                             {128, 4, 8}, {256, 4, 8}, {256, 8, 4}, {512, 4, 2},
                             {512, 2, 4}};

}  // namespace

template <typename T>
GradPlan grad_plan(int64_t n, int64_t d, int k) {
  {
    std::lock_guard<std::mutex> g(g_plan_mu);
    auto it = g_plans.find(PlanKey{(int)sizeof(T), pow2_ceil(n), d, k});
    if (it != g_plans.end()) return it->second;
  }
  const GradShape sh = pick_shape<T>(d);
  return GradPlan{sh.tpr, sh.nv, grad_partial_blocks(n), default_rows(sh.nv)};
}

template <typename T>
static bool launch_plan(const GradPlan& pl, const T* A, int64_t n, int64_t d, int64_t lda,
                        const T* b, const double* X, int k, double* partial, const int* status,
                        hipStream_t s, bool prof = true) {
  const GradShape sh{pl.tpr, pl.nv, pl.r};
  const int64_t rpb = (n + pl.grid - 1) / pl.grid;
  switch (k) {
    case 1: return dispatch_k<T, 1>(sh, A, n, d, lda, b, X, partial, pl.grid, rpb, status, s, prof);
    case 2: return dispatch_k<T, 2>(sh, A, n, d, lda, b, X, partial, pl.grid, rpb, status, s, prof);
    case 3: return dispatch_k<T, 3>(sh, A, n, d, lda, b, X, partial, pl.grid, rpb, status, s, prof);
    case 4: return dispatch_k<T, 4>(sh, A, n, d, lda, b, X, partial, pl.grid, rpb, status, s, prof);
  }
  return false;
}

template <typename T>
rs_status gradient_launch(const T* A, int64_t n, int64_t d, int64_t lda, const T* b, double nu2,
                          const double* X, int k, double* G, double* partial, int grid_cap,
                          const int* status, hipStream_t s, const double* c, bool prof) {
  if (k < 1 || k > 4) return set_error(RS_ERR_ARG, "gradient: k must be in 1..4");
  GradPlan pl = grad_plan<T>(n, d, k);
  if (pl.tpr == 0) return set_error(RS_ERR_UNSUPPORTED, "gradient: d above the widest gradient kernel");
  if (pl.grid > grid_cap) pl.grid = grid_cap;
  if (!launch_plan<T>(pl, A, n, d, lda, b, X, k, partial, status, s, prof)) {
    // a plan this call cannot use (e.g. the wide kernel's 32-bit row offsets for a
    // larger leading dimension): the default shape for d
    const GradShape sh = pick_shape<T>(d);
    pl = GradPlan{sh.tpr, sh.nv, std::min(grad_partial_blocks(n), grid_cap), default_rows(sh.nv)};
    if (!launch_plan<T>(pl, A, n, d, lda, b, X, k, partial, status, s, prof))
      return set_error(RS_ERR_UNSUPPORTED, "gradient: no kernel for this shape");
  }
  const int64_t kd = (int64_t)k * d;
  hipLaunchKernelGGL(k_grad_finish, dim3((unsigned)((kd + 7) / 8)), dim3(256), 0, s, partial,
                     pl.grid, kd, nu2, X, G, status, c, d);
  return check_launch("gradient");
}

bool gradient_two_fits(int64_t n, int64_t d, int64_t lda, int grid_cap) {
  GradPlan pl = grad_plan<float>(n, d, 2);
  if (pl.grid > grid_cap) pl.grid = grid_cap;
  const int64_t rpb = (n + pl.grid - 1) / pl.grid;
  return pl.tpr == 512 && ((pl.nv == 4 && pl.r == 2) || (pl.nv == 2 && pl.r == 4)) &&
         rpb * lda * 4 < ((int64_t)1 << 31);
}

rs_status gradient_two_launch(const float* A, int64_t n, int64_t d, int64_t lda, const float* b,
                              const double* nu2, const double* const* X, double* const* G,
                              double* const* partial, int grid_cap, const int* const* status,
                              hipStream_t s) {
  if (!gradient_two_fits(n, d, lda, grid_cap))
    return set_error(RS_ERR_UNSUPPORTED, "gradient: no two-job kernel for this plan");
  GradPlan pl = grad_plan<float>(n, d, 2);
  if (pl.grid > grid_cap) pl.grid = grid_cap;
  const int64_t rpb = (n + pl.grid - 1) / pl.grid;
  const int iters = (int)((rpb + pl.r - 1) / pl.r);
  const ProfSlot ps = prof_begin();
  if (pl.nv == 4)
    launch_timed(k_grad_wide_two<4, 2>, dim3(pl.grid), dim3(512), s, ps.begin, ps.end, A, n, d,
                 lda, b, X[0], X[1], rpb, iters, partial[0], partial[1], status[0], status[1],
                 ps.ran);
  else
    launch_timed(k_grad_wide_two<2, 4>, dim3(pl.grid), dim3(512), s, ps.begin, ps.end, A, n, d,
                 lda, b, X[0], X[1], rpb, iters, partial[0], partial[1], status[0], status[1],
                 ps.ran);
  const int64_t kd = 2 * d;
  for (int j = 0; j < 2; ++j)
    hipLaunchKernelGGL(k_grad_finish, dim3((unsigned)((kd + 7) / 8)), dim3(256), 0, s, partial[j],
                       pl.grid, kd, nu2[j], X[j], G[j], status[j], (const double*)nullptr, d);
  return check_launch("gradient (two jobs)");
}

template <typename T>
rs_status gradient_autotune(const T* A, int64_t n, int64_t d, int64_t lda, const T* b,
                            const double* X, int k, double* G, double* partial, int grid_cap,
                            hipStream_t s, GradPlan* chosen) {
  if (k < 1 || k > 4) return set_error(RS_ERR_ARG, "autotune: k must be in 1..4");
  constexpr int VEC = VecOf<T>::n;
  const int64_t row = (d + VEC - 1) / VEC;
  std::vector<GradPlan> cand;
  for (const GradShape& sh : kShapes) {
    const int64_t cover = (int64_t)sh.tpr * sh.nv;
    if (cover < row || cover > 4 * std::max<int64_t>(row, 16)) continue;
    if (sh.tpr == 512 && sizeof(T) != 4) continue;  // the wide kernel is FP32 only
    for (int f : {1, 2, 4}) {
      int g = (int)std::min<int64_t>((int64_t)device_cus() * f, std::max<int64_t>(n / 64, 1));
      g = std::min(g, grid_cap);
      if (sh.tpr == 512 && (n + g - 1) / g * lda * 4 >= ((int64_t)1 << 31)) continue;
      bool dup = false;
      for (const GradPlan& c : cand)
        dup |= (c.tpr == sh.tpr && c.nv == sh.nv && c.grid == g && c.r == sh.r);
      if (!dup) cand.push_back(GradPlan{sh.tpr, sh.nv, g, sh.r});
    }
  }
  if (cand.empty()) return set_error(RS_ERR_UNSUPPORTED, "autotune: d above the widest gradient kernel");
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
    return set_error(RS_ERR_HIP, "autotune: event creation failed");
  GradPlan best = cand[0];
  float best_ms = 1e30f;
  rs_status st = RS_OK;
  for (const GradPlan& c : cand) {
    const int64_t kd = (int64_t)k * d;
    auto once = [&]() {
      launch_plan<T>(c, A, n, d, lda, b, X, k, partial, nullptr, s);
      hipLaunchKernelGGL(k_grad_finish, dim3((unsigned)((kd + 7) / 8)), dim3(256), 0, s, partial,
                         c.grid, kd, 0.0, X, G, (const int*)nullptr, (const double*)nullptr, d);
    };
    once();
    float ms = 1e30f;
    for (int r = 0; r < 3; ++r) {
      (void)hipEventRecord(e0, s);
      once();
      (void)hipEventRecord(e1, s);
      if (hipEventSynchronize(e1) != hipSuccess) { st = set_error(RS_ERR_HIP, "autotune: sync"); break; }
      float t = 0.0f;
      (void)hipEventElapsedTime(&t, e0, e1);
      ms = std::min(ms, t);
    }
    if (st != RS_OK) break;
    if (ms < best_ms) { best_ms = ms; best = c; }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st != RS_OK) return st;
  {
    std::lock_guard<std::mutex> g(g_plan_mu);
    g_plans[PlanKey{(int)sizeof(T), pow2_ceil(n), d, k}] = best;
  }
  if (chosen) *chosen = best;
  return check_launch("autotune");
}

// A caller-chosen plan for a key: the shape must be one of the built ones and cover
// the row of d columns (at most 4x over), the grid at least 1 block.
template <typename T>
rs_status gradient_set_plan(int64_t n, int64_t d, int k, const GradPlan& pl) {
  constexpr int VEC = VecOf<T>::n;
  const int64_t row = (d + VEC - 1) / VEC;
  bool built = false;
  for (const GradShape& sh : kShapes)
    built |= sh.tpr == pl.tpr && sh.nv == pl.nv && sh.r == pl.r;
  if (!built || (pl.tpr == 512 && sizeof(T) != 4))
    return set_error(RS_ERR_UNSUPPORTED, "gradient plan: shape not built");
  const int64_t cover = (int64_t)pl.tpr * pl.nv;
  if (cover < row || cover > 4 * std::max<int64_t>(row, 16))
    return set_error(RS_ERR_SHAPE, "gradient plan: shape does not fit this d");
  if (pl.grid < 1 || pl.grid > grad_partial_blocks_max(n))
    return set_error(RS_ERR_ARG, "gradient plan: grid outside [1, 4 blocks per CU]");
  std::lock_guard<std::mutex> g(g_plan_mu);
  g_plans[PlanKey{(int)sizeof(T), pow2_ceil(n), d, k}] = pl;
  return RS_OK;
}

template rs_status gradient_set_plan<float>(int64_t, int64_t, int, const GradPlan&);
template rs_status gradient_set_plan<double>(int64_t, int64_t, int, const GradPlan&);
template GradPlan grad_plan<float>(int64_t, int64_t, int);
template GradPlan grad_plan<double>(int64_t, int64_t, int);
template rs_status gradient_autotune<float>(const float*, int64_t, int64_t, int64_t, const float*,
                                            const double*, int, double*, double*, int,
                                            hipStream_t, GradPlan*);
template rs_status gradient_autotune<double>(const double*, int64_t, int64_t, int64_t,
                                             const double*, const double*, int, double*, double*,
                                             int, hipStream_t, GradPlan*);
template rs_status gradient_launch<float>(const float*, int64_t, int64_t, int64_t, const float*,
                                          double, const double*, int, double*, double*, int,
                                          const int*, hipStream_t, const double*, bool);
template rs_status gradient_launch<double>(const double*, int64_t, int64_t, int64_t, const double*,
                                           double, const double*, int, double*, double*, int,
                                           const int*, hipStream_t, const double*, bool);

}  // namespace rs
