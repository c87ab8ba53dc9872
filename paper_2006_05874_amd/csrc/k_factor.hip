// Factor of the sketched Hessian H_S = (SA)^T SA + nu^2 I (eq. (3)).
//
// m >= d: M = (SA)^T SA + nu^2 I_d (d x d).  m < d: Woodbury through
// M = nu^2 I_m + SA (SA)^T (m x m), as in the proof of Theorem 7.
//   1. Gram on the matrix cores (FP32 MFMA for FP32/BF16 data with FP32
//      accumulation; FP64 MFMA for FP64 data), written as FP64 with nu^2 added.
//   2. Blocked right-looking Cholesky M = L L^T in FP64, 64 x 64 tiles.  The
//      inverse Linv = L^-1 is built during the same sweep: after tile column k
//      is factored, tile row k of Linv follows from the rows above it.
//   3. The explicit FP64 inverse Hinv = H_S^-1:
//        m >= d: Hinv = Linv^T Linv;
//        m <  d: C = Linv SA, Hinv = nu^-2 (I - C^T C).
//      An apply is then a single FP64 matrix-vector product.
// Every square buffer is padded to a multiple of 64 with identity in the pad.
#include "rs_internal.hpp"

namespace rs {

constexpr int NB = 64;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ Gram
// C[i][j] = sum_l X(l, i) X(l, j) with X(l, i) = src[l*ld + i]      (TN: columns)
//                                  or X(l, i) = src[i*ld + l]      (NT: rows)
// over l < q, for i, j < p; lower-triangle 64x64 tiles; FP64 output with
// nu2 on the diagonal and identity past p.  Block: 4 waves, each a 32x32
// quadrant made of 2x2 MFMA 16x16 tiles; K chunks of 16 staged in LDS.
template <typename TAcc, typename T>
__device__ __forceinline__ TAcc load_as(T v) { return (TAcc)v; }
template <>
__device__ __forceinline__ float load_as<float, uint16_t>(uint16_t v) { return bf16_to_f32(v); }
template <>
__device__ __forceinline__ float load_as<float, uint8_t>(uint8_t v) { return e4m3_to_f32(v); }

// colscale (FP8 data only, else null): element (r, c) of SA is stored * scale[c].
template <typename TIn, typename TAcc, bool TN>
__global__ __launch_bounds__(256) void k_gram(const TIn* __restrict__ src, int64_t ld, int64_t p,
                                              int64_t q, int64_t qchunk, TAcc* __restrict__ P,
                                              int64_t ldc, const float* __restrict__ colscale) {
  // triangular tile index -> (I, J), J <= I
  const int64_t bid = blockIdx.x;
  int64_t I = (int64_t)((sqrt(8.0 * (double)bid + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= bid) ++I;
  while (I * (I + 1) / 2 > bid) --I;
  const int64_t J = bid - I * (I + 1) / 2;
  const int64_t i0 = I * NB, j0 = J * NB;

  constexpr int KC = 16;
  __shared__ TAcc As[KC][NB + 1];
  __shared__ TAcc Bs[KC][NB + 1];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;
  const int wr = w >> 1, wc = w & 1;

  using Acc4 = typename std::conditional<sizeof(TAcc) == 4, f32x4, f64x4>::type;
  Acc4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = Acc4{0, 0, 0, 0};

  const int64_t lbeg = (int64_t)blockIdx.y * qchunk;
  const int64_t lend = lbeg + qchunk < q ? lbeg + qchunk : q;
  for (int64_t l0 = lbeg; l0 < lend; l0 += KC) {
    // stage X(l0..l0+16, i0..i0+64) and X(l0.., j0..) : 1024 elements each
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = t * 4 + e;  // 0..1023
      int kk, ii;
      if (TN) { kk = idx / NB; ii = idx % NB; }   // row-major along i: coalesced
      else    { ii = idx / KC; kk = idx % KC; }   // row-major along l: coalesced
      const int64_t l = l0 + kk;
      const int64_t ia = i0 + ii, ja = j0 + ii;
      TAcc va = 0, vb = 0;
      if (l < lend) {
        if (ia < p) va = load_as<TAcc>(TN ? src[l * ld + ia] : src[ia * ld + l]);
        if (ja < p) vb = load_as<TAcc>(TN ? src[l * ld + ja] : src[ja * ld + l]);
        if (colscale) {
          if (TN) {
            if (ia < p) va *= (TAcc)colscale[ia];
            if (ja < p) vb *= (TAcc)colscale[ja];
          } else {
            const TAcc cs = (TAcc)colscale[l];
            va *= cs;
            vb *= cs;
          }
        }
      }
      As[kk][ii] = va;
      Bs[kk][ii] = vb;
    }
    __syncthreads();
#pragma unroll
    for (int k4 = 0; k4 < KC / 4; ++k4) {
      const int kr = k4 * 4 + (lane >> 4);
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const TAcc av = As[kr][wr * 32 + a * 16 + (lane & 15)];
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const TAcc bv = Bs[kr][wc * 32 + b * 16 + (lane & 15)];
          if constexpr (sizeof(TAcc) == 4)
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc[a][b], 0, 0, 0);
          else
            acc[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc[a][b], 0, 0, 0);
        }
      }
    }
    __syncthreads();
  }
  // lane holds column lane % 16 of each 16x16 tile, rows per mfma16_row;
  // partial Gram of this K range into slice blockIdx.y
  TAcc* Ps = P + (int64_t)blockIdx.y * ldc * ldc;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + wr * 32 + a * 16 + mfma16_row<TAcc>(lane, r);
        const int64_t j = j0 + wc * 32 + b * 16 + (lane & 15);
        Ps[i * ldc + j] = acc[a][b][r];
      }
}

// Low-precision TN Gram on the gfx950 K=32 matrix instructions:
// C[i][j] = sum_l X[l][i] X[l][j] over a K range, X stored as BF16 (uint16) or
// FP8 E4M3 (uint8, with per-column scales applied to the FP32 result).  A 64-row
// chunk of X is staged transposed in LDS (Xs[i][l]) so that each lane reads its
// 8 consecutive k values of the 16x16x32 operand layout (lane l: row l % 16,
// k = 8 (l / 16) .. + 7) with one 16- or 8-byte LDS read.
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

template <typename TIn>
__global__ __launch_bounds__(256) void k_gram_lp_tn(const TIn* __restrict__ src, int64_t ld,
                                                    int64_t p, int64_t q, int64_t qchunk,
                                                    float* __restrict__ P, int64_t ldc,
                                                    const float* __restrict__ colscale) {
  const int64_t bid = blockIdx.x;
  int64_t I = (int64_t)((sqrt(8.0 * (double)bid + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= bid) ++I;
  while (I * (I + 1) / 2 > bid) --I;
  const int64_t J = bid - I * (I + 1) / 2;
  const int64_t i0 = I * NB, j0 = J * NB;
  constexpr int KC = 64;
  constexpr int PADK = KC + 16 / (int)sizeof(TIn);   // keeps rows 16-byte aligned
  __shared__ __attribute__((aligned(16))) TIn As[NB][PADK];
  __shared__ __attribute__((aligned(16))) TIn Bs[NB][PADK];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  f32x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0, 0, 0, 0};
  const int64_t lbeg = (int64_t)blockIdx.y * qchunk;
  const int64_t lend = lbeg + qchunk < q ? lbeg + qchunk : q;
  constexpr int EPV = 16 / (int)sizeof(TIn);  // elements per 16-byte vector
  constexpr int VPR = NB / EPV;               // vectors per 64-wide row segment
  for (int64_t l0 = lbeg; l0 < lend; l0 += KC) {
    // stage: KC rows x 64 columns for each operand, 16-byte vectors
    for (int v = t; v < KC * VPR; v += 256) {
      const int kk = v / VPR, cv = v % VPR;
      const int64_t l = l0 + kk;
      const bool lok = l < lend;
      const int64_t lc = lok ? l : lbeg;
      uint4 va = *reinterpret_cast<const uint4*>(src + lc * ld + i0 + cv * EPV);
      uint4 vb = *reinterpret_cast<const uint4*>(src + lc * ld + j0 + cv * EPV);
      const TIn* ea = reinterpret_cast<const TIn*>(&va);
      const TIn* eb = reinterpret_cast<const TIn*>(&vb);
#pragma unroll
      for (int e = 0; e < EPV; ++e) {
        const int64_t ci = i0 + cv * EPV + e, cj = j0 + cv * EPV + e;
        As[cv * EPV + e][kk] = (lok && ci < p) ? ea[e] : (TIn)0;
        Bs[cv * EPV + e][kk] = (lok && cj < p) ? eb[e] : (TIn)0;
      }
    }
    __syncthreads();
#pragma unroll
    for (int k32 = 0; k32 < KC / 32; ++k32) {
      const int kof = k32 * 32 + 8 * (lane >> 4);
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int ia = wr * 32 + a * 16 + (lane & 15);
#pragma unroll
        for (int b = 0; b < 2; ++b) {
          const int jb = wc * 32 + b * 16 + (lane & 15);
          if constexpr (sizeof(TIn) == 2) {
            const bf16x8 av = *reinterpret_cast<const bf16x8*>(&As[ia][kof]);
            const bf16x8 bv = *reinterpret_cast<const bf16x8*>(&Bs[jb][kof]);
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av, bv, acc[a][b], 0, 0, 0);
          } else {
            const long av = *reinterpret_cast<const long*>(&As[ia][kof]);
            const long bv = *reinterpret_cast<const long*>(&Bs[jb][kof]);
            acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(av, bv, acc[a][b], 0, 0, 0);
          }
        }
      }
    }
    __syncthreads();
  }
  float* Ps = P + (int64_t)blockIdx.y * ldc * ldc;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + wr * 32 + a * 16 + mfma16_row<float>(lane, r);
        const int64_t j = j0 + wc * 32 + b * 16 + (lane & 15);
        float v = acc[a][b][r];
        if (colscale && i < p && j < p) v *= colscale[i] * colscale[j];
        Ps[i * ldc + j] = v;
      }
}

// BF16 Gram on the K=32 matrix instructions with a software pipeline:
//   TN: C[i][j] = sum_l X[l][i] X[l][j]   (SA^T SA; X row l is a sketch row)
//   NT: C[i][j] = sum_l X[i][l] X[j][l]   (SA SA^T; K runs along the rows)
// over l in this block's K range, for the lower 64 x 64 tile (I, J).  Each stage
// holds KC = 128 values of l for the 64 columns of each operand in LDS as
// S[col][l] (l contiguous, the operand layout of v_mfma_f32_16x16x32_bf16: lane
// reads 8 consecutive l of one column with one 16-byte read).  For TN every
// thread loads an 8 x 8 block (8 rows of X, 8 columns) and writes it transposed;
// for NT the rows of X already run along l.  The next stage's global loads are
// in flight while the current stage multiplies; two LDS buffers, one barrier per
// stage.  A diagonal tile stages one operand.
namespace {
constexpr int GKC = 128;          // l per stage
constexpr int GKP = GKC + 8;      // LDS row pitch (elements): 16-byte aligned rows

__device__ __forceinline__ uint4 bf16_transpose_col(const uint4 (&in)[8], int c) {
  // column c of the 8 x 8 block: rows 0..7 packed two per 32-bit word
  const int wsel = c >> 1;
  uint32_t o[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const uint32_t a = reinterpret_cast<const uint32_t*>(&in[2 * q])[wsel];
    const uint32_t b = reinterpret_cast<const uint32_t*>(&in[2 * q + 1])[wsel];
    o[q] = (c & 1) ? ((a >> 16) | (b & 0xFFFF0000u)) : ((a & 0xFFFFu) | (b << 16));
  }
  return make_uint4(o[0], o[1], o[2], o[3]);
}
}  // namespace

template <bool TN>
__global__ __launch_bounds__(256) void k_gram_bf16(const uint16_t* __restrict__ src, int64_t ld,
                                                   int64_t p, int64_t q, int64_t qchunk,
                                                   float* __restrict__ P, int64_t ldc) {
  const int64_t bid = blockIdx.x;
  int64_t I = (int64_t)((sqrt(8.0 * (double)bid + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= bid) ++I;
  while (I * (I + 1) / 2 > bid) --I;
  const int64_t J = bid - I * (I + 1) / 2;
  const int64_t i0 = I * NB, j0 = J * NB;
  const bool diag = I == J;
  __shared__ __attribute__((aligned(16))) uint16_t S[2][2][NB][GKP];
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  const int64_t lbeg = (int64_t)blockIdx.y * qchunk;
  const int64_t lend = lbeg + qchunk < q ? lbeg + qchunk : q;
  const int nst = (int)((lend - lbeg + GKC - 1) / GKC);
  // this thread's staging piece: operand op, 8 x 8 block (TN) or 4 row segments (NT)
  const int op = t >> 7;
  const bool stager = !(diag && op == 1);
  const int64_t c0 = op ? j0 : i0;
  uint4 rg[8];
  auto load = [&](int st) {
    const int64_t l0 = lbeg + (int64_t)st * GKC;
    if (TN) {
      // rows l0 + 8 g .. + 7, columns c0 + 8 cb .. + 7
      const int g = (t >> 3) & 15, cb = t & 7;
      const int64_t col = c0 + 8 * cb;
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int64_t l = l0 + 8 * g + e;
        const bool ok = l < lend && col < p;
        const int64_t lc = l < lend ? l : lbeg;
        const uint4 v = *reinterpret_cast<const uint4*>(src + lc * ld + (col < p ? col : 0));
        uint4 z = ok ? v : make_uint4(0, 0, 0, 0);
        if (ok && col + 8 > p) {  // columns past p inside the last group
          uint16_t* h = reinterpret_cast<uint16_t*>(&z);
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (col + u >= p) h[u] = 0;
        }
        rg[e] = z;
      }
    } else {
      // row c0 + r of X, l0 + 8 seg .. + 7 for 8 (r, seg) pairs
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int idx = (t & 127) + 128 * e;  // 0..1023 = 64 rows x 16 segments
        const int r = idx >> 4, seg = idx & 15;
        const int64_t row = c0 + r;
        const int64_t l = l0 + 8 * seg;
        const bool ok = row < p && l < lend;
        const uint4 v = *reinterpret_cast<const uint4*>(src + (row < p ? row : 0) * ld +
                                                       (l < lend ? l : lbeg));
        uint4 z = ok ? v : make_uint4(0, 0, 0, 0);
        if (ok && l + 8 > lend) {  // ragged end of K inside the segment
          uint16_t* h = reinterpret_cast<uint16_t*>(&z);
#pragma unroll
          for (int u = 0; u < 8; ++u)
            if (l + u >= lend) h[u] = 0;
        }
        rg[e] = z;
      }
    }
  };
  auto store = [&](int buf) {
    if (!stager) return;
    if (TN) {
      const int g = (t >> 3) & 15, cb = t & 7;
#pragma unroll
      for (int c = 0; c < 8; ++c)
        *reinterpret_cast<uint4*>(&S[buf][op][8 * cb + c][8 * g]) = bf16_transpose_col(rg, c);
    } else {
#pragma unroll
      for (int e = 0; e < 8; ++e) {
        const int idx = (t & 127) + 128 * e;
        *reinterpret_cast<uint4*>(&S[buf][op][idx >> 4][8 * (idx & 15)]) = rg[e];
      }
    }
  };
  f32x4 acc[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) acc[a][b] = f32x4{0, 0, 0, 0};
  if (stager) load(0);
  store(0);
  __syncthreads();
  const int opb = diag ? 0 : 1;
  for (int st = 0; st < nst; ++st) {
    const int buf = st & 1;
    if (st + 1 < nst && stager) load(st + 1);
#pragma unroll
    for (int k32 = 0; k32 < GKC / 32; ++k32) {
      const int kof = k32 * 32 + 8 * (lane >> 4);
      bf16x8 av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a)
        av[a] = *reinterpret_cast<const bf16x8*>(&S[buf][0][wr * 32 + a * 16 + (lane & 15)][kof]);
#pragma unroll
      for (int b = 0; b < 2; ++b)
        bv[b] = *reinterpret_cast<const bf16x8*>(&S[buf][opb][wc * 32 + b * 16 + (lane & 15)][kof]);
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          acc[a][b] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(av[a], bv[b], acc[a][b], 0, 0, 0);
    }
    if (st + 1 < nst) store(buf ^ 1);
    __syncthreads();
  }
  float* Ps = P + (int64_t)blockIdx.y * ldc * ldc;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + wr * 32 + a * 16 + mfma16_row<float>(lane, r);
        const int64_t j = j0 + wc * 32 + b * 16 + (lane & 15);
        Ps[i * ldc + j] = acc[a][b][r];
      }
}

// M = sum_s P[s] (fixed order, FP64) + nu2 I on the lower tiles; identity past p.
// Also sets the same tile of the L^-1 buffer (when given) to the identity: the
// lower tiles are all the factor sweep reads of it.
template <typename TAcc>
__global__ __launch_bounds__(256) void k_gram_reduce(const TAcc* __restrict__ P, int nsplit,
                                                     int64_t p, double nu2,
                                                     double* __restrict__ C, int64_t ldc,
                                                     FactorBatch zb, double* __restrict__ X) {
  C += blockIdx.z * zb.sM;
  if (X) X += blockIdx.z * zb.sL;
  if (zb.nu2) nu2 = zb.nu2[blockIdx.z];
  const int64_t bid = blockIdx.x;
  int64_t I = (int64_t)((sqrt(8.0 * (double)bid + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= bid) ++I;
  while (I * (I + 1) / 2 > bid) --I;
  const int64_t J = bid - I * (I + 1) / 2;
  const int64_t slice = ldc * ldc;
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    const int64_t i = I * NB + e / NB, j = J * NB + e % NB;
    double v = 0.0;
    for (int sI = 0; sI < nsplit; ++sI) v += (double)P[sI * slice + i * ldc + j];
    if (i == j) v += nu2;
    if (i >= p || j >= p) v = (i == j) ? 1.0 : 0.0;
    C[i * ldc + j] = v;
    if (X) X[i * ldc + j] = (i == j) ? 1.0 : 0.0;
  }
}

// ------------------------------------------------------------------ FP64 tiles
// acc (4x4 per thread; thread (ty, tx) owns rows 4ty.., cols 4tx..) +=
// opA (64 x kd) * opB (kd x 64), each operand read through a lambda-free
// descriptor: element (r, c) of op(X) = trans ? X[c*ld + r] : X[r*ld + c],
// zero outside (rows, cols).
struct Opnd {
  const double* p;
  int64_t ld;
  int64_t rows, cols;  // extent of op(X) from its origin
  bool trans;
};

__device__ __forceinline__ double opnd_at(const Opnd& o, int64_t r, int64_t c) {
  // clamped in-bounds address and a select: no branch around the load
  const bool ok = r < o.rows && c < o.cols;
  const int64_t rr = ok ? r : 0, cc = ok ? c : 0;
  const double v = o.p[o.trans ? cc * o.ld + rr : rr * o.ld + cc];
  return ok ? v : 0.0;
}

struct FOpnd {  // FP32 source, same addressing
  const float* p;
  int64_t ld;
  int64_t rows, cols;
  bool trans;
};
__device__ __forceinline__ double opnd_at(const FOpnd& o, int64_t r, int64_t c) {
  const bool ok = r < o.rows && c < o.cols;
  const int64_t rr = ok ? r : 0, cc = ok ? c : 0;
  const double v = (double)o.p[o.trans ? cc * o.ld + rr : rr * o.ld + cc];
  return ok ? v : 0.0;
}
struct HOpnd {  // BF16 source
  const uint16_t* p;
  int64_t ld;
  int64_t rows, cols;
  bool trans;
};
__device__ __forceinline__ double opnd_at(const HOpnd& o, int64_t r, int64_t c) {
  const bool ok = r < o.rows && c < o.cols;
  const int64_t rr = ok ? r : 0, cc = ok ? c : 0;
  const double v = (double)bf16_to_f32(o.p[o.trans ? cc * o.ld + rr : rr * o.ld + cc]);
  return ok ? v : 0.0;
}

struct QOpnd {  // FP8 E4M3 source with per-column scales of the stored matrix
  const uint8_t* p;
  int64_t ld;
  int64_t rows, cols;
  bool trans;
  const float* scale;  // indexed by the stored matrix's column
};
__device__ __forceinline__ double opnd_at(const QOpnd& o, int64_t r, int64_t c) {
  const bool ok = r < o.rows && c < o.cols;
  const int64_t rr = ok ? r : 0, cc = ok ? c : 0;
  const int64_t sc = o.trans ? rr : cc;
  const double v = (double)e4m3_to_f32(o.p[o.trans ? cc * o.ld + rr : rr * o.ld + cc]) *
                   (double)o.scale[sc];
  return ok ? v : 0.0;
}

// The next 32-deep chunk of both operands is loaded into registers while the
// current one is multiplied from LDS (double-buffered, one barrier per chunk).
constexpr int TKC = 32;
struct TileLds {
  double A[2][TKC][NB + 1];
  double B[2][TKC][NB + 1];
};

template <typename OA, typename OB>
__device__ __forceinline__ void tile_fetch(const OA& A, const OB& B, int64_t k0, double (&ra)[8],
                                           double (&rb)[8]) {
  const int t = threadIdx.x;
#pragma unroll
  for (int e = 0; e < 8; ++e) {
    const int idx = t + 256 * e;                 // 0..2047
    const int r = idx >> 5, kk = idx & 31;       // A: 64 rows x 32 k
    ra[e] = opnd_at(A, r, k0 + kk);
    const int kb = idx >> 6, cb = idx & 63;      // B: 32 k x 64 cols
    rb[e] = opnd_at(B, k0 + kb, cb);
  }
}

// quadrants (MFMA layout, wave w owns (w / 2, w % 2)) -> LDS (64 x 65) -> the
// per-thread 4 x 4 layout, added into acc; ends with a barrier.
__device__ __forceinline__ void quadrants_to_acc(const f64x4 (&q)[2][2], double (&acc)[4][4],
                                                 TileLds& L) {
  const int t = threadIdx.x;
  const int ty = t >> 4, tx = t & 15;
  const int lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  double* F = &L.A[0][0][0];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        F[(wr * 32 + a * 16 + (lane >> 4) + 4 * r) * (NB + 1) + wc * 32 + b * 16 + (lane & 15)] =
            q[a][b][r];
  __syncthreads();
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] += F[(ty * 4 + i) * (NB + 1) + tx * 4 + j];
  __syncthreads();
}

// acc (thread (ty, tx) holds rows 4ty.., columns 4tx..) += op(A) op(B) over kd.
// The products run on the FP64 matrix cores: wave w owns the 32 x 32 quadrant
// (w / 2, w % 2) as 2 x 2 tiles of v_mfma_f64_16x16x4 (operands A[row][k] and
// B[k][col] read from the staged chunks); at the end the quadrants pass through
// LDS into the per-thread 4 x 4 layout the callers use.
template <typename OA, typename OB>
__device__ void tile_mm(double (&acc)[4][4], const OA& A, const OB& B, int64_t kd, TileLds& L) {
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  f64x4 q[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) q[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  double ra[8], rb[8];
  tile_fetch(A, B, 0, ra, rb);
  int buf = 0;
  for (int64_t k0 = 0; k0 < kd; k0 += TKC) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int idx = t + 256 * e;
      L.A[buf][idx & 31][idx >> 5] = ra[e];
      L.B[buf][idx >> 6][idx & 63] = rb[e];
    }
    __syncthreads();
    if (k0 + TKC < kd) tile_fetch(A, B, k0 + TKC, ra, rb);
#pragma unroll
    for (int k4 = 0; k4 < TKC / 4; ++k4) {
      const int kk = 4 * k4 + (lane >> 4);
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = L.A[buf][kk][wr * 32 + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = L.B[buf][kk][wc * 32 + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          q[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], q[a][b], 0, 0, 0);
    }
    buf ^= 1;
  }
  __syncthreads();
  quadrants_to_acc(q, acc, L);
}

// The same product for kd = 64 (one tile of the blocked factor): both K chunks are
// fetched at once, so the product waits for one round trip to memory instead of
// two.  The summation order is that of tile_mm.
template <typename OA, typename OB>
__device__ void tile_mm_k64(double (&acc)[4][4], const OA& A, const OB& B, TileLds& L) {
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  f64x4 q[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) q[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
  double ra[2][8], rb[2][8];
  tile_fetch(A, B, 0, ra[0], rb[0]);
  tile_fetch(A, B, TKC, ra[1], rb[1]);
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int idx = t + 256 * e;
      L.A[c][idx & 31][idx >> 5] = ra[c][e];
      L.B[c][idx >> 6][idx & 63] = rb[c][e];
    }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int k4 = 0; k4 < TKC / 4; ++k4) {
      const int kk = 4 * k4 + (lane >> 4);
      double av[2], bv[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = L.A[c][kk][wr * 32 + a * 16 + (lane & 15)];
#pragma unroll
      for (int b = 0; b < 2; ++b) bv[b] = L.B[c][kk][wc * 32 + b * 16 + (lane & 15)];
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          q[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[b], q[a][b], 0, 0, 0);
    }
  __syncthreads();
  quadrants_to_acc(q, acc, L);
}

__device__ __forceinline__ void zero_acc(double (&acc)[4][4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = 0.0;
}

// ------------------------------------------------------------------ Cholesky
// Right-looking blocked Cholesky M = L L^T, and Linv = L^-1 by block forward
// substitution of L X = I carried along the same sweep: the Linv buffer starts
// as the identity and holds the partially reduced right-hand side Y.  At step k
//   diag  : L_kk and Linv_kk = L_kk^-1 (into the Linv buffer);
//   panel : L_ik = M_ik Linv_kk^T (i > k, into M), and X_kj = Linv_kk Y_kj (j < k);
//   update: M_ij -= L_ik L_jk^T (k < j <= i), Y_ij -= L_ik X_kj (i > k, j <= k).
// The three run as one launch per step (k_chol_step): the update of step k - 1 is
// applied by the blocks of step k that read the tiles it changes, and every block
// that needs Linv_kk factors the diagonal tile itself.  The critical path of a step
// is one tile product, the diagonal factor and one more tile product.

// 1/sqrt(x) in FP64: hardware estimate refined by two Newton steps.
__device__ __forceinline__ double rsqrt64(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  y = y * fma(-h * y, y, 1.5);
  return y;
}

// Diagonal tile k: factor and invert the 64 x 64 block in LDS, 16 columns at a
// time.  For each 16-wide panel: one wave factors the 16 x 16 diagonal piece
// (lane i holds row i in registers) four columns at a time: the 4 x 4 pivot block
// is factored (L_D) and inverted (M = L_D^-1) by every lane alike, each row's four
// entries v_i become P_i = v_i L_D^-T by forward substitution, and the columns
// past them take the rank-4 update -P_i P_j^T, the P_j read back from LDS; then
// lane c builds column c of the 16 x 16 inverse by block forward substitution
// over the 4 x 4 blocks.
// After that the whole block applies the panel below, the matching block row of
// the inverse, and the trailing update on the FP64 matrix cores.  X = L^-1 is
// carried along as the right-hand side of L X = I.
//
// LDS traffic inside the one wave needs no barrier: a wave's LDS operations
// execute in order, and the wavefront fence keeps the compiler from moving the
// reads of other lanes' rows above the writes.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

template <int Q>
__device__ __forceinline__ void diag_panel(double (*a)[NB + 1], double (*x)[NB + 1],
                                           double (*dinv)[17], double (*pbuf)[4], bool& bad) {
  const int t = threadIdx.x;
  const int lane = t & 63;
  const int w = t >> 6;
  // A: factor the 16 x 16 block at (Q, Q) and invert it
  if (w == 0) {
    const int li = lane & 15;
    double r[16];
#pragma unroll
    for (int c = 0; c < 16; ++c) r[c] = a[Q + li][Q + c];
    double M[4][4][4];  // inverse of each 4 x 4 diagonal factor (lower part used)
#pragma unroll
    for (int sb = 0; sb < 4; ++sb) {
      const int c0 = 4 * sb;
      // the rows' current entries in columns c0..c0+3; the pivot block (rows
      // c0..c0+3) read back by every lane
      if (lane < 16) {
#pragma unroll
        for (int e = 0; e < 4; ++e) pbuf[li][e] = r[c0 + e];
      }
      wave_lds_sync();
      double D[4][4];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j <= i; ++j) D[i][j] = pbuf[c0 + i][j];
      // 4 x 4 Cholesky L_D and its inverse, the same in every lane
      double L[4][4], inv[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        double dd = D[j][j];
#pragma unroll
        for (int k = 0; k < j; ++k) dd = fma(-L[j][k], L[j][k], dd);
        bad |= !(dd > 0.0);
        inv[j] = rsqrt64(dd);
        L[j][j] = dd * inv[j];
#pragma unroll
        for (int i = j + 1; i < 4; ++i) {
          double v = D[i][j];
#pragma unroll
          for (int k = 0; k < j; ++k) v = fma(-L[i][k], L[j][k], v);
          L[i][j] = v * inv[j];
        }
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        M[sb][i][i] = inv[i];
#pragma unroll
        for (int j = i - 1; j >= 0; --j) {
          double v = 0.0;
#pragma unroll
          for (int k = j; k < i; ++k) v = fma(L[i][k], M[sb][k][j], v);
          M[sb][i][j] = -inv[i] * v;
        }
      }
      // P_i = v_i L_D^-T by forward substitution: on the pivot rows this repeats
      // the operations above and gives L_D exactly
      double P[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        double v = r[c0 + j];
#pragma unroll
        for (int k = 0; k < j; ++k) v = fma(-P[k], L[j][k], v);
        P[j] = v * inv[j];
        r[c0 + j] = P[j];
      }
      // rank-4 update of the columns past the block (rows above them update
      // entries that are never read)
      if (c0 + 4 < 16) {
        wave_lds_sync();
        if (lane < 16) {
#pragma unroll
          for (int e = 0; e < 4; ++e) pbuf[li][e] = P[e];
        }
        wave_lds_sync();
#pragma unroll
        for (int j = c0 + 4; j < 16; ++j) {
          double v = r[j];
#pragma unroll
          for (int e = 0; e < 4; ++e) v = fma(-P[e], pbuf[j][e], v);
          r[j] = v;
        }
        wave_lds_sync();
      }
    }
    if (lane < 16) {
#pragma unroll
      for (int c = 0; c < 16; ++c) a[Q + lane][Q + c] = c <= lane ? r[c] : 0.0;
    }
    wave_lds_sync();
    // column li of L^-1: block row s is M_s (e_li - sum_{u<s} L_su x_u)
    double col[16];
#pragma unroll
    for (int sb = 0; sb < 4; ++sb) {
      double y[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) y[i] = (4 * sb + i == li) ? 1.0 : 0.0;
#pragma unroll
      for (int u = 0; u < sb; ++u)
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int k = 0; k < 4; ++k)
            y[i] = fma(-a[Q + 4 * sb + i][Q + 4 * u + k], col[4 * u + k], y[i]);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        double v = 0.0;
#pragma unroll
        for (int k = 0; k <= i; ++k) v = fma(M[sb][i][k], y[k], v);
        col[4 * sb + i] = v;
      }
    }
    if (lane < 16) {
#pragma unroll
      for (int i = 0; i < 16; ++i) dinv[i][lane] = col[i];
    }
  }
  __syncthreads();
  // C: panel below (rows Q+16.., 16 columns) and block row Q.. of the inverse, as
  // 16 x 16 tiles on the FP64 matrix cores: the panel has (48 - Q) / 16 tiles and
  // the inverse block row (Q + 16) / 16, four in all, one per wave.  Lane layout
  // of v_mfma_f64_16x16x4: A[lane % 16][k0 + lane / 16], B[k0 + lane / 16][lane % 16],
  // result slot r at row lane / 16 + 4 r, column lane % 16.
  {
    constexpr int NPT = (NB - Q - 16) / 16;
    const int li = lane & 15, lk = lane >> 4;
    f64x4 acc = {0.0, 0.0, 0.0, 0.0};
    if (w < NPT) {
      const int r0 = Q + 16 + 16 * w;
#pragma unroll
      for (int k4 = 0; k4 < 4; ++k4)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r0 + li][Q + 4 * k4 + lk],
                                                   dinv[li][4 * k4 + lk], acc, 0, 0, 0);
    } else {
      const int c0 = 16 * (w - NPT);
#pragma unroll
      for (int k4 = 0; k4 < 4; ++k4)
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(dinv[li][4 * k4 + lk],
                                                   x[Q + 4 * k4 + lk][c0 + li], acc, 0, 0, 0);
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = lk + 4 * r;
      if (w < NPT) a[Q + 16 + 16 * w + row][Q + li] = acc[r];
      else x[Q + row][16 * (w - NPT) + li] = acc[r];
    }
  }
  __syncthreads();
  // D: trailing update of the lower part (tiles I >= J of the rows and columns
  // past the panel) and of the rows of Y below the panel, tiles spread over the
  // waves; each output tile belongs to one wave
  constexpr int NT = (NB - Q - 16) / 16;
  constexpr int NTRI = NT * (NT + 1) / 2;
  constexpr int NYT = NT * ((Q + 16) / 16);
  if constexpr (NT > 0) {
    const int li = lane & 15, lk = lane >> 4;
    for (int tile = w; tile < NTRI + NYT; tile += 4) {
      f64x4 acc = {0.0, 0.0, 0.0, 0.0};
      if (tile < NTRI) {
        int I = 0;
        while ((I + 1) * (I + 2) / 2 <= tile) ++I;
        const int J = tile - I * (I + 1) / 2;
        const int r0 = Q + 16 + 16 * I, c0 = Q + 16 + 16 * J;
#pragma unroll
        for (int k4 = 0; k4 < 4; ++k4)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r0 + li][Q + 4 * k4 + lk],
                                                     a[c0 + li][Q + 4 * k4 + lk], acc, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) a[r0 + lk + 4 * r][c0 + li] -= acc[r];
      } else {
        const int y = tile - NTRI;
        const int I = y / ((Q + 16) / 16), J = y % ((Q + 16) / 16);
        const int r0 = Q + 16 + 16 * I, c0 = 16 * J;
#pragma unroll
        for (int k4 = 0; k4 < 4; ++k4)
          acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a[r0 + li][Q + 4 * k4 + lk],
                                                     x[Q + 4 * k4 + lk][c0 + li], acc, 0, 0, 0);
#pragma unroll
        for (int r = 0; r < 4; ++r) x[r0 + lk + 4 * r][c0 + li] -= acc[r];
      }
    }
  }
  __syncthreads();
}

// LDS-operand 64 x 64 x 64 product on the FP64 matrix cores: q = op(A) op(B) with
// op(A)[r][l] = A[r][l] and op(B)[l][c] = TB ? B[c][l] : B[l][c].  Wave w owns the
// 32 x 32 quadrant (w / 2, w % 2) as 2 x 2 tiles; slot r of tile (a, b) is row
// 32 (w / 2) + 16 a + lane / 16 + 4 r, column 32 (w % 2) + 16 b + lane % 16.
template <bool TB>
__device__ __forceinline__ void lds_mm(f64x4 (&q)[2][2], const double (*A)[NB + 1],
                                       const double (*B)[NB + 1]) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w >> 1, wc = w & 1;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) q[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll 4
  for (int k4 = 0; k4 < NB / 4; ++k4) {
    const int kk = 4 * k4 + (lane >> 4);
    double av[2], bv[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) av[i] = A[wr * 32 + i * 16 + (lane & 15)][kk];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int c = wc * 32 + j * 16 + (lane & 15);
      bv[j] = TB ? B[c][kk] : B[kk][c];
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
        q[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], q[i][j], 0, 0, 0);
  }
}

__device__ __forceinline__ void store_quadrants(const f64x4 (&q)[2][2], double* dst, int64_t ld) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int wr = w >> 1, wc = w & 1;
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r)
        dst[(int64_t)(wr * 32 + i * 16 + (lane >> 4) + 4 * r) * ld + wc * 32 + j * 16 +
            (lane & 15)] = q[i][j][r];
}

// The lazy products of one factor step in one pass over two staged operands:
// U (A-layout, L.A[k][row] = U[row][k]) and V (B-layout, L.B[k][col] = V[k][col]),
// both 64 x 64 with K = 64, fetched in one round trip.  d += S S^T where S is the
// step's previous column tile L_k,k-1, read from L.A (sfromA: S = U) or from L.B
// (S^T = V); with pair set also p += U V.  The k order is that of tile_mm, so every
// block that forms S S^T gets the same bits.
template <typename OU, typename OV>
__device__ void step_products(double (&dacc)[4][4], double (&pacc)[4][4], const OU& U,
                              const OV& V, bool stage_v, bool sfromA, bool pair, TileLds& L) {
  const int t = threadIdx.x;
  const int lane = t & 63, w = t >> 6;
  const int wr = w >> 1, wc = w & 1;
  f64x4 qd[2][2], qp[2][2];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      qd[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
      qp[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
    }
  double ra[2][8], rb[2][8];
  tile_fetch(U, V, 0, ra[0], rb[0]);
  tile_fetch(U, V, TKC, ra[1], rb[1]);
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int idx = t + 256 * e;
      L.A[c][idx & 31][idx >> 5] = ra[c][e];
      if (stage_v) L.B[c][idx >> 6][idx & 63] = rb[c][e];
    }
  __syncthreads();
#pragma unroll
  for (int c = 0; c < 2; ++c)
#pragma unroll
    for (int k4 = 0; k4 < TKC / 4; ++k4) {
      const int kk = 4 * k4 + (lane >> 4);
      double sr[2], sc[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) {
        const int r = wr * 32 + a * 16 + (lane & 15);
        sr[a] = sfromA ? L.A[c][kk][r] : L.B[c][kk][r];
      }
#pragma unroll
      for (int b = 0; b < 2; ++b) {
        const int col = wc * 32 + b * 16 + (lane & 15);
        sc[b] = sfromA ? L.A[c][kk][col] : L.B[c][kk][col];
      }
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
          qd[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(sr[a], sc[b], qd[a][b], 0, 0, 0);
      if (pair) {
        double ur[2], vc[2];
#pragma unroll
        for (int a = 0; a < 2; ++a) ur[a] = L.A[c][kk][wr * 32 + a * 16 + (lane & 15)];
#pragma unroll
        for (int b = 0; b < 2; ++b) vc[b] = L.B[c][kk][wc * 32 + b * 16 + (lane & 15)];
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
          for (int b = 0; b < 2; ++b)
            qp[a][b] = __builtin_amdgcn_mfma_f64_16x16x4f64(ur[a], vc[b], qp[a][b], 0, 0, 0);
      }
    }
  __syncthreads();
  quadrants_to_acc(qd, dacc, L);
  if (pair) quadrants_to_acc(qp, pacc, L);
}

// One step k of the blocked factor in a single launch.  The trailing update of step
// k - 1 is applied lazily here, by the blocks that need it:
//   block 0         : diagonal tile M_kk - L_k,k-1 L_k,k-1^T, factored and inverted
//                     in LDS; writes Linv_kk (and the pivot flag);
//   blocks 1..nrest : the same diagonal factor (recomputed, bitwise equal), then
//                     L_ik = (M_ik - L_i,k-1 L_k,k-1^T) Linv_kk^T, i = k + b;
//   next k blocks   : the same diagonal factor, then
//                     X_kj = Linv_kk (Y_kj - L_k,k-1 X_k-1,j), j < k;
//   the rest        : M_ij -= L_i,k-1 L_j,k-1^T (k < j <= i) and
//                     Y_ij -= L_i,k-1 X_k-1,j (i > k, j < k).
// No block writes what another block of the same launch reads: the diagonal tile of
// M is only read (its factor is not needed after the step), column k of M and row k
// of Linv are written by their own blocks, and the lazy updates touch only tiles past
// column k or below row k.  Panels of the diagonal tile that lie entirely in the
// identity padding (index >= p) are skipped: there L = I and X = I already.
__global__ __launch_bounds__(256) void k_chol_step(double* __restrict__ M, int64_t ld, int k,
                                                   int nblk, double* __restrict__ Linv,
                                                   int* __restrict__ info, int64_t p,
                                                   FactorBatch zb) {
  M += blockIdx.z * zb.sM;
  Linv += blockIdx.z * zb.sL;
  // one LDS region: the tile products' staging first, then the diagonal tile, its
  // inverse and the small factor buffers (every product precedes the factor)
  constexpr size_t kTile = sizeof(double) * NB * (NB + 1);
  constexpr size_t kFac = 2 * kTile + sizeof(double) * (16 * 17 + 16 * 4);
  constexpr size_t kLds = kFac > sizeof(TileLds) ? kFac : sizeof(TileLds);
  __shared__ __attribute__((aligned(16))) unsigned char lds[kLds];
  TileLds& tl = *reinterpret_cast<TileLds*>(lds);
  double (*a)[NB + 1] = reinterpret_cast<double (*)[NB + 1]>(lds);
  double (*x)[NB + 1] = reinterpret_cast<double (*)[NB + 1]>(lds + kTile);
  double (*dinv)[17] = reinterpret_cast<double (*)[17]>(lds + 2 * kTile);
  double (*pbuf)[4] = reinterpret_cast<double (*)[4]>(lds + 2 * kTile + sizeof(double) * 16 * 17);
  const int t = threadIdx.x;
  const int ty = t >> 4, tx = t & 15;
  const int nrest = nblk - 1 - k;
  const int64_t ok = (int64_t)k * NB, okm = ok - NB;
  const int64_t bid = blockIdx.x;
  const int64_t nfac = 1 + nrest + k;
  double acc[4][4];
  zero_acc(acc);
  if (bid >= nfac) {
    // lazy trailing update by column block k - 1 (present only when k > 0)
    const int64_t u = bid - nfac;
    const int64_t tri = (int64_t)nrest * (nrest + 1) / 2;
    double* dst;
    if (u < tri) {
      int64_t I = (int64_t)((sqrt(8.0 * (double)u + 1.0) - 1.0) * 0.5);
      while ((I + 1) * (I + 2) / 2 <= u) ++I;
      while (I * (I + 1) / 2 > u) --I;
      const int64_t J = u - I * (I + 1) / 2;
      const int64_t oi = ok + (1 + I) * NB, oj = ok + (1 + J) * NB;
      Opnd A{M + oi * ld + okm, ld, NB, NB, false};
      Opnd B{M + oj * ld + okm, ld, NB, NB, true};
      tile_mm_k64(acc, A, B, tl);
      dst = M + oi * ld + oj;
    } else {
      const int64_t r = u - tri;
      const int64_t I = r / k, J = r % k;
      const int64_t oi = ok + (1 + I) * NB, oj = J * NB;
      Opnd A{M + oi * ld + okm, ld, NB, NB, false};
      Opnd B{Linv + okm * ld + oj, ld, NB, NB, false};
      tile_mm_k64(acc, A, B, tl);
      dst = Linv + oi * ld + oj;
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) dst[(int64_t)(ty * 4 + i) * ld + tx * 4 + j] -= acc[i][j];
    return;
  }
  const bool pan = bid >= 1 && bid <= nrest;  // panel block (row tile k + bid)
  const bool xrow = bid > nrest;              // inverse block row (column tile bid - nrest - 1)
  // the update of step k - 1 on the diagonal tile (acc) and on the block's panel or
  // inverse tile (tile2, kept in registers across the diagonal factor), from one
  // staging of L_k,k-1 and the tile's own operand
  double tile2[4][4];
  zero_acc(tile2);
  // this block's tiles of M (and of the inverse buffer), loaded now so that the
  // loads overlap the products below
  double mkk[4][4], m2[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t r = ty * 4 + i, c = tx * 4 + j;
      mkk[i][j] = M[(ok + r) * ld + ok + c];
      m2[i][j] = pan ? M[(ok + bid * NB + r) * ld + ok + c]
                     : (xrow ? Linv[(ok + r) * ld + (bid - nrest - 1) * NB + c] : 0.0);
    }
  if (k > 0) {
    const Opnd S{M + ok * ld + okm, ld, NB, NB, false};     // L_k,k-1
    const Opnd ST{M + ok * ld + okm, ld, NB, NB, true};     // L_k,k-1^T
    if (pan) {
      const Opnd U{M + (ok + bid * NB) * ld + okm, ld, NB, NB, false};  // L_i,k-1
      step_products(acc, tile2, U, ST, true, false, true, tl);
    } else if (xrow) {
      const Opnd V{Linv + okm * ld + (bid - nrest - 1) * NB, ld, NB, NB, false};  // X_k-1,j
      step_products(acc, tile2, S, V, true, true, true, tl);
    } else {
      step_products(acc, tile2, S, S, false, true, false, tl);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) tile2[i][j] = m2[i][j] - tile2[i][j];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int r = ty * 4 + i, c = tx * 4 + j;
      a[r][c] = mkk[i][j] - acc[i][j];
      x[r][c] = (r == c) ? 1.0 : 0.0;
    }
  __syncthreads();
  bool bad = false;
  const int64_t valid = p - ok;  // valid indices in this tile (>= 1)
  diag_panel<0>(a, x, dinv, pbuf, bad);
  if (valid > 16) diag_panel<16>(a, x, dinv, pbuf, bad);
  if (valid > 32) diag_panel<32>(a, x, dinv, pbuf, bad);
  if (valid > 48) diag_panel<48>(a, x, dinv, pbuf, bad);
  if (bid == 0) {
    if (bad) atomicExch(info, 1);
    for (int idx = t; idx < NB * NB; idx += 256) {
      const int i = idx >> 6, j = idx & 63;
      Linv[(ok + i) * ld + ok + j] = j <= i ? x[i][j] : 0.0;
    }
    return;
  }
  // a is free (diag_panel ends with a barrier): the saved tile goes there
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) a[ty * 4 + i][tx * 4 + j] = tile2[i][j];
  __syncthreads();
  f64x4 q[2][2];
  if (pan) {
    // L_ik = (M_ik - L_i,k-1 L_k,k-1^T) Linv_kk^T
    lds_mm<true>(q, a, x);
    store_quadrants(q, M + (ok + bid * NB) * ld + ok, ld);
  } else {
    // X_kj = Linv_kk (Y_kj - L_k,k-1 X_k-1,j)
    lds_mm<false>(q, x, a);
    store_quadrants(q, Linv + ok * ld + (bid - nrest - 1) * NB, ld);
  }
}

// Hinv = Linv^T Linv (p x p, both triangles): tile (I, J), J <= I:
// sum_{l >= I} Linv_lI^T Linv_lJ.
__global__ __launch_bounds__(256) void k_lauum(const double* __restrict__ Linv, int64_t ld,
                                               int nblk, double* __restrict__ H, int64_t ldh,
                                               FactorBatch zb) {
  Linv += blockIdx.z * zb.sL;
  H += (zb.hz ? zb.hz[blockIdx.z] : (int)blockIdx.z) * zb.sH;
  __shared__ TileLds tl;
  const int64_t bid = blockIdx.x;
  int64_t I = (int64_t)((sqrt(8.0 * (double)bid + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= bid) ++I;
  while (I * (I + 1) / 2 > bid) --I;
  const int64_t J = bid - I * (I + 1) / 2;
  double acc[4][4];
  zero_acc(acc);
  const int64_t oI = I * NB, oJ = J * NB;
  const int64_t rows = (nblk - I) * NB;
  Opnd A{Linv + oI * ld + oI, ld, NB, rows, true};   // op(A) = (Linv[oI.., oI..])^T: 64 x rows
  Opnd B{Linv + oI * ld + oJ, ld, rows, NB, false};
  tile_mm(acc, A, B, rows, tl);
  const int t = threadIdx.x, ty = t >> 4, tx = t & 15;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      H[(oI + ty * 4 + i) * ldh + oJ + tx * 4 + j] = acc[i][j];
      H[(oJ + tx * 4 + j) * ldh + oI + ty * 4 + i] = acc[i][j];
    }
}

// The same product split over row chunks of Linv (chunk s covers block rows
// [s CH, (s+1) CH) from I on), for factors whose few long tile chains would
// otherwise run on a few CUs: partial P[s][tile] then a fixed-order sum.
__global__ __launch_bounds__(256) void k_lauum_part(const double* __restrict__ Linv, int64_t ld,
                                                    int nblk, int ch, double* __restrict__ P) {
  __shared__ TileLds tl;
  const int64_t bid = blockIdx.x;
  int64_t I = (int64_t)((sqrt(8.0 * (double)bid + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= bid) ++I;
  while (I * (I + 1) / 2 > bid) --I;
  const int64_t J = bid - I * (I + 1) / 2;
  const int64_t l0 = std::max<int64_t>(I, (int64_t)blockIdx.y * ch);
  const int64_t l1 = std::min<int64_t>(nblk, ((int64_t)blockIdx.y + 1) * ch);
  if (l0 >= l1) return;  // the sum skips this chunk
  double acc[4][4];
  zero_acc(acc);
  const int64_t oI = I * NB, oJ = J * NB, o0 = l0 * NB;
  const int64_t rows = (l1 - l0) * NB;
  Opnd A{Linv + o0 * ld + oI, ld, NB, rows, true};
  Opnd B{Linv + o0 * ld + oJ, ld, rows, NB, false};
  tile_mm(acc, A, B, rows, tl);
  const int64_t tiles = (int64_t)nblk * (nblk + 1) / 2;
  double* out = P + ((int64_t)blockIdx.y * tiles + bid) * NB * NB;
  const int t = threadIdx.x, ty = t >> 4, tx = t & 15;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) out[(ty * 4 + i) * NB + tx * 4 + j] = acc[i][j];
}

__global__ __launch_bounds__(256) void k_lauum_sum(const double* __restrict__ P, int nblk, int ch,
                                                   int nsplit, double* __restrict__ H,
                                                   int64_t ldh) {
  const int64_t bid = blockIdx.x;
  int64_t I = (int64_t)((sqrt(8.0 * (double)bid + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= bid) ++I;
  while (I * (I + 1) / 2 > bid) --I;
  const int64_t J = bid - I * (I + 1) / 2;
  const int64_t tiles = (int64_t)nblk * (nblk + 1) / 2;
  const int s0 = (int)(I / ch);
  for (int e = threadIdx.x; e < NB * NB; e += 256) {
    double v = 0.0;
    for (int sp = s0; sp < nsplit; ++sp) v += P[((int64_t)sp * tiles + bid) * NB * NB + e];
    const int64_t r = I * NB + e / NB, c = J * NB + e % NB;
    H[r * ldh + c] = v;
    H[c * ldh + r] = v;
  }
}

// Chunks of the split product: about two blocks per CU over all tiles.
static int lauum_chunk(int nblk) {
  const int64_t tiles = (int64_t)nblk * (nblk + 1) / 2;
  const int64_t want = std::max<int64_t>(1, (2 * device_cus() + tiles - 1) / tiles);
  const int64_t ch = std::max<int64_t>(1, (nblk + want - 1) / want);
  return (int)ch;
}

template <typename O>
__device__ __forceinline__ void shift_scale(O&, int64_t) {}
__device__ __forceinline__ void shift_scale(QOpnd& o, int64_t off) { o.scale += off; }

// C = Linv SA (m x d): tile (I over m, Jd over d): sum_{l <= I} Linv_Il SA_l.
template <typename OSA>
__global__ __launch_bounds__(256) void k_whiten(const double* __restrict__ Linv, int64_t ld,
                                                OSA SA, int64_t d, double* __restrict__ Cw,
                                                int64_t ldc, FactorBatch zb) {
  Linv += blockIdx.z * zb.sL;
  Cw += blockIdx.z * zb.sC;
  __shared__ TileLds tl;
  const int64_t I = blockIdx.y, Jd = blockIdx.x;
  double acc[4][4];
  zero_acc(acc);
  const int64_t oI = I * NB, oJ = Jd * NB;
  Opnd A{Linv + oI * ld, ld, NB, (I + 1) * NB, false};
  OSA B = SA;
  B.p = SA.p + oJ;
  B.cols = d - oJ;
  shift_scale(B, oJ);
  tile_mm(acc, A, B, (I + 1) * NB, tl);
  const int t = threadIdx.x, ty = t >> 4, tx = t & 15;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) Cw[(oI + ty * 4 + i) * ldc + oJ + tx * 4 + j] = acc[i][j];
}

// Hinv = nu^-2 (I - C^T C) over d x d (both triangles), C padded with zero rows.
__global__ __launch_bounds__(256) void k_woodbury_inv(const double* __restrict__ Cw, int64_t ldc,
                                                      int64_t mpad, double inv_nu2, int64_t dp,
                                                      double* __restrict__ H, int64_t ldh,
                                                      FactorBatch zb) {
  Cw += blockIdx.z * zb.sC;
  H += (zb.hz ? zb.hz[blockIdx.z] : (int)blockIdx.z) * zb.sH;
  if (zb.nu2) inv_nu2 = 1.0 / zb.nu2[blockIdx.z];
  __shared__ TileLds tl;
  const int64_t bid = blockIdx.x;
  int64_t I = (int64_t)((sqrt(8.0 * (double)bid + 1.0) - 1.0) * 0.5);
  while ((I + 1) * (I + 2) / 2 <= bid) ++I;
  while (I * (I + 1) / 2 > bid) --I;
  const int64_t J = bid - I * (I + 1) / 2;
  double acc[4][4];
  zero_acc(acc);
  const int64_t oI = I * NB, oJ = J * NB;
  Opnd A{Cw + oI, ldc, NB, mpad, true};
  Opnd B{Cw + oJ, ldc, mpad, NB, false};
  tile_mm(acc, A, B, mpad, tl);
  const int t = threadIdx.x, ty = t >> 4, tx = t & 15;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      const int64_t r = oI + ty * 4 + i, c = oJ + tx * 4 + j;
      const double v = inv_nu2 * ((r == c ? 1.0 : 0.0) - acc[i][j]);
      H[r * ldh + c] = v;
      H[c * ldh + r] = v;
    }
}

// ------------------------------------------------------------------ driver
static inline int64_t pad64(int64_t v) { return (v + NB - 1) / NB * NB; }

// Split of the Gram's summed dimension (the number of partial products).
static void gram_split(int64_t m, int64_t d, int& nsplit, int64_t& qchunk) {
  const bool wood = m < d;
  const int64_t p = wood ? m : d;
  const int nblk = (int)(pad64(p) / NB);
  const int64_t tiles = (int64_t)nblk * (nblk + 1) / 2;
  const int64_t q = wood ? d : m;
  const int64_t cus = device_cus();
  nsplit = (int)std::max<int64_t>(1, std::min<int64_t>((2 * cus + tiles - 1) / tiles,
                                                       (q + 255) / 256));
  nsplit = std::min(nsplit, 16);
  qchunk = ((q + nsplit - 1) / nsplit + 15) / 16 * 16;
  nsplit = (int)((q + qchunk - 1) / qchunk);
}

int gram_partial_count(int64_t m, int64_t d) {
  int ns;
  int64_t qc;
  gram_split(m, d, ns, qc);
  return ns;
}

// 1. Gram partial products of SA into F.gram (FP32, or FP64 for FP64 SA)
rs_status gram_partials(const FactorBuffers& F, const void* SA, rs_dtype sa_t,
                        const float* colscale, int64_t m, int64_t d, int64_t ldsa, hipStream_t s) {
  const bool wood = m < d;
  const int64_t p = wood ? m : d;
  const int64_t pp = pad64(p);
  const int nblk = (int)(pp / NB);
  const int64_t tiles = (int64_t)nblk * (nblk + 1) / 2;
  // 1. Gram, split over the summed dimension so that the launch fills the chip
  const int64_t q = wood ? d : m;
  int nsplit;
  int64_t qchunk;
  gram_split(m, d, nsplit, qchunk);
  const dim3 gg((unsigned)tiles, (unsigned)nsplit);
  const size_t esz = sa_t == RS_F64 ? 8 : 4;
  // the low-precision TN kernel reads 16-byte vectors of 64-column segments: it
  // needs 16-byte aligned rows and a padded width (columns up to pad64(d) exist)
  const size_t lpes = sa_t == RS_BF16 ? 2 : 1;
  const bool lp_ok = (sa_t == RS_BF16 || sa_t == RS_FP8E4M3) &&
                     ((uintptr_t)SA % 16 == 0) && ((ldsa * lpes) % 16 == 0) && ldsa >= pp;
  // the pipelined BF16 kernel reads 8-element groups: rows 16-byte aligned and
  // the summed (NT) or column (TN) extent readable up to a multiple of 8
  const bool bf16_ok = sa_t == RS_BF16 && ((uintptr_t)SA % 16 == 0) && (ldsa % 8 == 0) &&
                       ldsa >= (wood ? (d + 7) / 8 * 8 : (p + 7) / 8 * 8);
  if ((size_t)nsplit * pp * pp * esz > F.gram_bytes)
    return set_error(RS_ERR_ARG, "factor: Gram scratch too small");
  if (sa_t == RS_F32) {
    const float* X = reinterpret_cast<const float*>(SA);
    float* P = reinterpret_cast<float*>(F.gram);
    if (wood)
      hipLaunchKernelGGL((k_gram<float, float, false>), gg, dim3(256), 0, s, X, ldsa, p, q, qchunk, P, pp, (const float*)nullptr);
    else
      hipLaunchKernelGGL((k_gram<float, float, true>), gg, dim3(256), 0, s, X, ldsa, p, q, qchunk, P, pp, (const float*)nullptr);
  } else if (sa_t == RS_F64) {
    const double* X = reinterpret_cast<const double*>(SA);
    double* P = reinterpret_cast<double*>(F.gram);
    if (wood)
      hipLaunchKernelGGL((k_gram<double, double, false>), gg, dim3(256), 0, s, X, ldsa, p, q, qchunk, P, pp, (const float*)nullptr);
    else
      hipLaunchKernelGGL((k_gram<double, double, true>), gg, dim3(256), 0, s, X, ldsa, p, q, qchunk, P, pp, (const float*)nullptr);
  } else if (sa_t == RS_BF16 && bf16_ok) {
    float* P = reinterpret_cast<float*>(F.gram);
    const uint16_t* X = reinterpret_cast<const uint16_t*>(SA);
    if (wood)
      hipLaunchKernelGGL(k_gram_bf16<false>, gg, dim3(256), 0, s, X, ldsa, p, q, qchunk, P, pp);
    else
      hipLaunchKernelGGL(k_gram_bf16<true>, gg, dim3(256), 0, s, X, ldsa, p, q, qchunk, P, pp);
  } else if (sa_t == RS_FP8E4M3 && !wood && lp_ok) {
    float* P = reinterpret_cast<float*>(F.gram);
    hipLaunchKernelGGL(k_gram_lp_tn<uint8_t>, gg, dim3(256), 0, s,
                       reinterpret_cast<const uint8_t*>(SA), ldsa, p, q, qchunk, P, pp, colscale);
  } else if (sa_t == RS_BF16) {
    const uint16_t* X = reinterpret_cast<const uint16_t*>(SA);
    float* P = reinterpret_cast<float*>(F.gram);
    if (wood)
      hipLaunchKernelGGL((k_gram<uint16_t, float, false>), gg, dim3(256), 0, s, X, ldsa, p, q, qchunk, P, pp, (const float*)nullptr);
    else
      hipLaunchKernelGGL((k_gram<uint16_t, float, true>), gg, dim3(256), 0, s, X, ldsa, p, q, qchunk, P, pp, (const float*)nullptr);
  } else if (sa_t == RS_FP8E4M3) {
    const uint8_t* X = reinterpret_cast<const uint8_t*>(SA);
    float* P = reinterpret_cast<float*>(F.gram);
    if (wood)
      hipLaunchKernelGGL((k_gram<uint8_t, float, false>), gg, dim3(256), 0, s, X, ldsa, p, q, qchunk, P, pp, colscale);
    else
      hipLaunchKernelGGL((k_gram<uint8_t, float, true>), gg, dim3(256), 0, s, X, ldsa, p, q, qchunk, P, pp, colscale);
  } else {
    return set_error(RS_ERR_UNSUPPORTED, "factor: SA dtype not supported");
  }
  return check_launch("gram");
}

// 2.-3. For B shifted copies of one Gram (nu2[z], or the scalar nu2 when B = 1
// and nu2_dev is null): M_z = Gram + nu2_z I, Cholesky + Linv, explicit inverse
// into F.Hinv + z * zb.sH.  M, Linv, Cw advance by zb.sM, zb.sL, zb.sC per z.
rs_status factor_finish(const FactorBuffers& F, const void* SA, rs_dtype sa_t,
                        const float* colscale, int64_t m, int64_t d, int64_t ldsa, double nu2,
                        int B, FactorBatch zb, hipStream_t s) {
  const bool wood = m < d;
  const int64_t p = wood ? m : d;
  const int64_t pp = pad64(p);
  const int nblk = (int)(pp / NB);
  const int64_t tiles = (int64_t)nblk * (nblk + 1) / 2;
  const unsigned Bz = (unsigned)B;
  int nsplit;
  int64_t qchunk;
  gram_split(m, d, nsplit, qchunk);
  // (the reduction also starts the L^-1 buffer as the identity)
  if (sa_t == RS_F64)
    hipLaunchKernelGGL(k_gram_reduce<double>, dim3((unsigned)tiles, 1, Bz), dim3(256), 0, s,
                       reinterpret_cast<const double*>(F.gram), nsplit, p, nu2, F.M, pp, zb,
                       F.Linv);
  else
    hipLaunchKernelGGL(k_gram_reduce<float>, dim3((unsigned)tiles, 1, Bz), dim3(256), 0, s,
                       reinterpret_cast<const float*>(F.gram), nsplit, p, nu2, F.M, pp, zb,
                       F.Linv);
  // 2. Cholesky + Linv
  for (int k = 0; k < nblk; ++k) {
    const int nrest = nblk - 1 - k;
    const int64_t nfac = 1 + nrest + k;
    const int64_t nupd = k > 0 ? (int64_t)nrest * (nrest + 1) / 2 + (int64_t)nrest * k : 0;
    hipLaunchKernelGGL(k_chol_step, dim3((unsigned)(nfac + nupd), 1, Bz), dim3(256), 0, s, F.M,
                       pp, k, nblk, F.Linv, F.info, p, zb);
  }
  // 3. explicit inverse (skipped when the caller only needs L and L^-1; the
  //    Woodbury route with cw_only stops at the whitened sketch)
  if (!F.Hinv && !(wood && F.cw_only)) return check_launch("factor");
  const int64_t dp = pad64(d);
  if (!wood) {
    const int ch = lauum_chunk(nblk);
    const int nsplit = (nblk + ch - 1) / ch;
    const size_t need = (size_t)nsplit * tiles * NB * NB * sizeof(double);
    if (B == 1 && nsplit > 1 && F.Cw && F.cw_bytes >= need) {
      hipLaunchKernelGGL(k_lauum_part, dim3((unsigned)tiles, (unsigned)nsplit), dim3(256), 0, s,
                         F.Linv, pp, nblk, ch, F.Cw);
      hipLaunchKernelGGL(k_lauum_sum, dim3((unsigned)tiles), dim3(256), 0, s, F.Cw, nblk, ch,
                         nsplit, F.Hinv, dp);
    } else {
      hipLaunchKernelGGL(k_lauum, dim3((unsigned)tiles, 1, Bz), dim3(256), 0, s, F.Linv, pp, nblk,
                         F.Hinv, dp, zb);
    }
  } else {
    const dim3 g2((unsigned)(dp / NB), (unsigned)nblk, Bz);
    if (sa_t == RS_F32) {
      FOpnd Bo{reinterpret_cast<const float*>(SA), ldsa, m, d, false};
      hipLaunchKernelGGL((k_whiten<FOpnd>), g2, dim3(256), 0, s, F.Linv, pp, Bo, d, F.Cw, dp,
                         zb);
    } else if (sa_t == RS_F64) {
      Opnd Bo{reinterpret_cast<const double*>(SA), ldsa, m, d, false};
      hipLaunchKernelGGL((k_whiten<Opnd>), g2, dim3(256), 0, s, F.Linv, pp, Bo, d, F.Cw, dp,
                         zb);
    } else if (sa_t == RS_BF16) {
      HOpnd Bo{reinterpret_cast<const uint16_t*>(SA), ldsa, m, d, false};
      hipLaunchKernelGGL((k_whiten<HOpnd>), g2, dim3(256), 0, s, F.Linv, pp, Bo, d, F.Cw, dp,
                         zb);
    } else {
      QOpnd Bo{reinterpret_cast<const uint8_t*>(SA), ldsa, m, d, false, colscale};
      hipLaunchKernelGGL((k_whiten<QOpnd>), g2, dim3(256), 0, s, F.Linv, pp, Bo, d, F.Cw, dp,
                         zb);
    }
    if (F.cw_only) return check_launch("factor");
    const int dblk = (int)(dp / NB);
    hipLaunchKernelGGL(k_woodbury_inv, dim3((unsigned)(dblk * (dblk + 1) / 2), 1, Bz), dim3(256),
                       0, s, F.Cw, dp, pp, 1.0 / nu2, dp, F.Hinv, dp, zb);
  }
  return check_launch("factor");
}

rs_status factor_build(const FactorBuffers& F, const void* SA, rs_dtype sa_t,
                       const float* colscale, int64_t m, int64_t d, int64_t ldsa, double nu2,
                       hipStream_t s) {
  const rs_status st = gram_partials(F, SA, sa_t, colscale, m, d, ldsa, s);
  if (st != RS_OK) return st;
  return factor_finish(F, SA, sa_t, colscale, m, d, ldsa, nu2, 1, FactorBatch{}, s);
}

size_t factor_bytes_M(int64_t m, int64_t d) {
  const int64_t p = m < d ? m : d;
  return (size_t)pad64(p) * pad64(p) * sizeof(double);
}
size_t factor_bytes_gram(int64_t m, int64_t d, rs_dtype sa_t) {
  const int64_t p = m < d ? m : d;
  const int64_t pp = pad64(p);
  return (size_t)16 * pp * pp * (sa_t == RS_F64 ? 8 : 4);
}
size_t factor_bytes_Hinv(int64_t d) { return (size_t)pad64(d) * pad64(d) * sizeof(double); }
size_t factor_bytes_Cw(int64_t m, int64_t d) {
  if (m < d) return (size_t)pad64(m) * pad64(d) * sizeof(double);
  // m >= d: partial products of the split LinvT Linv
  const int nblk = (int)(pad64(d) / NB);
  const int ch = lauum_chunk(nblk);
  const int64_t tiles = (int64_t)nblk * (nblk + 1) / 2;
  return (size_t)((nblk + ch - 1) / ch) * tiles * NB * NB * sizeof(double);
}

}  // namespace rs
