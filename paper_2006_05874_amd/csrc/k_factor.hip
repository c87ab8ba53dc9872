// Factor of the sketched Hessian H_S = (SA)^T SA + nu^2 I (eq. EqnApproximateHessian).
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

template <typename TIn, typename TAcc, bool TN>
__global__ __launch_bounds__(256) void k_gram(const TIn* __restrict__ src, int64_t ld, int64_t p,
                                              int64_t q, double nu2, double* __restrict__ C,
                                              int64_t ldc) {
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

  for (int64_t l0 = 0; l0 < q; l0 += KC) {
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
      if (l < q) {
        if (ia < p) va = load_as<TAcc>(TN ? src[l * ld + ia] : src[ia * ld + l]);
        if (ja < p) vb = load_as<TAcc>(TN ? src[l * ld + ja] : src[ja * ld + l]);
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
  // lane holds column lane % 16 of each 16x16 tile, rows per mfma16_row
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int b = 0; b < 2; ++b)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t i = i0 + wr * 32 + a * 16 + mfma16_row<TAcc>(lane, r);
        const int64_t j = j0 + wc * 32 + b * 16 + (lane & 15);
        double v = (double)acc[a][b][r];
        if (i == j) v += nu2;
        if (i >= p || j >= p) v = (i == j) ? 1.0 : 0.0;
        C[i * ldc + j] = v;
        if (I != J) C[j * ldc + i] = v;
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
  if (r >= o.rows || c >= o.cols) return 0.0;
  return o.trans ? o.p[c * o.ld + r] : o.p[r * o.ld + c];
}

struct FOpnd {  // FP32 source, same addressing
  const float* p;
  int64_t ld;
  int64_t rows, cols;
  bool trans;
};
__device__ __forceinline__ double opnd_at(const FOpnd& o, int64_t r, int64_t c) {
  if (r >= o.rows || c >= o.cols) return 0.0;
  return (double)(o.trans ? o.p[c * o.ld + r] : o.p[r * o.ld + c]);
}
struct HOpnd {  // BF16 source
  const uint16_t* p;
  int64_t ld;
  int64_t rows, cols;
  bool trans;
};
__device__ __forceinline__ double opnd_at(const HOpnd& o, int64_t r, int64_t c) {
  if (r >= o.rows || c >= o.cols) return 0.0;
  return (double)bf16_to_f32(o.trans ? o.p[c * o.ld + r] : o.p[r * o.ld + c]);
}

template <typename OA, typename OB>
__device__ void tile_mm(double (&acc)[4][4], const OA& A, const OB& B, int64_t kd,
                        double (*As)[NB + 1], double (*Bs)[NB + 1]) {
  const int t = threadIdx.x;
  const int ty = t >> 4, tx = t & 15;
  for (int64_t k0 = 0; k0 < kd; k0 += 16) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int idx = t * 4 + e;
      const int r = idx >> 4, kk = idx & 15;     // A: 64 rows x 16 k
      As[kk][r] = opnd_at(A, r, k0 + kk);
      const int kb = idx >> 6, cb = idx & 63;    // B: 16 k x 64 cols
      Bs[kb][cb] = opnd_at(B, k0 + kb, cb);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) {
      double a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kk][ty * 4 + i];
#pragma unroll
      for (int j = 0; j < 4; ++j) b[j] = Bs[kk][tx * 4 + j];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = fma(a[i], b[j], acc[i][j]);
    }
    __syncthreads();
  }
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
//   diag  : L_kk (in place in M) and Linv_kk = L_kk^-1 (into the Linv buffer);
//   panel : L_ik = M_ik Linv_kk^T (i > k), and X_kj = Linv_kk Y_kj (j < k);
//   update: M_ij -= L_ik L_jk^T (k < j <= i), Y_ij -= L_ik X_kj (i > k, j <= k).
// Every step adds one 64^3 tile product to the critical path.

// Diagonal tile k: factor in LDS (right-looking, one column per step), then
// invert the 64x64 lower factor by forward substitution row by row.
__global__ __launch_bounds__(256) void k_chol_diag(double* __restrict__ M, int64_t ld, int k,
                                                   double* __restrict__ Linv,
                                                   int* __restrict__ info) {
  __shared__ double a[NB][NB + 1];
  __shared__ double x[NB][NB + 1];
  __shared__ double dg[NB];
  const int t = threadIdx.x;
  const int64_t o = (int64_t)k * NB;
  for (int idx = t; idx < NB * NB; idx += 256) {
    const int i = idx / NB, j = idx % NB;
    a[i][j] = M[(o + i) * ld + o + j];
    x[i][j] = 0.0;
  }
  for (int j = 0; j < NB; ++j) {
    __syncthreads();
    const double piv = a[j][j];
    const bool bad = !(piv > 0.0);
    const double sq = bad ? __builtin_nan("") : sqrt(piv);
    if (t == 0) {
      dg[j] = sq;
      if (bad) atomicExch(info, 1);
    }
    if (t > j && t < NB) a[t][j] = a[t][j] / sq;
    __syncthreads();
    const int rem = NB - 1 - j;
    for (int idx = t; idx < rem * rem; idx += 256) {
      const int i = j + 1 + idx / rem, l = j + 1 + idx % rem;
      if (l <= i) a[i][l] -= a[i][j] * a[l][j];
    }
  }
  __syncthreads();
  if (t < NB) a[t][t] = dg[t];
  __syncthreads();
  for (int i = 0; i < NB; ++i) {
    if (t <= i) {
      double sm = (t == i) ? 1.0 : 0.0;
      for (int l = t; l < i; ++l) sm -= a[i][l] * x[l][t];
      x[i][t] = sm / a[i][i];
    }
    __syncthreads();
  }
  for (int idx = t; idx < NB * NB; idx += 256) {
    const int i = idx / NB, j = idx % NB;
    M[(o + i) * ld + o + j] = j <= i ? a[i][j] : 0.0;
    Linv[(o + i) * ld + o + j] = j <= i ? x[i][j] : 0.0;
  }
}

// Blocks [0, nrest): L_ik = M_ik Linv_kk^T, i = k + 1 + b.
// Blocks [nrest, nrest + k): X_kj = Linv_kk Y_kj in place, j = b - nrest.
__global__ __launch_bounds__(256) void k_chol_panel(double* __restrict__ M, int64_t ld, int k,
                                                    int nrest, double* __restrict__ Linv) {
  __shared__ double As[16][NB + 1];
  __shared__ double Bs[16][NB + 1];
  const int t = threadIdx.x;
  const int ty = t >> 4, tx = t & 15;
  const int64_t ok = (int64_t)k * NB;
  double acc[4][4];
  zero_acc(acc);
  double* dst;
  int64_t ldd = ld;
  if ((int)blockIdx.x < nrest) {
    const int64_t oi = ok + (int64_t)(blockIdx.x + 1) * NB;
    Opnd A{M + oi * ld + ok, ld, NB, NB, false};
    Opnd B{Linv + ok * ld + ok, ld, NB, NB, true};
    tile_mm(acc, A, B, NB, As, Bs);
    dst = M + oi * ld + ok;
  } else {
    const int64_t oj = (int64_t)(blockIdx.x - nrest) * NB;
    Opnd A{Linv + ok * ld + ok, ld, NB, NB, false};
    Opnd B{Linv + ok * ld + oj, ld, NB, NB, false};
    tile_mm(acc, A, B, NB, As, Bs);
    dst = Linv + ok * ld + oj;
  }
  // tile_mm ends with a barrier: every read of the destination tile is done
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) dst[(int64_t)(ty * 4 + i) * ldd + tx * 4 + j] = acc[i][j];
}

// Blocks [0, tri(nrest)): M_ij -= L_ik L_jk^T for k < j <= i.
// Blocks [tri(nrest), + nrest*(k+1)): Y_ij -= L_ik X_kj for i > k, j <= k.
__global__ __launch_bounds__(256) void k_chol_update(double* __restrict__ M, int64_t ld, int k,
                                                     int nrest, double* __restrict__ Linv) {
  __shared__ double As[16][NB + 1];
  __shared__ double Bs[16][NB + 1];
  const int64_t tri = (int64_t)nrest * (nrest + 1) / 2;
  const int64_t bid = blockIdx.x;
  const int64_t ok = (int64_t)k * NB;
  double acc[4][4];
  zero_acc(acc);
  double* dst;
  if (bid < tri) {
    int64_t I = (int64_t)((sqrt(8.0 * (double)bid + 1.0) - 1.0) * 0.5);
    while ((I + 1) * (I + 2) / 2 <= bid) ++I;
    while (I * (I + 1) / 2 > bid) --I;
    const int64_t J = bid - I * (I + 1) / 2;
    const int64_t oi = (k + 1 + I) * NB, oj = (k + 1 + J) * NB;
    Opnd A{M + oi * ld + ok, ld, NB, NB, false};
    Opnd B{M + oj * ld + ok, ld, NB, NB, true};
    tile_mm(acc, A, B, NB, As, Bs);
    dst = M + oi * ld + oj;
  } else {
    const int64_t r = bid - tri;
    const int64_t I = r / (k + 1), J = r % (k + 1);
    const int64_t oi = (k + 1 + I) * NB, oj = J * NB;
    Opnd A{M + oi * ld + ok, ld, NB, NB, false};
    Opnd B{Linv + ok * ld + oj, ld, NB, NB, false};
    tile_mm(acc, A, B, NB, As, Bs);
    dst = Linv + oi * ld + oj;
  }
  const int t = threadIdx.x, ty = t >> 4, tx = t & 15;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) dst[(int64_t)(ty * 4 + i) * ld + tx * 4 + j] -= acc[i][j];
}

// Linv buffer <- identity (p x p).
__global__ __launch_bounds__(256) void k_fill_identity(double* __restrict__ X, int64_t p) {
  const int64_t total = p * p;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total;
       i += (int64_t)gridDim.x * 256)
    X[i] = (i / p == i % p) ? 1.0 : 0.0;
}

// Hinv = Linv^T Linv (p x p, both triangles): tile (I, J), J <= I:
// sum_{l >= I} Linv_lI^T Linv_lJ.
__global__ __launch_bounds__(256) void k_lauum(const double* __restrict__ Linv, int64_t ld,
                                               int nblk, double* __restrict__ H, int64_t ldh) {
  __shared__ double As[16][NB + 1];
  __shared__ double Bs[16][NB + 1];
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
  tile_mm(acc, A, B, rows, As, Bs);
  const int t = threadIdx.x, ty = t >> 4, tx = t & 15;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      H[(oI + ty * 4 + i) * ldh + oJ + tx * 4 + j] = acc[i][j];
      H[(oJ + tx * 4 + j) * ldh + oI + ty * 4 + i] = acc[i][j];
    }
}

// C = Linv SA (m x d): tile (I over m, Jd over d): sum_{l <= I} Linv_Il SA_l.
template <typename OSA>
__global__ __launch_bounds__(256) void k_whiten(const double* __restrict__ Linv, int64_t ld,
                                                OSA SA, int64_t d, double* __restrict__ Cw,
                                                int64_t ldc) {
  __shared__ double As[16][NB + 1];
  __shared__ double Bs[16][NB + 1];
  const int64_t I = blockIdx.y, Jd = blockIdx.x;
  double acc[4][4];
  zero_acc(acc);
  const int64_t oI = I * NB, oJ = Jd * NB;
  Opnd A{Linv + oI * ld, ld, NB, (I + 1) * NB, false};
  OSA B = SA;
  B.p = SA.p + oJ;
  B.cols = d - oJ;
  tile_mm(acc, A, B, (I + 1) * NB, As, Bs);
  const int t = threadIdx.x, ty = t >> 4, tx = t & 15;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) Cw[(oI + ty * 4 + i) * ldc + oJ + tx * 4 + j] = acc[i][j];
}

// Hinv = nu^-2 (I - C^T C) over d x d (both triangles), C padded with zero rows.
__global__ __launch_bounds__(256) void k_woodbury_inv(const double* __restrict__ Cw, int64_t ldc,
                                                      int64_t mpad, double inv_nu2, int64_t dp,
                                                      double* __restrict__ H, int64_t ldh) {
  __shared__ double As[16][NB + 1];
  __shared__ double Bs[16][NB + 1];
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
  tile_mm(acc, A, B, mpad, As, Bs);
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

rs_status factor_build(const FactorBuffers& F, const void* SA, rs_dtype sa_t, int64_t m, int64_t d,
                       int64_t ldsa, double nu2, hipStream_t s) {
  const bool wood = m < d;
  const int64_t p = wood ? m : d;
  const int64_t pp = pad64(p);
  const int nblk = (int)(pp / NB);
  const int64_t tiles = (int64_t)nblk * (nblk + 1) / 2;
  // 1. Gram
  if (sa_t == RS_F32) {
    const float* X = reinterpret_cast<const float*>(SA);
    if (wood)
      hipLaunchKernelGGL((k_gram<float, float, false>), dim3((unsigned)tiles), dim3(256), 0, s, X,
                         ldsa, p, d, nu2, F.M, pp);
    else
      hipLaunchKernelGGL((k_gram<float, float, true>), dim3((unsigned)tiles), dim3(256), 0, s, X,
                         ldsa, p, m, nu2, F.M, pp);
  } else if (sa_t == RS_F64) {
    const double* X = reinterpret_cast<const double*>(SA);
    if (wood)
      hipLaunchKernelGGL((k_gram<double, double, false>), dim3((unsigned)tiles), dim3(256), 0, s,
                         X, ldsa, p, d, nu2, F.M, pp);
    else
      hipLaunchKernelGGL((k_gram<double, double, true>), dim3((unsigned)tiles), dim3(256), 0, s,
                         X, ldsa, p, m, nu2, F.M, pp);
  } else if (sa_t == RS_BF16) {
    const uint16_t* X = reinterpret_cast<const uint16_t*>(SA);
    if (wood)
      hipLaunchKernelGGL((k_gram<uint16_t, float, false>), dim3((unsigned)tiles), dim3(256), 0, s,
                         X, ldsa, p, d, nu2, F.M, pp);
    else
      hipLaunchKernelGGL((k_gram<uint16_t, float, true>), dim3((unsigned)tiles), dim3(256), 0, s,
                         X, ldsa, p, m, nu2, F.M, pp);
  } else {
    return set_error(RS_ERR_UNSUPPORTED, "factor: SA dtype not supported");
  }
  // 2. Cholesky + Linv
  {
    const int64_t tot = pp * pp;
    const unsigned g = (unsigned)std::min<int64_t>((tot + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill_identity, dim3(g), dim3(256), 0, s, F.Linv, pp);
  }
  for (int k = 0; k < nblk; ++k) {
    hipLaunchKernelGGL(k_chol_diag, dim3(1), dim3(256), 0, s, F.M, pp, k, F.Linv, F.info);
    const int nrest = nblk - 1 - k;
    if (nrest + k > 0)
      hipLaunchKernelGGL(k_chol_panel, dim3((unsigned)(nrest + k)), dim3(256), 0, s, F.M, pp, k,
                         nrest, F.Linv);
    if (nrest > 0) {
      const int64_t nb_upd = (int64_t)nrest * (nrest + 1) / 2 + (int64_t)nrest * (k + 1);
      hipLaunchKernelGGL(k_chol_update, dim3((unsigned)nb_upd), dim3(256), 0, s, F.M, pp, k,
                         nrest, F.Linv);
    }
  }
  // 3. explicit inverse
  const int64_t dp = pad64(d);
  if (!wood) {
    hipLaunchKernelGGL(k_lauum, dim3((unsigned)tiles), dim3(256), 0, s, F.Linv, pp, nblk, F.Hinv,
                       dp);
  } else {
    const dim3 g2((unsigned)(dp / NB), (unsigned)nblk);
    if (sa_t == RS_F32) {
      FOpnd B{reinterpret_cast<const float*>(SA), ldsa, m, d, false};
      hipLaunchKernelGGL((k_whiten<FOpnd>), g2, dim3(256), 0, s, F.Linv, pp, B, d, F.Cw, dp);
    } else if (sa_t == RS_F64) {
      Opnd B{reinterpret_cast<const double*>(SA), ldsa, m, d, false};
      hipLaunchKernelGGL((k_whiten<Opnd>), g2, dim3(256), 0, s, F.Linv, pp, B, d, F.Cw, dp);
    } else {
      HOpnd B{reinterpret_cast<const uint16_t*>(SA), ldsa, m, d, false};
      hipLaunchKernelGGL((k_whiten<HOpnd>), g2, dim3(256), 0, s, F.Linv, pp, B, d, F.Cw, dp);
    }
    const int dblk = (int)(dp / NB);
    hipLaunchKernelGGL(k_woodbury_inv, dim3((unsigned)(dblk * (dblk + 1) / 2)), dim3(256), 0, s,
                       F.Cw, dp, pp, 1.0 / nu2, dp, F.Hinv, dp);
  }
  return check_launch("factor");
}

size_t factor_bytes_M(int64_t m, int64_t d) {
  const int64_t p = m < d ? m : d;
  return (size_t)pad64(p) * pad64(p) * sizeof(double);
}
size_t factor_bytes_Hinv(int64_t d) { return (size_t)pad64(d) * pad64(d) * sizeof(double); }
size_t factor_bytes_Cw(int64_t m, int64_t d) {
  return m < d ? (size_t)pad64(m) * pad64(d) * sizeof(double) : 0;
}

}  // namespace rs
