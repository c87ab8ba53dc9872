// Kernels of the nu-grid form: many regularisation values on one A.
//
// The sketch S A, and with it the Gram (SA)^T SA or SA (SA)^T, does not depend
// on nu (Section 3: the sketched Hessian is (SA)^T SA + nu^2 I).  With fresh
// resampling every level m = m_init 2^L draws sketch_id L, and with nested
// resampling every level keeps sketch_id 0: in both cases all nu values at one
// level share the sketch and the Gram, and only the shifted factors differ.
//
// The gradients A^T (A x - b) + nu^2 x of all candidates of all active nu form
// one multi-right-hand-side product: R = A X^T - b 1^T (n x Kc), then
// G = A^T R (d x Kc) split over row chunks, both on the matrix cores (FP32
// MFMA 16x16x4 for FP32 A, FP64 MFMA for FP64 A); FP32 chunk sums are moved to
// FP64 every 256 rows.  The per-nu step kernels (candidates, apply, decide,
// resample bookkeeping) run as one launch over the active list: block row y
// serves list entry y, whose slot is zl[y].
#include <hip/hip_cooperative_groups.h>

#include "rs_internal.hpp"

namespace rs {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
using Acc4 = typename std::conditional<sizeof(T) == 4, f32x4, f64x4>::type;

template <typename T>
__device__ __forceinline__ Acc4<T> mfma4(T a, T b, Acc4<T> c) {
  if constexpr (sizeof(T) == 4)
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Eight consecutive elements at p (16-byte aligned) as 16-byte loads.
template <typename T>
__device__ __forceinline__ void load8(const T* __restrict__ p, T (&v)[8]) {
  using V = typename VecOf<T>::type;
  constexpr int VEC = VecOf<T>::n;
#pragma unroll
  for (int q = 0; q < 8 / VEC; ++q) {
    const V x = reinterpret_cast<const V*>(p)[q];
#pragma unroll
    for (int e = 0; e < VEC; ++e) v[q * VEC + e] = get(x, e);
  }
}

// ---------------------------------------------------------------- R = A X^T - b
// Block: 128 rows x TC columns of R (TC = 32, 64 or 128, the narrowest that holds
// Kc), 8 waves of 32 rows x TC/2 columns (two waves per SIMD); k (the d dimension)
// in chunks of 32 through LDS.  XT is X (Kc x d)
// already in T.  Block b covers column block b % ncb of row block b / ncb, so
// the blocks that read one row panel of A run next to each other.
// The tile body (bx: the tile, As / Xs: the block's LDS) serves this kernel and
// the persistent step kernel below.
template <typename T, int TC>
__device__ __forceinline__ void mr_resid_tile(int64_t bx, const T* __restrict__ A, int64_t n,
                                              int64_t d, int64_t lda, const T* __restrict__ b,
                                              const T* __restrict__ XT, int64_t Kc,
                                              T* __restrict__ R, int64_t ldr, int ncb,
                                              T (*As)[129], T (*Xs)[TC + 1]) {
  constexpr int TM = 128, KC = 32, NC = TC / 32;  // NC 16-column tiles per wave
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wr = w & 3, wc = w >> 2;  // wave tile: rows wr*32.., columns wc*TC/2..
  const int64_t r0 = (bx / ncb) * TM;
  const int64_t c0 = (bx % ncb) * TC;
  Acc4<T> acc[2][NC];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < NC; ++c) acc[a][c] = Acc4<T>{0, 0, 0, 0};
  // loader mapping: thread -> (row or column = t / 4, 8 consecutive k); the next
  // chunk is fetched into registers while the current one is multiplied
  const int lrow = t >> 2, lk = (t & 3) * 8;
  const int64_t arow = r0 + lrow, xcol = c0 + lrow;
  const bool rok = arow < n, cok = lrow < TC && xcol < Kc;
  const T* asrc = A + (rok ? arow : 0) * lda;
  const T* xsrc = XT + (cok ? xcol : 0) * d;
  // rows of A are 16-byte aligned (lda a multiple of 16 bytes); rows of XT when d is
  constexpr int VEC = VecOf<T>::n;
  const bool xvec = d % VEC == 0;
  T va[8], vx[8];
  auto fetch = [&](int64_t k0) {
    const int64_t kb = k0 + lk;
    if (kb + 8 <= d) {
      // a whole segment: 16-byte loads (the same values as the element loads)
      if (rok) {
        load8<T>(asrc + kb, va);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) va[e] = (T)0;
      }
      if (cok && xvec) {
        load8<T>(xsrc + kb, vx);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) {
          const T y = xsrc[cok ? kb + e : 0];
          vx[e] = cok ? y : (T)0;
        }
      }
      return;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t k = kb + e;
      const bool okk = k < d;
      const T x = asrc[(rok && okk) ? k : 0];
      const T y = xsrc[(cok && okk) ? k : 0];
      va[e] = (rok && okk) ? x : (T)0;
      vx[e] = (cok && okk) ? y : (T)0;
    }
  };
  fetch(0);
  for (int64_t k0 = 0; k0 < d; k0 += KC) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      As[lk + e][lrow] = va[e];
      if (lrow < TC) Xs[lk + e][lrow] = vx[e];
    }
    __syncthreads();
    if (k0 + KC < d) fetch(k0 + KC);
#pragma unroll
    for (int k4 = 0; k4 < KC / 4; ++k4) {
      const int kr = k4 * 4 + (lane >> 4);
      T av[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[kr][wr * 32 + a * 16 + (lane & 15)];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const T bv = Xs[kr][wc * (TC / 2) + c * 16 + (lane & 15)];
#pragma unroll
        for (int a = 0; a < 2; ++a) acc[a][c] = mfma4<T>(av[a], bv, acc[a][c]);
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t row = r0 + wr * 32 + a * 16 + mfma16_row<T>(lane, r);
      if (row < n) {
        const T bv = b[row];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const int64_t col = c0 + wc * (TC / 2) + c * 16 + (lane & 15);
          if (col < Kc) R[row * ldr + col] = acc[a][c][r] - bv;
        }
      }
    }
}

template <typename T, int TC>
__global__ __launch_bounds__(512) void k_mr_resid(const T* __restrict__ A, int64_t n, int64_t d,
                                                  int64_t lda, const T* __restrict__ b,
                                                  const T* __restrict__ XT, int64_t Kc,
                                                  T* __restrict__ R, int64_t ldr, int ncb,
                                                  int* __restrict__ ran) {
  if (ran && blockIdx.x == 0 && threadIdx.x == 0) *ran = 1;
  __shared__ T As[32][129];
  __shared__ T Xs[32][TC + 1];
  mr_resid_tile<T, TC>(blockIdx.x, A, n, d, lda, b, XT, Kc, R, ldr, ncb, As, Xs);
}

// ---------------------------------------------------------------- Gp = A^T R per chunk
// Block (tile, split): 128 columns of A (j) x TC columns of R (c) over the
// split's rows, 8 waves of 32 j x TC/2 c; rows in chunks of 32 through LDS.
// Partial layout Gp[split][j][c] (ldr columns), FP64.
template <typename T, int TC>
__device__ __forceinline__ void mr_atr_tile(int64_t bx, int64_t by, const T* __restrict__ A,
                                            int64_t n, int64_t d, int64_t lda,
                                            const T* __restrict__ R, int64_t ldr, int64_t Kc,
                                            int64_t rows_per_split, int ncb,
                                            double* __restrict__ Gp, T (*As)[129],
                                            T (*Rs)[TC + 1]) {
  constexpr int TJ = 128, KC = 32, NC = TC / 32;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int wj = w & 3, wc = w >> 2;
  const int64_t j0 = (bx / ncb) * TJ;
  const int64_t c0 = (bx % ncb) * TC;
  const int64_t row_lo = by * rows_per_split;
  const int64_t row_hi = row_lo + rows_per_split < n ? row_lo + rows_per_split : n;
  Acc4<T> acc[2][NC];
  double acc64[2][NC][4];
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      acc[a][c] = Acc4<T>{0, 0, 0, 0};
#pragma unroll
      for (int r = 0; r < 4; ++r) acc64[a][c][r] = 0.0;
    }
  // loader mapping: thread -> (row = t / 16, 8 consecutive columns); the next
  // chunk is fetched into registers while the current one is multiplied
  const int lr = t >> 4, lc = (t & 15) * 8;
  T va[8], vr[8];
  auto fetch = [&](int64_t k0) {
    const int64_t row = k0 + lr;
    const bool rok = row < row_hi;
    const T* as = A + (rok ? row : 0) * lda;
    const T* rsrc = R + (rok ? row : 0) * ldr;
    // whole 8-element segments as 16-byte loads (A rows and R rows, ldr a multiple
    // of 4 elements, are 16-byte aligned): the same values as the element loads
    const bool wa = j0 + lc + 8 <= d, wr = lc < TC && c0 + lc + 8 <= Kc;
    if (wa && (wr || !(lc < TC))) {
      if (rok) {
        load8<T>(as + j0 + lc, va);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) va[e] = (T)0;
      }
      if (rok && wr) {
        load8<T>(rsrc + c0 + lc, vr);
      } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) vr[e] = (T)0;
      }
      return;
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      const int64_t j = j0 + lc + e, c = c0 + lc + e;
      const bool oj = rok && j < d, oc = rok && lc < TC && c < Kc;
      const T x = as[oj ? j : 0];
      const T y = rsrc[oc ? c : 0];
      va[e] = oj ? x : (T)0;
      vr[e] = oc ? y : (T)0;
    }
  };
  fetch(row_lo);
  int chunk = 0;
  for (int64_t k0 = row_lo; k0 < row_hi; k0 += KC, ++chunk) {
#pragma unroll
    for (int e = 0; e < 8; ++e) {
      As[lr][lc + e] = va[e];
      if (lc < TC) Rs[lr][lc + e] = vr[e];
    }
    __syncthreads();
    if (k0 + KC < row_hi) fetch(k0 + KC);
#pragma unroll
    for (int k4 = 0; k4 < KC / 4; ++k4) {
      const int kr = k4 * 4 + (lane >> 4);
      T av[2];
#pragma unroll
      for (int a = 0; a < 2; ++a) av[a] = As[kr][wj * 32 + a * 16 + (lane & 15)];
#pragma unroll
      for (int c = 0; c < NC; ++c) {
        const T bv = Rs[kr][wc * (TC / 2) + c * 16 + (lane & 15)];
#pragma unroll
        for (int a = 0; a < 2; ++a) acc[a][c] = mfma4<T>(av[a], bv, acc[a][c]);
      }
    }
    __syncthreads();
    if (sizeof(T) == 4 && (chunk & 7) == 7) {
#pragma unroll
      for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int c = 0; c < NC; ++c) {
#pragma unroll
          for (int r = 0; r < 4; ++r) acc64[a][c][r] += (double)acc[a][c][r];
          acc[a][c] = Acc4<T>{0, 0, 0, 0};
        }
    }
  }
  double* out = Gp + by * d * ldr;
#pragma unroll
  for (int a = 0; a < 2; ++a)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int64_t j = j0 + wj * 32 + a * 16 + mfma16_row<T>(lane, r);
      if (j < d) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          const int64_t col = c0 + wc * (TC / 2) + c * 16 + (lane & 15);
          if (col < Kc) out[j * ldr + col] = acc64[a][c][r] + (double)acc[a][c][r];
        }
      }
    }
}

template <typename T, int TC>
__global__ __launch_bounds__(512) void k_mr_atr(const T* __restrict__ A, int64_t n, int64_t d,
                                                int64_t lda, const T* __restrict__ R, int64_t ldr,
                                                int64_t Kc, int64_t rows_per_split, int ncb,
                                                double* __restrict__ Gp) {
  __shared__ T As[32][129];
  __shared__ T Rs[32][TC + 1];
  mr_atr_tile<T, TC>(blockIdx.x, blockIdx.y, A, n, d, lda, R, ldr, Kc, rows_per_split, ncb, Gp,
                     As, Rs);
}

// X (FP64) rounded to T once per sweep.
template <typename T>
__global__ __launch_bounds__(256) void k_round_x(const double* __restrict__ X, int64_t count,
                                                 T* __restrict__ XT) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * 256)
    XT[i] = (T)X[i];
}

// G[c][j] = sum_s Gp[s][j][c] (fixed order) + nu2[zl[c / kper]] X[c][j].
__global__ __launch_bounds__(256) void k_mr_reduce(const double* __restrict__ Gp, int nsplit,
                                                   int64_t d, int64_t ldr, int64_t Kc, int kper,
                                                   const double* __restrict__ X,
                                                   const double* __restrict__ nu2,
                                                   const int* __restrict__ zl,
                                                   double* __restrict__ G) {
  const int64_t total = Kc * d;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * 256) {
    const int64_t c = e % Kc, j = e / Kc;
    double s = 0.0;
    for (int sp = 0; sp < nsplit; ++sp) s += Gp[((int64_t)sp * d + j) * ldr + c];
    const int z = zl[c / kper];
    G[c * d + j] = s + nu2[z] * X[c * d + j];
  }
}

// Column tile of the two products: the narrowest of 32, 64, 128 that holds Kc
// (wider tiles only multiply padding).
static int mr_tc(int64_t Kc) { return Kc <= 32 ? 32 : (Kc <= 64 ? 64 : 128); }

int mr_splits(int64_t n, int64_t d, int64_t Kc, int64_t& rows_per_split) {
  const int tc = mr_tc(Kc);
  const int64_t tiles = ((d + 127) / 128) * ((Kc + tc - 1) / tc);
  const int64_t want = (2 * device_cus() + tiles - 1) / tiles;
  int64_t ns = std::max<int64_t>(1, std::min<int64_t>(want, (n + 255) / 256));
  rows_per_split = ((n + ns - 1) / ns + 31) / 32 * 32;
  ns = (n + rows_per_split - 1) / rows_per_split;
  return (int)ns;
}

template <typename T>
rs_status mr_gradient(const T* A, int64_t n, int64_t d, int64_t lda, const T* b, const double* X,
                      int64_t Kc, int kper, const double* nu2, const int* zl, T* R, int64_t ldr,
                      double* Gp, double* G, T* XT, hipStream_t s) {
  const int tc = mr_tc(Kc);
  const int ncb = (int)((Kc + tc - 1) / tc);
  const int64_t nx = Kc * d;
  const unsigned g0 = (unsigned)std::min<int64_t>((nx + 255) / 256, 4096);
  hipLaunchKernelGGL(k_round_x<T>, dim3(g0), dim3(256), 0, s, X, nx, XT);
  const unsigned g1 = (unsigned)(((n + 127) / 128) * ncb);
  int64_t rps = 0;
  const int ns = mr_splits(n, d, Kc, rps);
  const unsigned g2 = (unsigned)(((d + 127) / 128) * ncb);
  // profiled as one span: the first kernel's start to the second one's stop
  const ProfSlot ps = prof_begin();
#define RS_MR_PASS(TCV)                                                                          \
  launch_timed(k_mr_resid<T, TCV>, dim3(g1), dim3(512), s, ps.begin, nullptr, A, n, d, lda, b,    \
               (const T*)XT, Kc, R, ldr, ncb, ps.ran);                                            \
  launch_timed(k_mr_atr<T, TCV>, dim3(g2, (unsigned)ns), dim3(512), s, nullptr, ps.end, A, n, d,  \
               lda, (const T*)R, ldr, Kc, rps, ncb, Gp)
  if (tc == 32) {
    RS_MR_PASS(32);
  } else if (tc == 64) {
    RS_MR_PASS(64);
  } else {
    RS_MR_PASS(128);
  }
#undef RS_MR_PASS
  const unsigned g3 = (unsigned)std::min<int64_t>((Kc * d + 255) / 256, 4096);
  hipLaunchKernelGGL(k_mr_reduce, dim3(g3), dim3(256), 0, s, Gp, ns, d, ldr, Kc, kper, X, nu2, zl,
                     G);
  return check_launch("multi-rhs gradient");
}

template rs_status mr_gradient<float>(const float*, int64_t, int64_t, int64_t, const float*,
                                      const double*, int64_t, int, const double*, const int*,
                                      float*, int64_t, double*, double*, float*, hipStream_t);
template rs_status mr_gradient<double>(const double*, int64_t, int64_t, int64_t, const double*,
                                       const double*, int64_t, int, const double*, const int*,
                                       double*, int64_t, double*, double*, double*, hipStream_t);

// ---------------------------------------------------------------- batched step kernels
// Slot z (a nu value) owns: x = P.x + z d, vectors P.vec + z 4d (x_prev, g,
// gtilde, g_ref), control record P.ctl[z], event log P.ev + z ev_cap, inverse
// P.Hinv + z sH, decrement partials P.rpart + z nrp 2.  List entry y (slot
// zl[y]) owns the candidate blocks Xc, Gc, GTc + y K d.

__device__ __forceinline__ bool slot_running(const GridPtrs& P, int z) {
  return P.ctl[z].status == RS_CTL_RUNNING;
}

template <int K>
__global__ __launch_bounds__(256) void k_cand_g(GridPtrs P, int64_t d, double mu_p, double beta_p,
                                                double mu_gd) {
  const int y = blockIdx.y, z = P.zl[y];
  if (!slot_running(P, z)) return;
  const double* x = P.x + (int64_t)z * d;
  const double* xp = P.vec + (int64_t)z * 4 * d;
  const double* gt = xp + 2 * d;
  double* X = P.Xc + (int64_t)y * K * d;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < d; i += (int64_t)gridDim.x * 256) {
    const double xi = x[i], gi = gt[i];
    if (K == 2) {
      X[i] = xi - mu_p * gi + beta_p * (xi - xp[i]);
      X[d + i] = xi - mu_gd * gi;
    } else {
      X[i] = xi - mu_gd * gi;
    }
  }
}

// Copy x into the candidate block (first gradient) or [g, g_ref] (resample).
__global__ __launch_bounds__(256) void k_pack_g(GridPtrs P, int64_t d, int what, int kper) {
  const int y = blockIdx.y, z = P.zl[y];
  double* X = P.Xc + (int64_t)y * kper * d;
  const double* v = P.vec + (int64_t)z * 4 * d;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < d; i += (int64_t)gridDim.x * 256) {
    if (what == 0) {
      X[i] = P.x[(int64_t)z * d + i];
    } else {
      X[i] = v[d + i];
      X[d + i] = v[3 * d + i];
    }
  }
}

// GT[y] = Hinv_z G[y] (K columns) and decrement partials; gated on the slot's
// status unless `always`.
template <int K>
__global__ __launch_bounds__(256) void k_symv_g(GridPtrs P, int64_t d, const double* __restrict__ Gsrc,
                                                int always) {
  const int y = blockIdx.y, z = P.zl[y];
  if (!always && !slot_running(P, z)) return;
  symv_rows<K, 1>(P.Hinv + (int64_t)z * P.sH, P.ldh, d, Gsrc + (int64_t)y * K * d,
                  P.GTc + (int64_t)y * K * d, P.rpart + (int64_t)z * P.nrp * 2 + (int64_t)blockIdx.x * K);
}

// Same tests and state moves as the single-problem decision kernel.
template <int K>
__global__ __launch_bounds__(1024) void k_decide_g(GridPtrs P, DecideParams a, int64_t d) {
  const int y = blockIdx.y, z = P.zl[y];
  DevCtl* ctl = P.ctl + z;
  __shared__ double r[K];
  __shared__ double sh[1024 * K];
  __shared__ int chosen;
  if (ctl->status != RS_CTL_RUNNING) return;
  const double* rpart = P.rpart + (int64_t)z * P.nrp * 2;
  block_sum_cols<K, 1024>(rpart, P.nrp, sh, r);
  if (threadIdx.x < K) r[threadIdx.x] *= 0.5;
  __syncthreads();
  if (threadIdx.x == 0) {
    int st = RS_CTL_RUNNING;
    const int64_t t = ctl->t;
    ctl->passes += 1;
    const int rule = step_rule(K == 2, r[0], r[K - 1], ctl->r_t, ctl->r_1, t, ctl->at_cap,
                               a.cbar_p, a.cbar_gd, &st);
    const int c = rule == 0 ? 0 : (rule == 1 ? K - 1 : -1);
    if (c >= 0) {
      const int kind = (K == 2 && c == 0) ? 0 : 1;
      if (t < P.ev_cap) P.ev[(int64_t)z * P.ev_cap + t] = kind;
      if (kind == 0) ctl->polyak += 1; else ctl->gd += 1;
      ctl->r_t = r[c];
      ctl->t = t + 1;
      ctl->steps += 1;
      if (r[c] <= a.tol * ctl->r_ref) st = RS_CTL_CONVERGED;
      else if (t + 1 >= a.max_iter) st = RS_CTL_MAXITER;
    }
    ctl->last_r[0] = r[0];
    ctl->last_r[1] = r[K - 1];
    ctl->status = st;
    chosen = c;
  }
  __syncthreads();
  const int c = chosen;
  if (c < 0) return;
  double* x = P.x + (int64_t)z * d;
  double* v = P.vec + (int64_t)z * 4 * d;
  const double* X = P.Xc + (int64_t)y * K * d;
  const double* G = P.Gc + (int64_t)y * K * d;
  const double* GT = P.GTc + (int64_t)y * K * d;
  for (int64_t i = threadIdx.x; i < d; i += 1024) {
    v[i] = x[i];
    x[i] = X[(int64_t)c * d + i];
    v[d + i] = G[(int64_t)c * d + i];
    v[2 * d + i] = GT[(int64_t)c * d + i];
  }
}

// After the first gradient and apply (one column per slot).
__global__ __launch_bounds__(1024) void k_init_g(GridPtrs P, double tol, int64_t max_iter,
                                                 int64_t d, const int* __restrict__ at_cap) {
  const int y = blockIdx.y, z = P.zl[y];
  DevCtl* ctl = P.ctl + z;
  const double* rpart = P.rpart + (int64_t)z * P.nrp * 2;
  __shared__ double sh[1024];
  __shared__ double rs1[1];
  block_sum_cols<1, 1024>(rpart, P.nrp, sh, rs1);
  if (threadIdx.x == 0) {
    const double r = 0.5 * rs1[0];
    ctl->r_t = r;
    ctl->r_1 = r;
    ctl->r_ref = r;
    ctl->t = 1;
    ctl->steps = 0;
    ctl->passes = 1;
    ctl->polyak = 0;
    ctl->gd = 0;
    ctl->at_cap = at_cap[z];
    int st = start_rule(r, r, tol, at_cap[z]);
    if (st == RS_CTL_RUNNING && 1 >= max_iter) st = RS_CTL_MAXITER;
    ctl->status = st;
  }
  const double* x = P.x + (int64_t)z * d;
  double* v = P.vec + (int64_t)z * 4 * d;
  const double* G = P.Gc + (int64_t)y * d;
  const double* GT = P.GTc + (int64_t)y * d;
  for (int64_t i = threadIdx.x; i < d; i += 1024) {
    v[i] = x[i];
    v[d + i] = G[i];
    v[3 * d + i] = G[i];
    v[2 * d + i] = GT[i];
  }
}

// After a resample: apply was run on [g_t, g_ref] of the slot.
__global__ __launch_bounds__(1024) void k_post_resample_g(GridPtrs P, double tol, int64_t d,
                                                          const int* __restrict__ at_cap) {
  const int y = blockIdx.y, z = P.zl[y];
  DevCtl* ctl = P.ctl + z;
  const double* rpart = P.rpart + (int64_t)z * P.nrp * 2;
  __shared__ double sh[2048];
  __shared__ double s2[2];
  block_sum_cols<2, 1024>(rpart, P.nrp, sh, s2);
  if (threadIdx.x == 0) {
    ctl->r_t = 0.5 * s2[0];
    ctl->r_ref = 0.5 * s2[1];
    ctl->at_cap = at_cap[z];
    const int st = start_rule(ctl->r_t, ctl->r_ref, tol, at_cap[z]);
    // r_1 stays from the start unless the start's own factor was indefinite
    if (st == RS_CTL_RUNNING && !(ctl->r_1 >= 0.0)) ctl->r_1 = ctl->r_t;
    ctl->status = st;
  }
  double* gt = P.vec + (int64_t)z * 4 * d + 2 * d;
  const double* GT = P.GTc + (int64_t)y * 2 * d;
  for (int64_t i = threadIdx.x; i < d; i += 1024) gt[i] = GT[i];
}

// ---------------------------------------------------------------- persistent steps
// One cooperative launch runs up to `iters` steps of every listed nu (candidates,
// the multi-RHS gradient, the apply, the decision), the phases separated by grid
// barriers, and returns early once no listed nu is still running (a converged,
// stopped or doubling nu waits for the host, which resamples and factors between
// launches).  Each phase does exactly what the kernels above do for the same
// list (the same bodies, the same per-element sums in the same order), so the
// results equal those of the separate launches bit for bit.  Block: 512 threads;
// a 256-thread apply block runs as one half of a block, a 1024-thread decision
// block's sums are taken by 512 threads in the 1024-thread order.
struct StepArgs {
  GridPtrs P;
  int nl;
  int64_t n, d, lda, ldr, Kc, rps;
  int ncb, nsplit, nrp, iters;
  double mu_p, beta_p, mu_gd;
  DecideParams dp;
  const double* nu2;
  double* Gp;
};

// A slot's status read at device scope (past the caches of this CU and XCD), so
// every block of the grid sees the value the decision wrote before the barrier.
__device__ __forceinline__ int status_of(const GridPtrs& P, int z) {
  return __hip_atomic_load(&P.ctl[z].status, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ bool any_running(const GridPtrs& P, int nl) {
  for (int y = 0; y < nl; ++y)
    if (status_of(P, P.zl[y]) == RS_CTL_RUNNING) return true;
  return false;
}

// Grid barrier with device-scope fences on both sides: the phase's stores are
// visible to every block after it, and no block reads data cached before it.
__device__ __forceinline__ void grid_barrier(cooperative_groups::grid_group& g) {
  __threadfence();
  g.sync();
  __threadfence();
}

template <typename T, int TC, int K>
__global__ __launch_bounds__(512) void k_grid_steps(StepArgs a, const T* __restrict__ A,
                                                    const T* __restrict__ bvec,
                                                    T* __restrict__ XT, T* __restrict__ R) {
  namespace cg = cooperative_groups;
  cg::grid_group grid = cg::this_grid();
  constexpr size_t kTiles = (size_t)32 * 129 * sizeof(T) + (size_t)32 * (TC + 1) * sizeof(T);
  constexpr size_t kDecide = (size_t)1024 * K * sizeof(double) + 64;
  constexpr size_t kBytes = kTiles > kDecide ? kTiles : kDecide;
  __shared__ __align__(16) char smem[kBytes];
  __shared__ double rr[2][4][K];
  __shared__ double rsum[K];
  __shared__ int chosen;
  const GridPtrs& P = a.P;
  const int64_t d = a.d;
  const int tid = threadIdx.x;
  const int64_t gthreads = (int64_t)gridDim.x * 512;
  const int64_t g0 = (int64_t)blockIdx.x * 512 + tid;
  for (int it = 0; it < a.iters; ++it) {
    // candidates (k_cand_g) and their rounding to T (k_round_x)
    for (int64_t e = g0; e < (int64_t)a.nl * d; e += gthreads) {
      const int y = (int)(e / d);
      const int64_t i = e - (int64_t)y * d;
      const int z = P.zl[y];
      double* X = P.Xc + (int64_t)y * K * d;
      if (status_of(P, z) == RS_CTL_RUNNING) {
        const double xi = P.x[(int64_t)z * d + i];
        const double* xp = P.vec + (int64_t)z * 4 * d;
        const double gi = xp[2 * d + i];
        if (K == 2) {
          X[i] = xi - a.mu_p * gi + a.beta_p * (xi - xp[i]);
          X[d + i] = xi - a.mu_gd * gi;
        } else {
          X[i] = xi - a.mu_gd * gi;
        }
      }
#pragma unroll
      for (int k = 0; k < K; ++k) XT[((int64_t)y * K + k) * d + i] = (T)X[(int64_t)k * d + i];
    }
    grid_barrier(grid);
    // R = A X^T - b
    {
      T(*As)[129] = reinterpret_cast<T(*)[129]>(smem);
      T(*Xs)[TC + 1] = reinterpret_cast<T(*)[TC + 1]>(smem + (size_t)32 * 129 * sizeof(T));
      const int64_t nt = (a.n + 127) / 128 * a.ncb;
      for (int64_t v = blockIdx.x; v < nt; v += gridDim.x)
        mr_resid_tile<T, TC>(v, A, a.n, d, a.lda, bvec, XT, a.Kc, R, a.ldr, a.ncb, As, Xs);
    }
    grid_barrier(grid);
    // Gp = A^T R per row split
    {
      T(*As)[129] = reinterpret_cast<T(*)[129]>(smem);
      T(*Rs)[TC + 1] = reinterpret_cast<T(*)[TC + 1]>(smem + (size_t)32 * 129 * sizeof(T));
      const int64_t g2 = (d + 127) / 128 * a.ncb;
      const int64_t nt = g2 * a.nsplit;
      for (int64_t v = blockIdx.x; v < nt; v += gridDim.x)
        mr_atr_tile<T, TC>(v % g2, v / g2, A, a.n, d, a.lda, R, a.ldr, a.Kc, a.rps, a.ncb, a.Gp,
                           As, Rs);
    }
    grid_barrier(grid);
    // G = sum of the splits + nu^2 X (k_mr_reduce)
    for (int64_t e = g0; e < a.Kc * d; e += gthreads) {
      const int64_t c = e % a.Kc, j = e / a.Kc;
      double sacc = 0.0;
      for (int sp = 0; sp < a.nsplit; ++sp) sacc += a.Gp[((int64_t)sp * d + j) * a.ldr + c];
      const int z = P.zl[c / K];
      P.Gc[c * d + j] = sacc + a.nu2[z] * P.Xc[c * d + j];
    }
    grid_barrier(grid);
    // GT = H_z^-1 G and the decrement partials (k_symv_g): two 256-thread
    // blocks per block, virtual block v = (row block, list entry)
    {
      const int half = tid >> 8, lt = tid & 255, lane = lt & 63, w = lt >> 6;
      const int64_t nv = (int64_t)a.nrp * a.nl;
      for (int64_t v0 = 2 * (int64_t)blockIdx.x; v0 < nv; v0 += 2 * (int64_t)gridDim.x) {
        const int64_t v = v0 + half;
        const bool inb = v < nv;
        const int y = inb ? (int)(v / a.nrp) : 0;
        const int bx = inb ? (int)(v % a.nrp) : 0;
        const int z = P.zl[y];
        const bool act = inb && status_of(P, z) == RS_CTL_RUNNING;
        const double* H = P.Hinv + (int64_t)z * P.sH;
        const double* G = P.Gc + (int64_t)y * K * d;
        double* Y = P.GTc + (int64_t)y * K * d;
        const int64_t row = (int64_t)bx * 4 + w;
        double acc[K];
#pragma unroll
        for (int c = 0; c < K; ++c) acc[c] = 0.0;
        if (act) {
          for (int64_t j0 = 0; j0 < d; j0 += 128) {
            const int64_t j = j0 + 2 * lane;
            const bool ok0 = j < d, ok1 = j + 1 < d;
            const int64_t jc = ok0 ? j : 0;
            double gg0[K], gg1[K];
#pragma unroll
            for (int c = 0; c < K; ++c) {
              const double a0 = G[c * d + jc];
              const double a1 = G[c * d + (ok1 ? j + 1 : 0)];
              gg0[c] = ok0 ? a0 : 0.0;
              gg1[c] = ok1 ? a1 : 0.0;
            }
            const int64_t rr_ = row < d ? row : 0;
            const double2 h = *reinterpret_cast<const double2*>(H + rr_ * P.ldh + jc);
#pragma unroll
            for (int c = 0; c < K; ++c) acc[c] = fma(h.x, gg0[c], fma(h.y, gg1[c], acc[c]));
          }
        }
        double rloc[K];
#pragma unroll
        for (int c = 0; c < K; ++c) {
          rloc[c] = 0.0;
          const double yv = wave_sum(acc[c]);
          if (act && row < d) {
            if (lane == 0) Y[c * d + row] = yv;
            rloc[c] += yv * G[c * d + row];
          }
        }
        if (lane == 0)
#pragma unroll
          for (int c = 0; c < K; ++c) rr[half][w][c] = rloc[c];
        __syncthreads();
        if (act && lt < K) {
          double sum = 0.0;
          for (int ww = 0; ww < 4; ++ww) sum += rr[half][ww][lt];
          P.rpart[(int64_t)z * P.nrp * 2 + (int64_t)bx * K + lt] = sum;
        }
        __syncthreads();
      }
    }
    grid_barrier(grid);
    // the decision of every running list entry (k_decide_g)
    for (int y = blockIdx.x; y < a.nl; y += gridDim.x) {
      const int z = P.zl[y];
      DevCtl* ctl = P.ctl + z;
      if (status_of(P, z) != RS_CTL_RUNNING) continue;  // uniform over the block
      double* sh = reinterpret_cast<double*>(smem);
      const double* rp = P.rpart + (int64_t)z * P.nrp * 2;
      // block_sum_cols<K, 1024> with thread t standing for t and t + 512
      double v0[K], v1[K];
#pragma unroll
      for (int c = 0; c < K; ++c) v0[c] = v1[c] = 0.0;
      for (int bb = tid; bb < a.nrp; bb += 1024)
#pragma unroll
        for (int c = 0; c < K; ++c) v0[c] += rp[(int64_t)bb * K + c];
      for (int bb = tid + 512; bb < a.nrp; bb += 1024)
#pragma unroll
        for (int c = 0; c < K; ++c) v1[c] += rp[(int64_t)bb * K + c];
#pragma unroll
      for (int c = 0; c < K; ++c) {
        sh[c * 1024 + tid] = v0[c];
        sh[c * 1024 + tid + 512] = v1[c];
      }
      __syncthreads();
      for (int off = 512; off > 0; off >>= 1) {
        if (tid < off)
#pragma unroll
          for (int c = 0; c < K; ++c) sh[c * 1024 + tid] += sh[c * 1024 + tid + off];
        __syncthreads();
      }
      if (tid < K) rsum[tid] = sh[tid * 1024];
      __syncthreads();
      if (tid < K) rsum[tid] *= 0.5;
      __syncthreads();
      if (tid == 0) {
        int st = RS_CTL_RUNNING;
        const int64_t t = ctl->t;
        ctl->passes += 1;
        const int rule = step_rule(K == 2, rsum[0], rsum[K - 1], ctl->r_t, ctl->r_1, t,
                                   ctl->at_cap, a.dp.cbar_p, a.dp.cbar_gd, &st);
        const int c = rule == 0 ? 0 : (rule == 1 ? K - 1 : -1);
        if (c >= 0) {
          const int kind = (K == 2 && c == 0) ? 0 : 1;
          if (t < P.ev_cap) P.ev[(int64_t)z * P.ev_cap + t] = kind;
          if (kind == 0) ctl->polyak += 1; else ctl->gd += 1;
          ctl->r_t = rsum[c];
          ctl->t = t + 1;
          ctl->steps += 1;
          if (rsum[c] <= a.dp.tol * ctl->r_ref) st = RS_CTL_CONVERGED;
          else if (t + 1 >= a.dp.max_iter) st = RS_CTL_MAXITER;
        }
        ctl->last_r[0] = rsum[0];
        ctl->last_r[1] = rsum[K - 1];
        __hip_atomic_store(&ctl->status, st, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        chosen = c;
      }
      __syncthreads();
      const int c = chosen;
      if (c >= 0) {
        double* x = P.x + (int64_t)z * d;
        double* vv = P.vec + (int64_t)z * 4 * d;
        const double* X = P.Xc + (int64_t)y * K * d;
        const double* G = P.Gc + (int64_t)y * K * d;
        const double* GT = P.GTc + (int64_t)y * K * d;
        for (int64_t i = tid; i < d; i += 512) {
          vv[i] = x[i];
          x[i] = X[(int64_t)c * d + i];
          vv[d + i] = G[(int64_t)c * d + i];
          vv[2 * d + i] = GT[(int64_t)c * d + i];
        }
      }
      __syncthreads();
    }
    grid_barrier(grid);
    if (!any_running(P, a.nl)) break;  // the same answer in every block
  }
}

static unsigned vgrid(int64_t d) { return (unsigned)std::min<int64_t>((d + 255) / 256, 64); }

template <typename T, int TC, int K>
static rs_status steps_launch(const StepArgs& a, const T* A, const T* b, T* XT, T* R,
                              hipStream_t s) {
  const void* f = reinterpret_cast<const void*>(&k_grid_steps<T, TC, K>);
  int per_cu = 0;
  hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, f, 512, 0);
  if (e != hipSuccess) return set_error(RS_ERR_HIP, hipGetErrorString(e));
  if (per_cu < 1) return set_error(RS_ERR_UNSUPPORTED, "grid steps: kernel does not fit a CU");
  const unsigned grid = (unsigned)(per_cu * device_cus());
  StepArgs av = a;
  const T* Av = A;
  const T* bv = b;
  T* XTv = XT;
  T* Rv = R;
  void* args[] = {&av, &Av, &bv, &XTv, &Rv};
  e = hipLaunchCooperativeKernel(f, dim3(grid), dim3(512), args, 0, s);
  if (e != hipSuccess) return set_error(RS_ERR_HIP, hipGetErrorString(e));
  return check_launch("grid steps");
}

template <typename T>
rs_status grid_steps(const GridPtrs& P, int nl, int K, const T* A, int64_t n, int64_t d,
                     int64_t lda, const T* b, const double* nu2, T* R, int64_t ldr, double* Gp,
                     T* XT, double mu_p, double beta_p, double mu_gd, const DecideParams& dp,
                     int iters, hipStream_t s) {
  if (K != 1 && K != 2) return set_error(RS_ERR_ARG, "grid steps: K must be 1 or 2");
  StepArgs a{};
  a.P = P;
  a.nl = nl;
  a.n = n;
  a.d = d;
  a.lda = lda;
  a.ldr = ldr;
  a.Kc = (int64_t)nl * K;
  const int tc = mr_tc(a.Kc);
  a.ncb = (int)((a.Kc + tc - 1) / tc);
  a.nsplit = mr_splits(n, d, a.Kc, a.rps);
  a.nrp = P.nrp;
  a.iters = iters;
  a.mu_p = mu_p;
  a.beta_p = beta_p;
  a.mu_gd = mu_gd;
  a.dp = dp;
  a.nu2 = nu2;
  a.Gp = Gp;
#define RS_STEPS(TCV, KV) return steps_launch<T, TCV, KV>(a, A, b, XT, R, s)
  if (K == 2) {
    if (tc == 32) RS_STEPS(32, 2);
    if (tc == 64) RS_STEPS(64, 2);
    RS_STEPS(128, 2);
  }
  if (tc == 32) RS_STEPS(32, 1);
  if (tc == 64) RS_STEPS(64, 1);
  RS_STEPS(128, 1);
#undef RS_STEPS
}

template rs_status grid_steps<float>(const GridPtrs&, int, int, const float*, int64_t, int64_t,
                                     int64_t, const float*, const double*, float*, int64_t,
                                     double*, float*, double, double, double,
                                     const DecideParams&, int, hipStream_t);
template rs_status grid_steps<double>(const GridPtrs&, int, int, const double*, int64_t, int64_t,
                                      int64_t, const double*, const double*, double*, int64_t,
                                      double*, double*, double, double, double,
                                      const DecideParams&, int, hipStream_t);

rs_status grid_candidates(const GridPtrs& P, int nl, int K, int64_t d, double mu_p, double beta_p,
                          double mu_gd, hipStream_t s) {
  const dim3 g(vgrid(d), (unsigned)nl);
  if (K == 2) hipLaunchKernelGGL(k_cand_g<2>, g, dim3(256), 0, s, P, d, mu_p, beta_p, mu_gd);
  else hipLaunchKernelGGL(k_cand_g<1>, g, dim3(256), 0, s, P, d, mu_p, beta_p, mu_gd);
  return check_launch("grid candidates");
}

rs_status grid_pack(const GridPtrs& P, int nl, int64_t d, int what, hipStream_t s) {
  hipLaunchKernelGGL(k_pack_g, dim3(vgrid(d), (unsigned)nl), dim3(256), 0, s, P, d, what,
                     what == 0 ? 1 : 2);
  return check_launch("grid pack");
}

rs_status grid_apply(const GridPtrs& P, int nl, int K, int64_t d, const double* Gsrc, int always,
                     hipStream_t s) {
  const dim3 g((unsigned)apply_blocks(d), (unsigned)nl);
  if (K == 2) hipLaunchKernelGGL(k_symv_g<2>, g, dim3(256), 0, s, P, d, Gsrc, always);
  else hipLaunchKernelGGL(k_symv_g<1>, g, dim3(256), 0, s, P, d, Gsrc, always);
  return check_launch("grid apply");
}

rs_status grid_decide(const GridPtrs& P, int nl, int K, const DecideParams& a, int64_t d,
                      hipStream_t s) {
  const dim3 g(1, (unsigned)nl);
  if (K == 2) hipLaunchKernelGGL(k_decide_g<2>, g, dim3(1024), 0, s, P, a, d);
  else hipLaunchKernelGGL(k_decide_g<1>, g, dim3(1024), 0, s, P, a, d);
  return check_launch("grid decide");
}

rs_status grid_init(const GridPtrs& P, int nl, double tol, int64_t max_iter, int64_t d,
                    const int* at_cap, hipStream_t s) {
  hipLaunchKernelGGL(k_init_g, dim3(1, (unsigned)nl), dim3(1024), 0, s, P, tol, max_iter, d,
                     at_cap);
  return check_launch("grid init");
}

rs_status grid_post_resample(const GridPtrs& P, int nl, double tol, int64_t d, const int* at_cap,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_post_resample_g, dim3(1, (unsigned)nl), dim3(1024), 0, s, P, tol, d,
                     at_cap);
  return check_launch("grid post resample");
}

}  // namespace rs
