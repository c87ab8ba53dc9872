// Learned starting sketch size: features of a problem, and a small MLP trained
// on the GPU by these kernels (forward, backward, Adam).
//
// Algorithm 1's guarantees hold for any initial sketch size (Theorems 5 and 6);
// the predictor only decides where the doubling ladder starts.
//
// Features (16): log2 n, log2 d, log10 nu^2; ln of 8 Hutchinson probes
// q_k = (A^T w_k)^T H_S0^-1 (A^T w_k) (w_k Rademacher from Philox stream 7, H_S0
// from a 256-row SRHT); quantiles 0, 1/4, 1/2, 3/4, 1 of ln ||A e_j||.
// MLP: 16 -> 128 -> 128 -> 1, exact GELU, inputs standardised (f - mu) / sd.
#include "rs_internal.hpp"

namespace rs {

constexpr int kFeat = 16;
constexpr int kHid = 128;
constexpr int kProbes = 8;
constexpr int OFF_W1 = 0;
constexpr int OFF_B1 = OFF_W1 + kFeat * kHid;
constexpr int OFF_W2 = OFF_B1 + kHid;
constexpr int OFF_B2 = OFF_W2 + kHid * kHid;
constexpr int OFF_W3 = OFF_B2 + kHid;
constexpr int OFF_B3 = OFF_W3 + kHid;
constexpr int kParams = OFF_B3 + 1;
constexpr int kCache = kFeat + 2 * kHid + 1;   // xn, z1, z2, y per sample
constexpr int kWork = 2 * kHid + 1;            // dz1, dz2, dy per sample

// ------------------------------------------------------------------ features
// Column sums over a chunk of rows: part[chunk][k][j] = sum_i w_k(i) A[i][j] for
// the 8 probes, part[chunk][8][j] = sum_i A[i][j]^2 and, when b is given,
// part[chunk][9][j] = sum_i b_i A[i][j] (A^T b, the gradient at the origin up to
// its sign, so a solve started at 0 needs no gradient pass of its own), FP64.  Block: 64 lanes x
// VEC columns (one 16-byte vector per lane and row), 4 waves taking every 4th
// row of the chunk, 4 rows per wave in flight; the probe signs of the chunk's
// rows are drawn once into LDS.  The waves' sums meet in LDS in a fixed order.
constexpr int kProbeChunkMax = 4096;
constexpr int kPCols = kProbes + 2;  // the probes, the squared norms, A^T b
static_assert(kPCols == kProbeCols, "one layout for both forms of the probe sums");

template <typename T>
__global__ __launch_bounds__(256) void k_probe_partial(const T* __restrict__ A, int64_t n,
                                                       int64_t d, int64_t lda,
                                                       const T* __restrict__ b, uint64_t seed,
                                                       int64_t rows_per_chunk,
                                                       double* __restrict__ part) {
  using V = typename VecOf<T>::type;
  constexpr int VEC = VecOf<T>::n;
  constexpr int COLS = 64 * VEC;
  constexpr int U = 4;
  __shared__ uint8_t sgn[kProbeChunkMax];
  __shared__ double red[kPCols][COLS];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  const int64_t c0 = (int64_t)blockIdx.x * COLS + lane * VEC;
  const int64_t r0 = (int64_t)blockIdx.y * rows_per_chunk;
  const int64_t r1 = r0 + rows_per_chunk < n ? r0 + rows_per_chunk : n;
  const int cnt = (int)(r1 - r0);
  for (int i = t; i < cnt; i += 256) {
    uint8_t bits = 0;
#pragma unroll
    for (int k = 0; k < kProbes; ++k) {
      const uint4 wd = draw(seed, kStreamProbe, (uint32_t)k, (uint64_t)(r0 + i));
      bits |= (uint8_t)((wd.x & 1u) << k);
    }
    sgn[i] = bits;
  }
  __syncthreads();
  bool cok[VEC];
#pragma unroll
  for (int e = 0; e < VEC; ++e) cok[e] = c0 + e < d;
  const int64_t cc = c0 < d ? c0 : 0;
  double acc[kPCols][VEC];
#pragma unroll
  for (int k = 0; k < kPCols; ++k)
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[k][e] = 0.0;
  for (int i0 = w; i0 < cnt; i0 += 4 * U) {
    V a[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + 4 * u;
      const int ic = i < cnt ? i : 0;
      a[u] = *reinterpret_cast<const V*>(A + (r0 + ic) * lda + cc);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = i0 + 4 * u;
      const bool rok = i < cnt;
      const uint8_t bits = sgn[rok ? i : 0];
      const double bi = b ? (double)b[r0 + (rok ? i : 0)] : 0.0;
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const double x = (rok && cok[e]) ? (double)get(a[u], e) : 0.0;
#pragma unroll
        for (int k = 0; k < kProbes; ++k) acc[k][e] += ((bits >> k) & 1) ? -x : x;
        acc[kProbes][e] = fma(x, x, acc[kProbes][e]);
        acc[kProbes + 1][e] = fma(bi, x, acc[kProbes + 1][e]);
      }
    }
  }
  // waves 0..3 in order
  for (int ww = 0; ww < 4; ++ww) {
    if (w == ww) {
#pragma unroll
      for (int k = 0; k < kPCols; ++k)
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const int col = lane * VEC + e;
          red[k][col] = (ww == 0 ? 0.0 : red[k][col]) + acc[k][e];
        }
    }
    __syncthreads();
  }
  for (int e = t; e < kPCols * COLS; e += 256) {
    const int k = e / COLS, col = e % COLS;
    const int64_t j = (int64_t)blockIdx.x * COLS + col;
    if (j < d) part[((int64_t)blockIdx.y * kPCols + k) * d + j] = red[k][col];
  }
}

// U[k][j] = sum over chunks (fixed order), k = 0..9.  Block: 8 consecutive
// elements x 32 chunk strides, then a tree over the strides in LDS.
__global__ __launch_bounds__(256) void k_probe_finish(const double* __restrict__ part, int nchunk,
                                                      int64_t d, double* __restrict__ U) {
  __shared__ double sh[32][8];
  const int cl = threadIdx.x & 7, st = threadIdx.x >> 3;
  const int64_t tot = (int64_t)kPCols * d;
  const int64_t e = (int64_t)blockIdx.x * 8 + cl;
  double v = 0.0;
  if (e < tot)
    for (int c = st; c < nchunk; c += 32) v += part[(int64_t)c * tot + e];
  sh[st][cl] = v;
  __syncthreads();
  for (int off = 16; off > 0; off >>= 1) {
    if (st < off) sh[st][cl] += sh[st + off][cl];
    __syncthreads();
  }
  if (st == 0 && e < tot) U[e] = sh[0][cl];
}

// Probe quadratic forms through the m0 x m0 factor when m0 < d (Woodbury): with
// W = nu^2 I + SA SA^T = L L^T, u^T H^-1 u = (|u|^2 - |L^-1 SA u|^2) / nu^2.
// k_probe_sav: v[k][i] = SA_i . u_k, one wave per row i, lanes along d.
template <typename TS>
__global__ __launch_bounds__(256) void k_probe_sav(const TS* __restrict__ SA, int64_t m,
                                                   int64_t d, int64_t ldsa,
                                                   const double* __restrict__ U,
                                                   double* __restrict__ V) {
  const int k = blockIdx.x;
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.y * 4 + (threadIdx.x >> 6);
  if (i >= m) return;
  const double* u = U + (int64_t)k * d;
  const TS* row = SA + i * ldsa;
  double acc = 0.0;
  for (int64_t j = lane; j < d; j += 64) acc = fma((double)row[j], u[j], acc);
  acc = wave_sum(acc);
  if (lane == 0) V[(int64_t)k * m + i] = acc;
}

// One block per probe: y = L^-1 v (thread i takes row i of the triangle), then
// r_k = (|u_k|^2 - |y|^2) / (2 nu^2) (the decrement convention r = q / 2).
__global__ __launch_bounds__(256) void k_probe_quad(const double* __restrict__ V, int64_t m,
                                                    const double* __restrict__ Linv, int64_t ldl,
                                                    const double* __restrict__ U, int64_t d,
                                                    double nu2, double* __restrict__ r) {
  __shared__ double sh[2 * 256];
  const int k = blockIdx.x, t = threadIdx.x;
  const double* v = V + (int64_t)k * m;
  double yy = 0.0;
  for (int64_t i = t; i < m; i += 256) {
    double y = 0.0;
    for (int64_t l = 0; l <= i; ++l) y = fma(Linv[i * ldl + l], v[l], y);
    yy = fma(y, y, yy);
  }
  double uu = 0.0;
  const double* u = U + (int64_t)k * d;
  for (int64_t j = t; j < d; j += 256) uu = fma(u[j], u[j], uu);
  sh[t] = yy;
  sh[256 + t] = uu;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if (t < off) {
      sh[t] += sh[t + off];
      sh[256 + t] += sh[256 + t + off];
    }
    __syncthreads();
  }
  if (t == 0) r[k] = 0.5 * (sh[256] - sh[0]) / nu2;
}

rs_status probe_quads(const void* SA, rs_dtype sa_t, int64_t m, int64_t d, int64_t ldsa,
                      const double* Linv, int64_t ldl, const double* U, double nu2, double* V,
                      double* r, hipStream_t s) {
  const dim3 g1(kProbes, (unsigned)((m + 3) / 4));
  if (sa_t == RS_F64)
    hipLaunchKernelGGL(k_probe_sav<double>, g1, dim3(256), 0, s,
                       reinterpret_cast<const double*>(SA), m, d, ldsa, U, V);
  else
    hipLaunchKernelGGL(k_probe_sav<float>, g1, dim3(256), 0, s,
                       reinterpret_cast<const float*>(SA), m, d, ldsa, U, V);
  hipLaunchKernelGGL(k_probe_quad, dim3(kProbes), dim3(256), 0, s, V, m, Linv, ldl, U, d, nu2, r);
  return check_launch("probe quadratic forms");
}

// One block: q_k = 2 r_k (r from the apply of the probes), log column norms,
// sort, quantiles, and the 16 features.
__global__ __launch_bounds__(1024) void k_feature_final(const double* __restrict__ U, int64_t d,
                                                        const double* __restrict__ rprobe,
                                                        int64_t n, double nu2,
                                                        float* __restrict__ feat) {
  __shared__ float v[8192];
  int P = 1;
  while (P < d) P <<= 1;
  for (int i = threadIdx.x; i < P; i += 1024) {
    float x = 3.0e38f;
    if (i < d) {
      const double c2 = U[(int64_t)kProbes * d + i];
      x = (float)(0.5 * log(c2 > 1e-300 ? c2 : 1e-300));
    }
    v[i] = x;
  }
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += 1024) {
        const int l = i ^ j;
        if (l > i) {
          const bool up = (i & k) == 0;
          if ((v[i] > v[l]) == up) {
            const float t = v[i];
            v[i] = v[l];
            v[l] = t;
          }
        }
      }
      __syncthreads();
    }
  }
  if (threadIdx.x == 0) {
    feat[0] = (float)log2((double)n);
    feat[1] = (float)log2((double)d);
    feat[2] = (float)log10(nu2);
    for (int k = 0; k < kProbes; ++k) {
      const double q = 2.0 * rprobe[k];
      feat[3 + k] = (float)log(q > 1e-30 ? q : 1e-30);
    }
    const double qs[5] = {0.0, 0.25, 0.5, 0.75, 1.0};
    for (int i = 0; i < 5; ++i) {
      const int idx = (int)rint(qs[i] * (double)(d - 1));
      feat[11 + i] = v[idx];
    }
  }
}

// Row chunks of the probe pass: enough blocks to fill the chip, at most
// kProbeChunkMax rows each.
static int64_t probe_rows_per_chunk(int64_t n, int64_t d, int vec) {
  const int64_t colblocks = (d + 64 * vec - 1) / (64 * vec);
  int64_t want = (4 * device_cus() + colblocks - 1) / colblocks;
  want = std::max<int64_t>(1, std::min<int64_t>(want, (n + 255) / 256));
  int64_t rpc = ((n + want - 1) / want + 63) / 64 * 64;
  if (rpc > kProbeChunkMax) rpc = kProbeChunkMax;
  return rpc;
}

int feature_chunks(int64_t n, int64_t d, int vec) {
  const int64_t rpc = probe_rows_per_chunk(n, d, vec);
  return (int)((n + rpc - 1) / rpc);
}

template <typename T>
rs_status features_pass(const T* A, int64_t n, int64_t d, int64_t lda, const T* b,
                        uint64_t seed, double* part, double* U, hipStream_t s) {
  constexpr int VEC = VecOf<T>::n;
  const int64_t rpc = probe_rows_per_chunk(n, d, VEC);
  const int nch = (int)((n + rpc - 1) / rpc);
  const unsigned colblocks = (unsigned)((d + 64 * VEC - 1) / (64 * VEC));
  hipLaunchKernelGGL(k_probe_partial<T>, dim3(colblocks, (unsigned)nch), dim3(256), 0, s, A, n, d,
                     lda, b, seed, rpc, part);
  const int64_t tot = (int64_t)kPCols * d;
  hipLaunchKernelGGL(k_probe_finish, dim3((unsigned)((tot + 7) / 8)), dim3(256), 0, s, part, nch,
                     d, U);
  return check_launch("features pass");
}
// The probe signs of every row as one byte (bit k: w_k(i) = -1), for the first pass
// of the probe sketch that takes the probe sums along (ProbeArgs).
__global__ __launch_bounds__(256) void k_probe_bits(uint64_t seed, int64_t n,
                                                    uint8_t* __restrict__ bits) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    uint8_t v = 0;
#pragma unroll
    for (int k = 0; k < kProbes; ++k) {
      const uint4 wd = draw(seed, kStreamProbe, (uint32_t)k, (uint64_t)i);
      v |= (uint8_t)((wd.x & 1u) << k);
    }
    bits[i] = v;
  }
}

rs_status probe_bits(uint64_t seed, int64_t n, uint8_t* bits, hipStream_t s) {
  const unsigned g = (unsigned)std::min<int64_t>((n + 255) / 256, 8192);
  hipLaunchKernelGGL(k_probe_bits, dim3(g), dim3(256), 0, s, seed, n, bits);
  return check_launch("probe bits");
}

// U[k][j] = sum over the tiles (in order) of the first pass's per-tile sums.
__global__ __launch_bounds__(256) void k_probe_tiles_finish(const double* __restrict__ part,
                                                            int64_t ntiles, int64_t d, int64_t dp,
                                                            double* __restrict__ U) {
  const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (e >= (int64_t)kProbeCols * d) return;
  const int64_t k = e / d, j = e - k * d;
  double v = 0.0;
  for (int64_t t = 0; t < ntiles; ++t) v += part[(t * kProbeCols + k) * dp + j];
  U[e] = v;
}

rs_status probe_tiles_finish(const double* part, int64_t ntiles, int64_t d, int64_t dp, double* U,
                             hipStream_t s) {
  const unsigned g = (unsigned)(((int64_t)kProbeCols * d + 255) / 256);
  hipLaunchKernelGGL(k_probe_tiles_finish, dim3(g), dim3(256), 0, s, part, ntiles, d, dp, U);
  return check_launch("probe sums");
}

// The gradient at a start x = 0 from the features pass: grad f(0) = -A^T b (eq. (1)
// with x = 0).  One block: if any x_j != 0 the flag stays 0 (the solve's own
// gradient pass runs); otherwise G = -A^T b and the flag tells that pass to skip.
__global__ __launch_bounds__(256) void k_start_from_atb(const double* __restrict__ x,
                                                        const double* __restrict__ atb,
                                                        int64_t d, double* __restrict__ G,
                                                        int* __restrict__ skip) {
  int nz = 0;
  for (int64_t j = threadIdx.x; j < d; j += 256) nz |= x[j] != 0.0;
  const int any = __syncthreads_or(nz);
  if (any) {
    if (threadIdx.x == 0) *skip = 0;
    return;
  }
  for (int64_t j = threadIdx.x; j < d; j += 256) G[j] = -atb[j];
  if (threadIdx.x == 0) *skip = 1;
}

rs_status start_from_atb(const double* x, const double* atb, int64_t d, double* G, int* skip,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_start_from_atb, dim3(1), dim3(256), 0, s, x, atb, d, G, skip);
  return check_launch("start from A^T b");
}

template rs_status features_pass<float>(const float*, int64_t, int64_t, int64_t, const float*,
                                        uint64_t, double*, double*, hipStream_t);
template rs_status features_pass<double>(const double*, int64_t, int64_t, int64_t, const double*,
                                         uint64_t, double*, double*, hipStream_t);

rs_status features_final(const double* U, int64_t d, const double* rprobe, int64_t n, double nu2,
                         float* feat, hipStream_t s) {
  if (d > 8192) return set_error(RS_ERR_UNSUPPORTED, "features: d above 8192");
  hipLaunchKernelGGL(k_feature_final, dim3(1), dim3(1024), 0, s, U, d, rprobe, n, nu2, feat);
  return check_launch("features final");
}

// ------------------------------------------------------------------ MLP
__device__ __forceinline__ float gelu_f(float z) {
  return 0.5f * z * (1.0f + erff(z * 0.70710678118654752f));
}
__device__ __forceinline__ float gelu_grad_f(float z) {
  return 0.5f * (1.0f + erff(z * 0.70710678118654752f)) +
         z * expf(-0.5f * z * z) * 0.39894228040143268f;
}

// One block (128 threads) per sample; cache row: xn (16), z1, z2 (128 each), y.
__global__ __launch_bounds__(128) void k_mlp_forward(const float* __restrict__ P,
                                                     const float* __restrict__ X, int64_t B,
                                                     const float* __restrict__ mu,
                                                     const float* __restrict__ sd,
                                                     float* __restrict__ Y,
                                                     float* __restrict__ cache) {
  __shared__ float xn[kFeat];
  __shared__ float h1[kHid];
  __shared__ float part[kHid];
  const int64_t s = blockIdx.x;
  const int u = threadIdx.x;
  if (u < kFeat) xn[u] = (X[s * kFeat + u] - mu[u]) / sd[u];
  __syncthreads();
  float z1 = P[OFF_B1 + u];
#pragma unroll
  for (int k = 0; k < kFeat; ++k) z1 = fmaf(xn[k], P[OFF_W1 + k * kHid + u], z1);
  h1[u] = gelu_f(z1);
  __syncthreads();
  float z2 = P[OFF_B2 + u];
  for (int v = 0; v < kHid; ++v) z2 = fmaf(h1[v], P[OFF_W2 + v * kHid + u], z2);
  part[u] = gelu_f(z2) * P[OFF_W3 + u];
  __syncthreads();
  for (int off = kHid / 2; off > 0; off >>= 1) {
    if (u < off) part[u] += part[u + off];
    __syncthreads();
  }
  const float y = part[0] + P[OFF_B3];
  if (u == 0) Y[s] = y;
  if (cache) {
    float* c = cache + s * kCache;
    if (u < kFeat) c[u] = xn[u];
    c[kFeat + u] = z1;
    c[kFeat + kHid + u] = z2;
    if (u == 0) c[kFeat + 2 * kHid] = y;
  }
}

// Per-sample deltas of the loss mean((y - t)^2): dy, dz2, dz1 into work.
__global__ __launch_bounds__(128) void k_mlp_delta(const float* __restrict__ P,
                                                   const float* __restrict__ cache,
                                                   const float* __restrict__ T, int64_t B,
                                                   float* __restrict__ work) {
  __shared__ float dz2[kHid];
  const int64_t s = blockIdx.x;
  const int u = threadIdx.x;
  const float* c = cache + s * kCache;
  const float dy = 2.0f * (c[kFeat + 2 * kHid] - T[s]) / (float)B;
  const float g2 = dy * P[OFF_W3 + u] * gelu_grad_f(c[kFeat + kHid + u]);
  dz2[u] = g2;
  __syncthreads();
  float dh1 = 0.0f;
  for (int w = 0; w < kHid; ++w) dh1 = fmaf(dz2[w], P[OFF_W2 + u * kHid + w], dh1);
  float* wk = work + s * kWork;
  wk[u] = dh1 * gelu_grad_f(c[kFeat + u]);
  wk[kHid + u] = g2;
  if (u == 0) wk[2 * kHid] = dy;
}

// Gradient of every parameter: a fixed-order sum over the batch.  Also the
// loss (by the thread of b3).
__global__ __launch_bounds__(256) void k_mlp_grad(const float* __restrict__ cache,
                                                  const float* __restrict__ work, int64_t B,
                                                  float* __restrict__ G, float* __restrict__ loss) {
  const int p = blockIdx.x * 256 + threadIdx.x;
  if (p >= kParams) return;
  float acc = 0.0f;
  float lacc = 0.0f;
  for (int64_t s = 0; s < B; ++s) {
    const float* c = cache + s * kCache;
    const float* w = work + s * kWork;
    float v;
    if (p < OFF_B1) {
      const int k = p / kHid, u = p % kHid;
      v = c[k] * w[u];
    } else if (p < OFF_W2) {
      v = w[p - OFF_B1];
    } else if (p < OFF_B2) {
      const int q = p - OFF_W2;
      const int vv = q / kHid, u = q % kHid;
      v = gelu_f(c[kFeat + vv]) * w[kHid + u];
    } else if (p < OFF_W3) {
      v = w[kHid + (p - OFF_B2)];
    } else if (p < OFF_B3) {
      const int u = p - OFF_W3;
      v = gelu_f(c[kFeat + kHid + u]) * w[2 * kHid];
    } else {
      v = w[2 * kHid];
      const float r = w[2 * kHid] * (float)B * 0.5f;
      lacc = fmaf(r, r, lacc);
    }
    acc += v;
  }
  G[p] = acc;
  if (p == OFF_B3 && loss) *loss = lacc / (float)B;
}

__global__ __launch_bounds__(256) void k_adam(float* __restrict__ Pm, const float* __restrict__ G,
                                              float* __restrict__ M, float* __restrict__ V,
                                              int64_t count, float lr, float b1, float b2,
                                              float eps, float c1, float c2) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i >= count) return;
  const float g = G[i];
  const float m = b1 * M[i] + (1.0f - b1) * g;
  const float v = b2 * V[i] + (1.0f - b2) * g * g;
  M[i] = m;
  V[i] = v;
  Pm[i] -= lr * (m / c1) / (sqrtf(v / c2) + eps);
}

rs_status mlp_forward(const float* P, const float* X, int64_t B, const float* mu, const float* sd,
                      float* Y, float* cache, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)B), dim3(kHid), 0, s, P, X, B, mu, sd, Y, cache);
  return check_launch("mlp forward");
}

rs_status mlp_backward(const float* P, const float* cache, const float* T, int64_t B, float* G,
                       float* loss, float* work, hipStream_t s) {
  hipLaunchKernelGGL(k_mlp_delta, dim3((unsigned)B), dim3(kHid), 0, s, P, cache, T, B, work);
  hipLaunchKernelGGL(k_mlp_grad, dim3((kParams + 255) / 256), dim3(256), 0, s, cache, work, B, G,
                     loss);
  return check_launch("mlp backward");
}

rs_status mlp_adam(float* P, const float* G, float* M, float* V, int64_t count, int64_t step,
                   float lr, float b1, float b2, float eps, hipStream_t s) {
  const float c1 = 1.0f - powf(b1, (float)step);
  const float c2 = 1.0f - powf(b2, (float)step);
  hipLaunchKernelGGL(k_adam, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, P, G, M, V,
                     count, lr, b1, b2, eps, c1, c2);
  return check_launch("adam");
}

int mlp_params() { return kParams; }
int mlp_cache_floats() { return kCache; }
int mlp_work_floats() { return kWork; }

}  // namespace rs
