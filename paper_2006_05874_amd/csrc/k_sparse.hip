// Sparse A (CSR) with the CountSketch, the O(nnz) embedding named for sparse data
// matrices: S has one signed nonzero per column, S[h_i, i] = s_i.  Every sum has a
// fixed order (no floating-point atomics): rows are grouped by bucket with a
// stable radix sort (written here: digit counts, a scan, an order-keeping
// scatter), the gradient's A^T r pass runs over a column-major (CSC) copy formed
// once per solve by the same sort.
#include "rs_internal.hpp"

namespace rs {

#define SP_HIP(call)                                                                \
  do {                                                                              \
    const hipError_t e_ = (call);                                                   \
    if (e_ != hipSuccess)                                                           \
      return set_error(e_ == hipErrorOutOfMemory ? RS_ERR_OOM : RS_ERR_HIP,         \
                       hipGetErrorString(e_));                                      \
  } while (0)
#define SP_TRY(expr)                   \
  do {                                 \
    const rs_status st_ = (expr);      \
    if (st_ != RS_OK) return st_;      \
  } while (0)

static size_t value_size(rs_dtype t) { return t == RS_F64 ? 8 : 4; }

rs_status GrowBuf::ensure(size_t want) {
  if (want <= bytes && p) return RS_OK;
  if (p) {
    // work already queued may still read the old block
    SP_HIP(hipDeviceSynchronize());
    (void)hipFree(p);
  }
  p = nullptr;
  bytes = 0;
  const size_t sz = want ? want : 256;
  const hipError_t e = hipMalloc(&p, sz);
  if (e != hipSuccess) {
    p = nullptr;
    return set_error(e == hipErrorOutOfMemory ? RS_ERR_OOM : RS_ERR_HIP, hipGetErrorString(e));
  }
  bytes = sz;
  return RS_OK;
}

// bad = 1 unless rowptr[0] = 0, rowptr[n] = nnz, rowptr never decreases and every
// column index is in [0, d)
__global__ __launch_bounds__(256) void k_csr_check(const int64_t* __restrict__ rowptr, int64_t n,
                                                   const int32_t* __restrict__ col, int64_t nnz,
                                                   int64_t d, int* __restrict__ bad) {
  const int64_t stride = (int64_t)gridDim.x * 256;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  bool ok = true;
  if (t == 0) ok = rowptr[0] == 0 && rowptr[n] == nnz;
  for (int64_t i = t; i < n; i += stride) ok = ok && rowptr[i] <= rowptr[i + 1];
  for (int64_t q = t; q < nnz; q += stride) ok = ok && col[q] >= 0 && col[q] < d;
  if (!ok) *bad = 1;
}

// bucket h_i = high word of (word0 * m), sign from word1 (Philox stream 8)
__global__ __launch_bounds__(256) void k_cs_hash(int64_t n, uint64_t seed, uint32_t sid,
                                                 uint32_t m, uint32_t* __restrict__ bucket,
                                                 int32_t* __restrict__ row,
                                                 float* __restrict__ sign) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * 256) {
    const uint4 w = draw(seed, kStreamCount, sid, (uint64_t)i);
    bucket[i] = (uint32_t)(((uint64_t)w.x * (uint64_t)m) >> 32);
    row[i] = (int32_t)i;
    sign[i] = (w.y & 1u) ? -1.0f : 1.0f;
  }
}

// off[k] = first position p of the sorted keys with key[p] >= k, k = 0..nk
__global__ __launch_bounds__(256) void k_segment_offsets(const uint32_t* __restrict__ key,
                                                         int64_t n, uint32_t nk,
                                                         int64_t* __restrict__ off) {
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p <= n;
       p += (int64_t)gridDim.x * 256) {
    const uint32_t lo = p == 0 ? 0u : key[p - 1] + 1u;
    const uint32_t hi = p == n ? nk : key[p];
    for (uint32_t k = lo; k <= hi && k <= nk; ++k) off[k] = p;
  }
}

// Rows are grouped by bucket (ascending within a bucket, from the stable sort) and
// each bucket's rows are cut into chunks of kCsChunk rows: chunk c of the chunk
// list (cst[h] = first chunk of bucket h) is one block.  The block's W groups of
// 16 lanes take the chunk's rows in turn, each group adding its rows in order into
// its own FP64 LDS row (a row's columns are distinct, so the lanes never collide);
// the W rows are then summed in group order into the chunk's partial row.
constexpr int kCsChunk = 256;

__device__ __forceinline__ int64_t upper_index(const int64_t* __restrict__ v, int64_t len,
                                               int64_t x) {  // last k with v[k] <= x
  int64_t lo = 0, hi = len - 1;
  while (lo < hi) {
    const int64_t mid = (lo + hi + 1) >> 1;
    if (v[mid] <= x) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__global__ __launch_bounds__(256) void k_chunk_counts(const int64_t* __restrict__ off, int64_t nseg,
                                                      int64_t per, int64_t* __restrict__ nch) {
  for (int64_t h = (int64_t)blockIdx.x * 256 + threadIdx.x; h <= nseg;
       h += (int64_t)gridDim.x * 256)
    nch[h] = h == nseg ? 0 : (off[h + 1] - off[h] + per - 1) / per;
}

template <typename T>
__global__ __launch_bounds__(256) void k_cs_partial(const int64_t* __restrict__ rowptr,
                                                    const int32_t* __restrict__ col,
                                                    const T* __restrict__ val,
                                                    const int32_t* __restrict__ srow,
                                                    const float* __restrict__ sign,
                                                    const int64_t* __restrict__ off,
                                                    const int64_t* __restrict__ cst, int64_t m,
                                                    int64_t d, int W, double* __restrict__ part) {
  extern __shared__ double acc[];
  const int64_t c = blockIdx.x;
  if (c >= cst[m]) return;
  const int64_t h = upper_index(cst, m + 1, c);
  const int64_t p0 = off[h] + (c - cst[h]) * kCsChunk;
  const int64_t p1 = min(off[h + 1], p0 + (int64_t)kCsChunk);
  const int w = threadIdx.x >> 4, lane = threadIdx.x & 15;
  for (int64_t j = threadIdx.x; j < (int64_t)W * d; j += blockDim.x) acc[j] = 0.0;
  __syncthreads();
  double* a = acc + (int64_t)w * d;
  // the group's rows p0 + w, p0 + w + W, ...: each lane fetches one row's id, sign
  // and bounds (16 rows at a time), then the rows' first 16 entries are loaded four
  // rows at a time before they are added, row after row (a row's remaining entries
  // right after its first 16), so the sums keep a fixed order
  for (int64_t pb = p0 + w; pb < p1; pb += (int64_t)W * 16) {
    const int64_t pl = pb + (int64_t)lane * W;
    long long rb = 0, re = 0;
    double sg = 0.0;
    if (pl < p1) {
      const int32_t i = srow[pl];
      sg = (double)sign[i];
      rb = rowptr[i];
      re = rowptr[i + 1];
    }
    const int nrow = (int)min<int64_t>(16, (p1 - pb + W - 1) / W);
    for (int r0 = 0; r0 < nrow; r0 += 4) {
      int32_t cc[4];
      double vv[4], su[4];
      long long qb[4], qe[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        qb[u] = __shfl(rb, r0 + u, 16);
        qe[u] = __shfl(re, r0 + u, 16);
        su[u] = __shfl(sg, r0 + u, 16);
        const long long q = qb[u] + lane;
        const bool on = r0 + u < nrow && q < qe[u];
        cc[u] = on ? col[q] : -1;
        vv[u] = on ? su[u] * (double)val[q] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        if (r0 + u >= nrow) break;
        if (cc[u] >= 0) a[cc[u]] += vv[u];
        for (long long q = qb[u] + 16 + lane; q < qe[u]; q += 16) a[col[q]] += su[u] * (double)val[q];
      }
    }
  }
  __syncthreads();
  for (int64_t j = threadIdx.x; j < d; j += blockDim.x) {
    double v = acc[j];
    for (int u = 1; u < W; ++u) v += acc[(int64_t)u * d + j];
    part[c * d + j] = v;
  }
}

// SA row h = the sum of the bucket's chunk partials (0 for an empty bucket).  A block
// covers 16 columns with 16 chunk lanes: lane z adds chunks z, z + 16, ... in order
// and the 16 sums are added in lane order, so a bucket with many chunks (small m)
// still spreads over 256 threads.
template <typename TO>
__global__ __launch_bounds__(256) void k_cs_sum(const double* __restrict__ part,
                                                const int64_t* __restrict__ cst, int64_t d,
                                                TO* __restrict__ SA, int64_t ldsa) {
  __shared__ double sh[16][17];
  const int64_t h = blockIdx.x;
  const int cl = threadIdx.x & 15, z = threadIdx.x >> 4;
  const int64_t j = (int64_t)blockIdx.y * 16 + cl;
  double v = 0.0;
  if (j < d)
    for (int64_t c = cst[h] + z; c < cst[h + 1]; c += 16) v += part[c * d + j];
  sh[z][cl] = v;
  __syncthreads();
  if (z == 0 && j < ldsa) {
    double t = sh[0][cl];
    for (int u = 1; u < 16; ++u) t += sh[u][cl];
    if constexpr (std::is_same<TO, uint16_t>::value)
      SA[h * ldsa + j] = f32_to_bf16_rne((float)t);
    else
      SA[h * ldsa + j] = (TO)t;
  }
}

// row id of every stored entry, and the entries' positions
__global__ __launch_bounds__(256) void k_expand_rows(const int64_t* __restrict__ rowptr, int64_t n,
                                                     int32_t* __restrict__ rid) {
  for (int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); i < n;
       i += (int64_t)gridDim.x * 4)
    for (int64_t q = rowptr[i] + (threadIdx.x & 63); q < rowptr[i + 1]; q += 64)
      rid[q] = (int32_t)i;
}

__global__ __launch_bounds__(256) void k_iota(int64_t n, int64_t* __restrict__ v) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256)
    v[i] = i;
}

template <typename T>
__global__ __launch_bounds__(256) void k_gather_csc(int64_t nnz, const int64_t* __restrict__ pos,
                                                    const int32_t* __restrict__ rid,
                                                    const T* __restrict__ val,
                                                    int32_t* __restrict__ crow,
                                                    T* __restrict__ cval) {
  for (int64_t p = (int64_t)blockIdx.x * 256 + threadIdx.x; p < nnz;
       p += (int64_t)gridDim.x * 256) {
    const int64_t q = pos[p];
    crow[p] = rid[q];
    cval[p] = val[q];
  }
}

// R[i][k] = sum over row i of a_ij X[k][j] - b_i (FP64, interleaved so that the
// column pass gathers a row's K residuals from one cache line), K <= 4: 16 lanes
// per row stride its entries, then a fixed butterfly over the 16 lanes.  A group
// takes two rows at a time (i and i + 16) with their loads issued together.
template <typename T>
__global__ __launch_bounds__(256) void k_csr_resid(const int64_t* __restrict__ rowptr,
                                                   const int32_t* __restrict__ col,
                                                   const T* __restrict__ val,
                                                   const T* __restrict__ b, int64_t n, int64_t d,
                                                   const double* __restrict__ X, int K,
                                                   double* __restrict__ R,
                                                   const int* __restrict__ status,
                                                   int* __restrict__ ran) {
  if (status && *status != 0) return;
  if (ran && blockIdx.x == 0 && threadIdx.x == 0) *ran = 1;
  const int l = threadIdx.x & 15;
  for (int64_t i0 = (int64_t)blockIdx.x * 32; i0 < n; i0 += (int64_t)gridDim.x * 32) {
    int64_t ii[2], qb[2], qe[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      ii[u] = i0 + 16 * u + (threadIdx.x >> 4);
      qb[u] = ii[u] < n ? rowptr[ii[u]] : 0;
      qe[u] = ii[u] < n ? rowptr[ii[u] + 1] : 0;
    }
    double s[2][4] = {{0.0, 0.0, 0.0, 0.0}, {0.0, 0.0, 0.0, 0.0}};
    const int64_t len = max(qe[0] - qb[0], qe[1] - qb[1]);
    for (int64_t o = l; o < len; o += 16) {
      int32_t jj[2];
      double aa[2];
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const bool on = qb[u] + o < qe[u];
        jj[u] = on ? col[qb[u] + o] : 0;
        aa[u] = on ? (double)val[qb[u] + o] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < 2; ++u)
        for (int k = 0; k < K; ++k) s[u][k] += aa[u] * X[(int64_t)k * d + jj[u]];
    }
#pragma unroll
    for (int u = 0; u < 2; ++u)
      for (int off = 8; off > 0; off >>= 1)
        for (int k = 0; k < 4; ++k) s[u][k] += __shfl_xor(s[u][k], off, 16);
    if (l == 0) {
#pragma unroll
      for (int u = 0; u < 2; ++u)
        if (ii[u] < n) {
          const double bi = (double)b[ii[u]];
          for (int k = 0; k < K; ++k) R[ii[u] * K + k] = s[u][k] - bi;
        }
    }
  }
}

// A^T R over the column-major copy, each column cut into chunks of kAtrChunk
// entries (ccst[j] = first chunk of column j): a block sums its chunk with a
// fixed-shape tree into part[c][k]; the finish adds the chunks of a column in
// order, G[k][j] = sum + nu2 X[k][j].
constexpr int kAtrChunk = 4096;

template <typename T>
__global__ __launch_bounds__(256) void k_csc_partial(const int64_t* __restrict__ colptr,
                                                     const int32_t* __restrict__ crow,
                                                     const T* __restrict__ cval,
                                                     const int64_t* __restrict__ ccst, int64_t n,
                                                     int64_t d, const double* __restrict__ R,
                                                     int K, double* __restrict__ part,
                                                     const int* __restrict__ status) {
  if (status && *status != 0) return;
  __shared__ double sh[4][256];
  const int64_t c = blockIdx.x;
  if (c >= ccst[d]) return;
  const int64_t j = upper_index(ccst, d + 1, c);
  const int64_t q0 = colptr[j] + (c - ccst[j]) * kAtrChunk;
  const int64_t q1 = min(colptr[j + 1], q0 + (int64_t)kAtrChunk);
  double s[4] = {0.0, 0.0, 0.0, 0.0};
  // four entries per thread at a time: their rows and values, then the residual
  // gathers, then the products in entry order
  for (int64_t qb = q0 + threadIdx.x; qb < q1; qb += 4 * 256) {
    int32_t ii[4];
    double aa[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int64_t q = qb + (int64_t)u * 256;
      ii[u] = q < q1 ? crow[q] : -1;
      aa[u] = q < q1 ? (double)cval[q] : 0.0;
    }
    double rr[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int k = 0; k < 4; ++k)
        rr[u][k] = (ii[u] >= 0 && k < K) ? R[(int64_t)ii[u] * K + k] : 0.0;
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
      for (int k = 0; k < 4; ++k) s[k] += aa[u] * rr[u][k];
  }
  for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] = s[k];
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w)
      for (int k = 0; k < 4; ++k) sh[k][threadIdx.x] += sh[k][threadIdx.x + w];
    __syncthreads();
  }
  if ((int)threadIdx.x < K) part[c * 4 + threadIdx.x] = sh[threadIdx.x][0];
}

__global__ __launch_bounds__(256) void k_csc_finish(const int64_t* __restrict__ ccst, int64_t d,
                                                    const double* __restrict__ part, int K,
                                                    double nu2, const double* __restrict__ X,
                                                    double* __restrict__ G,
                                                    const int* __restrict__ status) {
  if (status && *status != 0) return;
  const int64_t t = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (t >= (int64_t)K * d) return;
  const int64_t k = t / d, j = t - k * d;
  double v = 0.0;
  for (int64_t c = ccst[j]; c < ccst[j + 1]; ++c) v += part[c * 4 + k];
  G[t] = v + nu2 * X[t];
}

static unsigned grid_for(int64_t n) {
  return (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 8192));
}

static int bits_for(uint64_t v) {  // bits to hold values 0..v
  int b = 1;
  while (b < 32 && (v >> b) != 0) ++b;
  return b;
}

// ------------------------------------------------------------ scan and sort
// Exclusive prefix sums of int64 values: blocks of 1024 (256 threads x 4) scan
// their part in LDS and leave their totals, which are scanned the same way (one
// level per factor of 1024), then added back.
constexpr int kScanBlock = 1024;

__global__ __launch_bounds__(256) void k_scan_block(const int64_t* __restrict__ in, int64_t n,
                                                    int64_t* __restrict__ out,
                                                    int64_t* __restrict__ totals) {
  __shared__ int64_t sh[256];
  const int t = threadIdx.x;
  const int64_t base = (int64_t)blockIdx.x * kScanBlock + 4 * t;
  int64_t v[4], run = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    v[e] = base + e < n ? in[base + e] : 0;
    run += v[e];
  }
  sh[t] = run;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {  // inclusive scan of the thread sums
    const int64_t x = t >= off ? sh[t - off] : 0;
    __syncthreads();
    sh[t] += x;
    __syncthreads();
  }
  int64_t acc = sh[t] - run;  // exclusive start of this thread
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    if (base + e < n) out[base + e] = acc;
    acc += v[e];
  }
  if (t == 255 && totals) totals[blockIdx.x] = sh[255];
}

__global__ __launch_bounds__(256) void k_scan_add(int64_t* __restrict__ out, int64_t n,
                                                  const int64_t* __restrict__ starts) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) out[i] += starts[i / kScanBlock];
}

// Scratch int64 values needed by excl_scan for n values (every level's totals).
static int64_t scan_scratch(int64_t n) {
  int64_t need = 0;
  for (int64_t m = (n + kScanBlock - 1) / kScanBlock; m > 1; m = (m + kScanBlock - 1) / kScanBlock)
    need += 2 * m;
  return need + 2;
}

// out = exclusive prefix sums of in (n values); work holds scan_scratch(n) values.
static rs_status excl_scan(const int64_t* in, int64_t* out, int64_t n, int64_t* work,
                           hipStream_t s) {
  if (n <= 0) return RS_OK;
  const int64_t nb = (n + kScanBlock - 1) / kScanBlock;
  if (nb == 1) {
    hipLaunchKernelGGL(k_scan_block, dim3(1), dim3(256), 0, s, in, n, out, (int64_t*)nullptr);
    return check_launch("scan");
  }
  int64_t* totals = work;
  int64_t* starts = work + nb;
  hipLaunchKernelGGL(k_scan_block, dim3((unsigned)nb), dim3(256), 0, s, in, n, out, totals);
  SP_TRY(excl_scan(totals, starts, nb, work + 2 * nb, s));
  hipLaunchKernelGGL(k_scan_add, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, out, n,
                     (const int64_t*)starts);
  return check_launch("scan");
}

// Stable LSD radix sort of (key, value) pairs on the low end_bit key bits, 8 bits a
// pass.  A pass: every block counts the digits of its chunk of kSortChunk pairs
// (hist[digit][block]); one exclusive scan over that digit-major table gives each
// (digit, block) its first output slot; every block then walks its chunk in order,
// 256 pairs at a time, and places each pair after the equal digits before it (its
// rank in the wave from 8 ballots, the waves before it from LDS counts), so equal
// keys keep their input order.
constexpr int kSortChunk = 4096;

__global__ __launch_bounds__(256) void k_sort_hist(const uint32_t* __restrict__ key, int64_t n,
                                                   int shift, int nblk,
                                                   int64_t* __restrict__ hist) {
  __shared__ int cnt[256];
  const int t = threadIdx.x;
  cnt[t] = 0;
  __syncthreads();
  const int64_t c0 = (int64_t)blockIdx.x * kSortChunk;
  for (int i = t; i < kSortChunk; i += 256)
    if (c0 + i < n) atomicAdd(&cnt[(key[c0 + i] >> shift) & 255u], 1);
  __syncthreads();
  hist[(int64_t)t * nblk + blockIdx.x] = cnt[t];
}

template <typename V>
__global__ __launch_bounds__(256) void k_sort_scatter(const uint32_t* __restrict__ kin,
                                                      const V* __restrict__ vin, int64_t n,
                                                      int shift, int nblk,
                                                      const int64_t* __restrict__ start,
                                                      uint32_t* __restrict__ kout,
                                                      V* __restrict__ vout) {
  __shared__ int64_t base[256];
  __shared__ int wcnt[4][256];
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  base[t] = start[(int64_t)t * nblk + blockIdx.x];
#pragma unroll
  for (int ww = 0; ww < 4; ++ww) wcnt[ww][t] = 0;
  __syncthreads();
  const uint64_t lt = (1ull << lane) - 1ull;
  const int64_t c0 = (int64_t)blockIdx.x * kSortChunk;
  for (int tile = 0; tile < kSortChunk; tile += 256) {
    const int64_t i = c0 + tile + t;
    const bool ok = i < n;
    const uint32_t k = ok ? kin[i] : 0u;
    const V v = ok ? vin[i] : V(0);
    const int dg = (int)((k >> shift) & 255u);
    // lanes of this wave holding the same digit
    uint64_t same = __ballot(ok);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bits = __ballot((dg >> b) & 1);
      same &= ((dg >> b) & 1) ? bits : ~bits;
    }
    const int rank = __popcll(same & lt);
    if (ok && lane == 63 - __clzll(same)) wcnt[w][dg] = __popcll(same);
    __syncthreads();
    if (ok) {
      int64_t pos = base[dg] + rank;
      for (int ww = 0; ww < w; ++ww) pos += wcnt[ww][dg];
      kout[pos] = k;
      vout[pos] = v;
    }
    __syncthreads();
    base[t] += wcnt[0][t] + wcnt[1][t] + wcnt[2][t] + wcnt[3][t];
#pragma unroll
    for (int ww = 0; ww < 4; ++ww) wcnt[ww][t] = 0;
    __syncthreads();
  }
}

// Scratch bytes of radix_pairs for n pairs of value type V.
template <typename V>
static size_t sort_scratch(int64_t n) {
  const int64_t nblk = (n + kSortChunk - 1) / kSortChunk;
  return (size_t)n * (sizeof(uint32_t) + sizeof(V)) + 64 +  // + two 16-byte alignments
         (size_t)(2 * 256 * nblk + scan_scratch(256 * nblk)) * sizeof(int64_t);
}

// Stable sort of (key, value) pairs by the low end_bit key bits into kout / vout (kin
// and vin unchanged), scratch grown in place.
template <typename V>
static rs_status radix_pairs(const uint32_t* kin, uint32_t* kout, const V* vin, V* vout, int64_t n,
                             int end_bit, GrowBuf& tmp, hipStream_t s) {
  if (n <= 0) return RS_OK;
  if (n > ((int64_t)1 << 31)) return set_error(RS_ERR_SHAPE, "sparse: more than 2^31 pairs");
  SP_TRY(tmp.ensure(sort_scratch<V>(n)));
  const int nblk = (int)((n + kSortChunk - 1) / kSortChunk);
  char* p = tmp.as<char>();
  uint32_t* kalt = reinterpret_cast<uint32_t*>(p);
  p += (size_t)n * sizeof(uint32_t);
  p = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(p) + 15) & ~uintptr_t(15));
  V* valt = reinterpret_cast<V*>(p);
  p += (size_t)n * sizeof(V);
  p = reinterpret_cast<char*>((reinterpret_cast<uintptr_t>(p) + 15) & ~uintptr_t(15));
  int64_t* hist = reinterpret_cast<int64_t*>(p);
  int64_t* start = hist + (int64_t)256 * nblk;
  int64_t* work = start + (int64_t)256 * nblk;
  const int passes = (end_bit + 7) / 8;
  const uint32_t* ksrc = kin;
  const V* vsrc = vin;
  for (int ps = 0; ps < passes; ++ps) {
    // the last pass writes kout / vout
    const bool to_out = ((passes - 1 - ps) & 1) == 0;
    uint32_t* kdst = to_out ? kout : kalt;
    V* vdst = to_out ? vout : valt;
    hipLaunchKernelGGL(k_sort_hist, dim3((unsigned)nblk), dim3(256), 0, s, ksrc, n, 8 * ps, nblk,
                       hist);
    SP_TRY(excl_scan(hist, start, (int64_t)256 * nblk, work, s));
    hipLaunchKernelGGL(k_sort_scatter<V>, dim3((unsigned)nblk), dim3(256), 0, s, ksrc, vsrc, n,
                       8 * ps, nblk, (const int64_t*)start, kdst, vdst);
    ksrc = kdst;
    vsrc = vdst;
  }
  return check_launch("radix sort");
}

// cst = exclusive prefix sum of the chunk counts of the nseg segments given by off
// (cst[nseg] = total chunks)
static rs_status chunk_starts(const int64_t* off, int64_t nseg, int64_t per, GrowBuf& nch,
                              GrowBuf& cst, GrowBuf& tmp, hipStream_t s) {
  SP_TRY(nch.ensure((size_t)(nseg + 1) * sizeof(int64_t)));
  SP_TRY(cst.ensure((size_t)(nseg + 1) * sizeof(int64_t)));
  hipLaunchKernelGGL(k_chunk_counts, dim3(grid_for(nseg + 1)), dim3(256), 0, s, off, nseg, per,
                     nch.as<int64_t>());
  SP_TRY(tmp.ensure((size_t)scan_scratch(nseg + 1) * sizeof(int64_t)));
  SP_TRY(excl_scan(nch.as<int64_t>(), cst.as<int64_t>(), nseg + 1, tmp.as<int64_t>(), s));
  return check_launch("sparse chunks");
}

rs_status sparse_check(SparseWork& W, const SparseA& sp, hipStream_t s, int* bad_host) {
  SP_TRY(W.flag.ensure(sizeof(int)));
  SP_HIP(hipMemsetAsync(W.flag.p, 0, sizeof(int), s));
  hipLaunchKernelGGL(k_csr_check, dim3(grid_for(std::max(sp.n, sp.nnz))), dim3(256), 0, s,
                     sp.rowptr, sp.n, sp.col, sp.nnz, sp.d, W.flag.as<int>());
  SP_TRY(check_launch("sparse check"));
  SP_HIP(hipMemcpyAsync(bad_host, W.flag.p, sizeof(int), hipMemcpyDeviceToHost, s));
  SP_HIP(hipStreamSynchronize(s));
  return RS_OK;
}

rs_status sparse_to_csc(SparseWork& W, const SparseA& sp, hipStream_t s) {
  const int64_t nnz = sp.nnz;
  SP_TRY(W.ckey.ensure((size_t)nnz * sizeof(uint32_t) * 2));
  SP_TRY(W.cpos.ensure((size_t)nnz * sizeof(int64_t) * 2));
  SP_TRY(W.rid.ensure((size_t)std::max<int64_t>(nnz, 1) * sizeof(int32_t)));
  SP_TRY(W.crow.ensure((size_t)std::max<int64_t>(nnz, 1) * sizeof(int32_t)));
  SP_TRY(W.cval.ensure((size_t)std::max<int64_t>(nnz, 1) * value_size(sp.a_t)));
  SP_TRY(W.colptr.ensure((size_t)(sp.d + 1) * sizeof(int64_t)));
  uint32_t* k0 = W.ckey.as<uint32_t>();
  uint32_t* k1 = k0 + nnz;
  int64_t* p0 = W.cpos.as<int64_t>();
  int64_t* p1 = p0 + nnz;
  // column of every entry as the key, its position as the value (no entries: every
  // column is empty and only the offsets are written)
  if (nnz > 0) {
    SP_HIP(hipMemcpyAsync(k0, sp.col, (size_t)nnz * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    hipLaunchKernelGGL(k_iota, dim3(grid_for(nnz)), dim3(256), 0, s, nnz, p0);
    hipLaunchKernelGGL(k_expand_rows, dim3((unsigned)std::min<int64_t>((sp.n + 3) / 4, 65535)),
                       dim3(256), 0, s, sp.rowptr, sp.n, W.rid.as<int32_t>());
    SP_TRY(radix_pairs(k0, k1, p0, p1, nnz, bits_for((uint64_t)sp.d), W.tmp, s));
  }
  hipLaunchKernelGGL(k_segment_offsets, dim3(grid_for(nnz + 1)), dim3(256), 0, s, k1, nnz,
                     (uint32_t)sp.d, W.colptr.as<int64_t>());
  if (nnz == 0)
    ;
  else if (sp.a_t == RS_F32)
    hipLaunchKernelGGL(k_gather_csc<float>, dim3(grid_for(nnz)), dim3(256), 0, s, nnz, p1,
                       W.rid.as<int32_t>(), reinterpret_cast<const float*>(sp.val),
                       W.crow.as<int32_t>(), W.cval.as<float>());
  else
    hipLaunchKernelGGL(k_gather_csc<double>, dim3(grid_for(nnz)), dim3(256), 0, s, nnz, p1,
                       W.rid.as<int32_t>(), reinterpret_cast<const double*>(sp.val),
                       W.crow.as<int32_t>(), W.cval.as<double>());
  SP_TRY(check_launch("sparse csc"));
  // chunks of the columns for the A^T r pass: at most nnz / kAtrChunk + d
  W.atr_chunks = nnz / kAtrChunk + sp.d;
  SP_TRY(W.cpart.ensure((size_t)W.atr_chunks * 4 * sizeof(double)));
  return chunk_starts(W.colptr.as<int64_t>(), sp.d, kAtrChunk, W.cnch, W.ccst, W.tmp, s);
}

rs_status sparse_gradient(SparseWork& W, const SparseA& sp, const void* b, double nu2,
                          const double* X, int K, double* G, const int* status, hipStream_t s,
                          const double* sub) {
  if (K < 1 || K > 4) return set_error(RS_ERR_ARG, "sparse gradient: k must be in 1..4");
  if (sub) return set_error(RS_ERR_UNSUPPORTED, "sparse gradient: no subtracted vector");
  SP_TRY(W.R.ensure((size_t)4 * sp.n * sizeof(double)));
  double* R = W.R.as<double>();
  const unsigned rg = (unsigned)std::max<int64_t>(1, std::min<int64_t>((sp.n + 31) / 32, 65536));
  const unsigned cg = (unsigned)std::max<int64_t>(W.atr_chunks, 1);
  const unsigned fg = (unsigned)(((int64_t)K * sp.d + 255) / 256);
  // the pass is timed from the row kernel's start to the finish kernel's stop when
  // profiling is on
  const ProfSlot ps = prof_begin();
  if (sp.a_t == RS_F32) {
    launch_timed(k_csr_resid<float>, dim3(rg), dim3(256), s, ps.begin, nullptr, sp.rowptr, sp.col,
                 reinterpret_cast<const float*>(sp.val), reinterpret_cast<const float*>(b), sp.n,
                 sp.d, X, K, R, status, ps.ran);
    hipLaunchKernelGGL(k_csc_partial<float>, dim3(cg), dim3(256), 0, s, W.colptr.as<int64_t>(),
                       W.crow.as<int32_t>(), W.cval.as<float>(), W.ccst.as<int64_t>(), sp.n, sp.d,
                       R, K, W.cpart.as<double>(), status);
  } else {
    launch_timed(k_csr_resid<double>, dim3(rg), dim3(256), s, ps.begin, nullptr, sp.rowptr,
                 sp.col, reinterpret_cast<const double*>(sp.val),
                 reinterpret_cast<const double*>(b), sp.n, sp.d, X, K, R, status, ps.ran);
    hipLaunchKernelGGL(k_csc_partial<double>, dim3(cg), dim3(256), 0, s, W.colptr.as<int64_t>(),
                       W.crow.as<int32_t>(), W.cval.as<double>(), W.ccst.as<int64_t>(), sp.n, sp.d,
                       R, K, W.cpart.as<double>(), status);
  }
  launch_timed(k_csc_finish, dim3(fg), dim3(256), s, nullptr, ps.end, W.ccst.as<int64_t>(), sp.d,
               (const double*)W.cpart.as<double>(), K, nu2, X, G, status);
  return check_launch("sparse gradient");
}

rs_status count_sketch_run(SparseWork& W, const SparseA& sp, int64_t m, uint64_t seed,
                           uint32_t sid, void* SA, rs_dtype sa_t, int64_t ldsa, hipStream_t s) {
  const int64_t n = sp.n;
  if ((size_t)sp.d * sizeof(double) > 65536)
    return set_error(RS_ERR_SHAPE, "count sketch: d above 8192");
  SP_TRY(W.hkey.ensure((size_t)n * sizeof(uint32_t) * 2));
  SP_TRY(W.hrow.ensure((size_t)n * sizeof(int32_t) * 2));
  SP_TRY(W.hsign.ensure((size_t)n * sizeof(float)));
  SP_TRY(W.hoff.ensure((size_t)(m + 1) * sizeof(int64_t)));
  uint32_t* k0 = W.hkey.as<uint32_t>();
  uint32_t* k1 = k0 + n;
  int32_t* r0 = W.hrow.as<int32_t>();
  int32_t* r1 = r0 + n;
  hipLaunchKernelGGL(k_cs_hash, dim3(grid_for(n)), dim3(256), 0, s, n, seed, sid, (uint32_t)m, k0,
                     r0, W.hsign.as<float>());
  SP_TRY(radix_pairs(k0, k1, r0, r1, n, bits_for((uint64_t)(m - 1)), W.tmp, s));
  hipLaunchKernelGGL(k_segment_offsets, dim3(grid_for(n + 1)), dim3(256), 0, s, k1, n,
                     (uint32_t)m, W.hoff.as<int64_t>());
  // chunks of the buckets: at most n / kCsChunk + m
  SP_TRY(chunk_starts(W.hoff.as<int64_t>(), m, kCsChunk, W.hnch, W.hcst, W.tmp, s));
  const int64_t chunks = n / kCsChunk + m;
  SP_TRY(W.spart.ensure((size_t)chunks * sp.d * sizeof(double)));
  // groups of 16 lanes, each with an FP64 LDS row: 64 KB of LDS at most
  const int groups = (int)std::max<int64_t>(1, std::min<int64_t>(16, 8192 / sp.d));
  const size_t lds = (size_t)groups * sp.d * sizeof(double);
  if (sp.a_t == RS_F32)
    hipLaunchKernelGGL(k_cs_partial<float>, dim3((unsigned)chunks), dim3(16 * groups), lds, s,
                       sp.rowptr, sp.col, reinterpret_cast<const float*>(sp.val), r1,
                       W.hsign.as<float>(), W.hoff.as<int64_t>(), W.hcst.as<int64_t>(), m, sp.d,
                       groups, W.spart.as<double>());
  else
    hipLaunchKernelGGL(k_cs_partial<double>, dim3((unsigned)chunks), dim3(16 * groups), lds, s,
                       sp.rowptr, sp.col, reinterpret_cast<const double*>(sp.val), r1,
                       W.hsign.as<float>(), W.hoff.as<int64_t>(), W.hcst.as<int64_t>(), m, sp.d,
                       groups, W.spart.as<double>());
  const dim3 g2((unsigned)m, (unsigned)((ldsa + 15) / 16));
#define RS_CS_SUM(TO)                                                                             \
  hipLaunchKernelGGL((k_cs_sum<TO>), g2, dim3(256), 0, s, W.spart.as<double>(),                  \
                     W.hcst.as<int64_t>(), sp.d, reinterpret_cast<TO*>(SA), ldsa)
  if (sa_t == RS_F32) RS_CS_SUM(float);
  else if (sa_t == RS_BF16 && sp.a_t == RS_F32) RS_CS_SUM(uint16_t);
  else if (sa_t == RS_F64 && sp.a_t == RS_F64) RS_CS_SUM(double);
  else return set_error(RS_ERR_UNSUPPORTED, "count sketch: sketch dtype not supported");
#undef RS_CS_SUM
  return check_launch("count sketch");
}

#undef SP_HIP
#undef SP_TRY

}  // namespace rs
