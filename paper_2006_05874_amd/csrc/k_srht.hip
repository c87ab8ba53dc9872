// SRHT embedding SA = (1/sqrt(m)) R H diag(eps) A on the device (Appendix C.2).
//
// Randomness: eps_i and row keys from Philox4x32-10 (streams 4 and 5).  R is the
// m rows with the smallest (key, index): a one-level radix select on the top
// 12 key bits finds the boundary bin, its few members are sorted in one block,
// and a stream compaction writes the chosen rows in ascending order.
//
// Transform: H of order npad = n1 * n2 factors as H_{n1} (x) H_{n2} on the row
// index i = i1 * n2 + i2 (Sylvester order).  Pass 1 transforms every block of
// n2 = min(npad, 1024) consecutive rows (with the sign flip fused into the load)
// and keeps only the i2 values that some sampled row uses (Q of them).  Pass 2
// transforms along i1 (length n1) for those Q columns and writes the sampled
// rows, scaled by 1/sqrt(m), straight into SA.  A pass streams a tile of
// 1024 rows x 128 bytes per block: 32 rows per thread sit in registers for the
// butterflies of the high row bits, one LDS transpose brings the low row bits
// into registers for the rest, and HBM sees whole 128-byte row segments.
#include "rs_internal.hpp"

namespace rs {

constexpr int kHistBits = 12;
constexpr int kHistBins = 1 << kHistBits;
constexpr int kCandCap = 8192;
constexpr int kCompactBlock = 1024;  // elements per block in the compaction

// ---------------------------------------------------------------- selection
// hist (kHistBins) must be zero on entry.  Also writes the signs and resets the
// row->sample map to -1.
__global__ __launch_bounds__(256) void k_keys_hist(uint64_t seed, uint32_t sid, int64_t npad,
                                                   uint32_t* __restrict__ hist,
                                                   int8_t* __restrict__ signs,
                                                   int32_t* __restrict__ kmap) {
  __shared__ uint32_t h[kHistBins];
  for (int i = threadIdx.x; i < kHistBins; i += blockDim.x) h[i] = 0;
  __syncthreads();
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npad;
       i += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t key = row_key(seed, sid, (uint64_t)i);
    atomicAdd(&h[(uint32_t)(key >> (64 - kHistBits))], 1u);
    signs[i] = (int8_t)sign_of(seed, sid, (uint64_t)i);
    kmap[i] = -1;
  }
  __syncthreads();
  for (int i = threadIdx.x; i < kHistBins; i += blockDim.x)
    if (h[i]) atomicAdd(&hist[i], h[i]);
}

struct SelectState {
  uint32_t bstar;      // boundary bin
  uint32_t need;       // rows still to take from the boundary bin
  uint32_t ncand;      // members of the boundary bin found
  uint32_t overflow;   // set when the boundary bin exceeds kCandCap
  uint64_t tkey;       // (tkey, tidx): the last selected (key, index)
  int64_t tidx;
};

// One block of 1024 threads: prefix sums over the histogram, locate the bin
// holding the m-th smallest key; clears the histogram for the next call.
__global__ __launch_bounds__(1024) void k_select_bin(uint32_t* __restrict__ hist, int64_t m,
                                                     SelectState* __restrict__ st) {
  __shared__ uint32_t part[1024];
  constexpr int PER = kHistBins / 1024;
  uint32_t loc[PER];
  uint32_t tot = 0;
  for (int j = 0; j < PER; ++j) {
    loc[j] = hist[threadIdx.x * PER + j];
    tot += loc[j];
  }
  part[threadIdx.x] = tot;
  __syncthreads();
  // inclusive scan over 1024 thread totals (Hillis-Steele)
  for (int off = 1; off < 1024; off <<= 1) {
    uint32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t before = threadIdx.x ? part[threadIdx.x - 1] : 0u;
  for (int j = 0; j < PER; ++j) {
    const uint32_t after = before + loc[j];
    if ((uint64_t)before < (uint64_t)m && (uint64_t)m <= (uint64_t)after) {
      st->bstar = threadIdx.x * PER + j;
      st->need = (uint32_t)(m - before);
    }
    before = after;
  }
  for (int j = 0; j < PER; ++j) hist[threadIdx.x * PER + j] = 0u;
  if (threadIdx.x == 0) {
    st->ncand = 0;
    st->overflow = 0;
  }
}

// Members of the boundary bin -> candidate list; per-block counts of keys in
// lower bins.
__global__ __launch_bounds__(256) void k_collect(uint64_t seed, uint32_t sid, int64_t npad,
                                                 SelectState* __restrict__ st,
                                                 uint64_t* __restrict__ cand_key,
                                                 int64_t* __restrict__ cand_idx,
                                                 uint32_t* __restrict__ blk_less) {
  __shared__ uint32_t cnt;
  if (threadIdx.x == 0) cnt = 0;
  __syncthreads();
  const uint32_t bstar = st->bstar;
  const int64_t b0 = (int64_t)blockIdx.x * kCompactBlock;
  uint32_t mine = 0;
  for (int j = threadIdx.x; j < kCompactBlock; j += blockDim.x) {
    const int64_t i = b0 + j;
    if (i >= npad) break;
    const uint64_t key = row_key(seed, sid, (uint64_t)i);
    const uint32_t bin = (uint32_t)(key >> (64 - kHistBits));
    if (bin < bstar) ++mine;
    else if (bin == bstar) {
      const uint32_t pos = atomicAdd(&st->ncand, 1u);
      if (pos < (uint32_t)kCandCap) {
        cand_key[pos] = key;
        cand_idx[pos] = i;
      } else {
        st->overflow = 1u;
      }
    }
  }
  atomicAdd(&cnt, mine);
  __syncthreads();
  if (threadIdx.x == 0) blk_less[blockIdx.x] = cnt;
}

// One block: sort the candidates by (key, index) (bitonic), keep the first `need`,
// record the threshold, and turn blk_less into exclusive offsets.  The sort runs
// in LDS sized at launch for the expected bin population (`cap` entries, dynamic
// shared memory, so the block does not reserve the worst case and can start next
// to other kernels); a bin larger than that is sorted in place in global memory.
template <typename KeyT, typename IdxT>
__device__ __forceinline__ void bitonic_by_key_index(KeyT* sk, IdxT* si, uint32_t P) {
  for (uint32_t k = 2; k <= P; k <<= 1) {
    for (uint32_t j = k >> 1; j > 0; j >>= 1) {
      for (uint32_t i = threadIdx.x; i < P; i += blockDim.x) {
        const uint32_t l = i ^ j;
        if (l > i) {
          const bool up = (i & k) == 0;
          const bool gt = (sk[i] > sk[l]) || (sk[i] == sk[l] && si[i] > si[l]);
          if (gt == up) {
            KeyT tk = sk[i]; sk[i] = sk[l]; sk[l] = tk;
            IdxT ti = si[i]; si[i] = si[l]; si[l] = ti;
          }
        }
      }
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(1024) void k_cand_sort(SelectState* __restrict__ st,
                                                    uint64_t* __restrict__ cand_key,
                                                    int64_t* __restrict__ cand_idx,
                                                    uint32_t* __restrict__ blk_less, int nblk,
                                                    uint32_t cap) {
  extern __shared__ __attribute__((aligned(16))) unsigned char dyn[];
  __shared__ uint32_t part[1024];
  const uint32_t nc = st->ncand < (uint32_t)kCandCap ? st->ncand : (uint32_t)kCandCap;
  uint32_t P = 1;
  while (P < nc) P <<= 1;
  uint64_t* sk;
  int64_t* si;
  if (P <= cap) {
    sk = reinterpret_cast<uint64_t*>(dyn);
    si = reinterpret_cast<int64_t*>(dyn + (size_t)cap * sizeof(uint64_t));
    for (uint32_t i = threadIdx.x; i < P; i += blockDim.x) {
      sk[i] = i < nc ? cand_key[i] : ~0ull;
      si[i] = i < nc ? cand_idx[i] : (int64_t)0x7fffffffffffffffll;
    }
  } else {
    // rare: the lists in global memory (capacity kCandCap) padded in place
    sk = cand_key;
    si = cand_idx;
    for (uint32_t i = nc + threadIdx.x; i < P; i += blockDim.x) {
      sk[i] = ~0ull;
      si[i] = (int64_t)0x7fffffffffffffffll;
    }
  }
  __syncthreads();
  bitonic_by_key_index(sk, si, P);
  const uint32_t need = st->need;
  // write back the selected members sorted by index order is not needed: keep
  // them sorted by (key, idx); the scatter pass only counts them.
  // (in the global fallback the sorted indices are already in cand_idx)
  if (P <= cap)
    for (uint32_t i = threadIdx.x; i < need && i < nc; i += blockDim.x) cand_idx[i] = si[i];
  if (threadIdx.x == 0 && need >= 1 && need <= nc) {
    st->tkey = sk[need - 1];
    st->tidx = si[need - 1];
  }
  // exclusive scan of blk_less (nblk <= 1024 * PER)
  const int PER = (nblk + 1023) / 1024;
  uint32_t tot = 0;
  for (int j = 0; j < PER; ++j) {
    const int b = threadIdx.x * PER + j;
    tot += b < nblk ? blk_less[b] : 0u;
  }
  part[threadIdx.x] = tot;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    uint32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = threadIdx.x ? part[threadIdx.x - 1] : 0u;
  for (int j = 0; j < PER; ++j) {
    const int b = threadIdx.x * PER + j;
    if (b < nblk) {
      const uint32_t v = blk_less[b];
      blk_less[b] = run;
      run += v;
    }
  }
}

// Compaction: rows[offset + local rank] = i for every selected i, ascending.
// Also fills kmap[row] = k and marks the used low indices (row & (n2-1)).
__global__ __launch_bounds__(256) void k_scatter_rows(uint64_t seed, uint32_t sid, int64_t npad,
                                                      const SelectState* __restrict__ st,
                                                      const int64_t* __restrict__ sel_cand_idx,
                                                      const uint32_t* __restrict__ blk_off,
                                                      int64_t* __restrict__ rows,
                                                      int32_t* __restrict__ kmap,
                                                      int32_t* __restrict__ used, int64_t n2mask,
                                                      int64_t m) {
  __shared__ uint32_t wsum[4];
  __shared__ uint32_t base_s;
  const uint32_t bstar = st->bstar;
  const uint64_t tkey = st->tkey;
  const int64_t tidx = st->tidx;
  const int64_t b0 = (int64_t)blockIdx.x * kCompactBlock;
  if (threadIdx.x == 0) {
    // selected boundary members with index below this block
    uint32_t c = 0;
    const uint32_t need = min(st->need, (uint32_t)kCandCap);
    for (uint32_t j = 0; j < need; ++j) c += sel_cand_idx[j] < b0 ? 1u : 0u;
    base_s = blk_off[blockIdx.x] + c;
  }
  __syncthreads();
  uint32_t base = base_s;
  constexpr int PER = kCompactBlock / 256;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  for (int p = 0; p < PER; ++p) {
    const int64_t i = b0 + p * 256 + threadIdx.x;
    bool sel = false;
    if (i < npad) {
      const uint64_t key = row_key(seed, sid, (uint64_t)i);
      const uint32_t bin = (uint32_t)(key >> (64 - kHistBits));
      sel = bin < bstar || (bin == bstar && (key < tkey || (key == tkey && i <= tidx)));
    }
    const uint64_t ballot = __ballot(sel);
    const uint32_t below = (uint32_t)__popcll(ballot & ((1ull << lane) - 1ull));
    if (lane == 0) wsum[wave] = (uint32_t)__popcll(ballot);
    __syncthreads();
    uint32_t off = base;
    for (int w = 0; w < wave; ++w) off += wsum[w];
    if (sel && (int64_t)(off + below) < m) {
      const uint32_t k = off + below;
      rows[k] = i;
      kmap[i] = (int32_t)k;
      used[i & n2mask] = 1;
    }
    uint32_t tot = 0;
    for (int w = 0; w < 4; ++w) tot += wsum[w];
    __syncthreads();
    base += tot;
  }
}

// One block: used[n2] -> qmap (i2 -> q or -1), qlist (q -> i2), Q; clears used.
__global__ __launch_bounds__(1024) void k_qscan(int32_t* __restrict__ used, int n2,
                                                int32_t* __restrict__ qmap,
                                                int32_t* __restrict__ qlist,
                                                int32_t* __restrict__ qcount) {
  __shared__ int32_t part[1024];
  const int i = threadIdx.x;
  const int u = (i < n2) ? (used[i] != 0) : 0;
  part[i] = u;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    int v = i >= off ? part[i - off] : 0;
    __syncthreads();
    part[i] += v;
    __syncthreads();
  }
  if (i < n2) {
    const int q = part[i] - 1;
    qmap[i] = u ? q : -1;
    if (u) qlist[q] = i;
    used[i] = 0;
  }
  if (i == 1023) *qcount = part[1023];
}

// ---------------------------------------------------------------- transform
// One tile: 1024 rows x W columns (W*sizeof(T) = 128 bytes), 256 threads.
// Stage A: thread (g = t/8, c = t%8) holds rows r = g + 32 j, j = 0..31, and
// applies the butterflies of row bits 5..9; stage B (after an LDS transpose)
// holds rows r = 32 g + j and applies row bits 0..4.  Only row bits below lb
// take part (the transform length is 2^lb; tile rows above it are independent
// transforms).
template <typename T>
struct Tile {
  using V = typename VecOf<T>::type;
  static constexpr int VEC = VecOf<T>::n;
  static constexpr int CW = 8;           // vectors per tile row
  static constexpr int W = CW * VEC;     // columns per tile
  static constexpr int RT = 1024;        // rows per tile
  static constexpr int J = 32;           // rows per thread
};

template <typename V>
__device__ __forceinline__ void bfly(V& u, V& v);
template <>
__device__ __forceinline__ void bfly<float4>(float4& u, float4& v) {
  const float4 a = u, b = v;
  u = make_float4(a.x + b.x, a.y + b.y, a.z + b.z, a.w + b.w);
  v = make_float4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w);
}
template <>
__device__ __forceinline__ void bfly<double2>(double2& u, double2& v) {
  const double2 a = u, b = v;
  u = make_double2(a.x + b.x, a.y + b.y);
  v = make_double2(a.x - b.x, a.y - b.y);
}

template <typename V, int J>
__device__ __forceinline__ void reg_fwht(V (&v)[J], int bit_lo, int lb) {
  // butterflies over register-index bits; register bit s <-> row bit bit_lo + s
#pragma unroll
  for (int s = 0; s < 5; ++s) {
    if (bit_lo + s < lb) {
#pragma unroll
      for (int j = 0; j < J; ++j) {
        if ((j & (1 << s)) == 0) bfly(v[j], v[j | (1 << s)]);
      }
    }
  }
}

// Transpose buffer slot of (row r, vector c < 4): the row-bit-5..8 XOR spreads the
// 16 lanes served together over 16 different bank groups in both directions.
__device__ __forceinline__ int lds_slot(int r, int c) { return (r * 4 + c) ^ (((r >> 5) & 15) << 2); }

// The transform of one 1024-row tile held as v[j] = row g + 32 j by thread (g, c):
// stage A (row bits 5..9 in registers), an LDS transpose in two halves (vectors
// 0-3, then 4-7, so a block needs half the LDS and two blocks share a CU), stage B
// (row bits 0..4).  On return thread (g, c) holds rows 32 g + j.  Only row bits
// below lb take part.
template <typename V, int J>
__device__ __forceinline__ void tile_fwht(V (&v)[J], V* lds, int g, int c, int lb) {
  const int half = c >> 2;
  reg_fwht<V, J>(v, 5, lb);
  for (int h = 0; h < 2; ++h) {
    if (half == h) {
#pragma unroll
      for (int j = 0; j < J; ++j) lds[lds_slot(g + 32 * j, c & 3)] = v[j];
    }
    __syncthreads();
    if (half == h) {
#pragma unroll
      for (int j = 0; j < J; ++j) v[j] = lds[lds_slot(32 * g + j, c & 3)];
    }
    __syncthreads();
  }
  reg_fwht<V, J>(v, 0, lb);
}

// Row segment store: one 16-byte (8-byte for BF16) vector store when the segment
// lies inside the row and the destination is aligned (vec_ok, uniform), else
// element by element.
template <typename T>
__device__ __forceinline__ void store_row(T* out, int64_t ldo, int64_t orow, int64_t col0,
                                          int64_t d, const typename VecOf<T>::type& v, T scale,
                                          bool vec_ok) {
  using V = typename VecOf<T>::type;
  constexpr int VEC = VecOf<T>::n;
  if (vec_ok && col0 + VEC <= d) {
    V w;
#pragma unroll
    for (int e = 0; e < VEC; ++e) set(w, e, get(v, e) * scale);
    *reinterpret_cast<V*>(out + orow * ldo + col0) = w;
    return;
  }
#pragma unroll
  for (int e = 0; e < VEC; ++e)
    if (col0 + e < d) out[orow * ldo + col0 + e] = get(v, e) * scale;
}

__device__ __forceinline__ void store_row_bf16(uint16_t* out, int64_t ldo, int64_t orow,
                                               int64_t col0, int64_t d, const float4& v,
                                               float scale, bool vec_ok) {
  if (vec_ok && col0 + 4 <= d) {
    const uint32_t lo = (uint32_t)f32_to_bf16_rne(v.x * scale) |
                        ((uint32_t)f32_to_bf16_rne(v.y * scale) << 16);
    const uint32_t hi = (uint32_t)f32_to_bf16_rne(v.z * scale) |
                        ((uint32_t)f32_to_bf16_rne(v.w * scale) << 16);
    *reinterpret_cast<uint2*>(out + orow * ldo + col0) = make_uint2(lo, hi);
    return;
  }
#pragma unroll
  for (int e = 0; e < 4; ++e)
    if (col0 + e < d) out[orow * ldo + col0 + e] = f32_to_bf16_rne(get(v, e) * scale);
}

// mode 0: pass 1 writing Zc rows (j1*Q + qmap[i2]);
// mode 1: pass 1 writing SA rows kmap[row] (single pass, npad <= 1024);
// mode 2: pass 2 reading Zc, writing SA rows.  When the high index j1 has more
//   than 10 bits (npad > 2^20), its top hb bits are folded while loading: block
//   z = r1h sums Zc over j1h with signs (-1)^popcount(r1h & j1h), so the tile
//   transform over the low 10 bits of j1 yields the output rows whose high
//   index has r1h in its top bits.
// OutT: T, or uint16_t for BF16 output.
template <typename T, typename OutT, int MODE, bool FOLD = false>
__global__ __launch_bounds__(256) void k_fwht_tile(
    const T* __restrict__ src, int64_t n_src_rows, int64_t lds_src, int64_t d,
    const int8_t* __restrict__ signs, int lb, int64_t n2, int64_t Q,
    const int32_t* __restrict__ qmap, const int32_t* __restrict__ qlist,
    const int32_t* __restrict__ kmap, const int32_t* __restrict__ qcount,
    OutT* __restrict__ out, int64_t ldo, double scale, int hb) {
  using TT = Tile<T>;
  using V = typename TT::V;
  constexpr int VEC = TT::VEC;
  constexpr int J = TT::J;
  __shared__ V lds[TT::RT * TT::CW / 2];
  __shared__ int32_t dest[TT::RT];

  const int t = threadIdx.x;
  // lanes (g, c): 8 lanes cover a 128-byte row segment.  The LDS transpose runs in
  // two halves (vectors 0-3, then 4-7), so a block needs half the LDS and two
  // blocks fit a CU: one loads while the other computes
  const int c = t & 7;
  const int g = t >> 3;
  const int64_t col0 = ((int64_t)blockIdx.y * TT::CW + c) * VEC;
  const bool cvec = col0 < d;

  const int64_t tile = blockIdx.x;
  // destination of each tile row (index loads clamped in bounds, then masked)
  for (int r = t; r < TT::RT; r += 256) {
    int32_t dst = -1;
    if (MODE == 0) {
      const int32_t q = qmap[r < n2 ? r : 0];
      // q < Q holds for every kept index (the selection keeps at most Q of them);
      // the test keeps a tile's writes inside its Q rows regardless
      dst = (r < n2 && q >= 0 && q < Q) ? (int32_t)(tile * Q + q) : -1;
    } else if (MODE == 1) {
      const int32_t kk = kmap[r < n2 ? r : 0];
      dst = r < n2 ? kk : -1;
    } else {
      const int64_t n1 = (int64_t)1 << lb;
      const int64_t qq = r >> lb;
      const int64_t i1 = ((int64_t)blockIdx.z << lb) + (r & (n1 - 1));
      const int64_t q = tile * (TT::RT >> lb) + qq;
      const bool okq = q < (int64_t)(*qcount);
      const int32_t i2 = qlist[okq ? q : 0];
      const int32_t kk = kmap[okq ? i1 * n2 + i2 : 0];
      dst = okq ? kk : -1;
    }
    dest[r] = dst;
  }


  // load (stage A mapping): every load is issued unconditionally from a clamped
  // in-bounds address and masked afterwards, so all 32 stay in flight
  V v[J];
  T sgn[J];
  bool okr[J];
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int r = g + 32 * j;
    int64_t srow;
    bool ok;
    if (MODE == 2) {
      const int64_t n1 = (int64_t)1 << lb;
      const int64_t qq = r >> lb;
      const int64_t i1 = r & (n1 - 1);
      const int64_t q = tile * (TT::RT >> lb) + qq;
      srow = i1 * Q + q;
      ok = q < Q;
    } else {
      srow = tile * n2 + r;
      ok = (r < n2) && (srow < n_src_rows);
    }
    const int64_t srowc = ok ? srow : 0;
    okr[j] = ok && cvec;
    v[j] = *reinterpret_cast<const V*>(src + srowc * lds_src + (cvec ? col0 : 0));
    sgn[j] = (MODE == 2) ? (T)1 : (T)signs[srowc];
  }
  if (FOLD && MODE == 2 && hb > 0) {
    // fold the top hb bits of j1: Zc tile (h << lb) + i1 with sign by r1h & h
    const int64_t stride = ((int64_t)1 << lb) * Q;
    for (int h = 1; h < (1 << hb); ++h) {
      const T sh = (__popc(blockIdx.z & (unsigned)h) & 1) ? (T)-1 : (T)1;
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int r = g + 32 * j;
        const int64_t n1 = (int64_t)1 << lb;
        const int64_t q = tile * (TT::RT >> lb) + (r >> lb);
        const bool ok = q < Q;
        const int64_t srow = ok ? (int64_t)h * stride + (r & (n1 - 1)) * Q + q : 0;
        const V w = *reinterpret_cast<const V*>(src + srow * lds_src + (cvec ? col0 : 0));
#pragma unroll
        for (int e = 0; e < VEC; ++e) set(v[j], e, get(v[j], e) + sh * get(w, e));
      }
    }
  }
#pragma unroll
  for (int j = 0; j < J; ++j) {
#pragma unroll
    for (int e = 0; e < VEC; ++e) {
      const T xe = get(v[j], e) * sgn[j];
      set(v[j], e, (okr[j] && col0 + e < d) ? xe : (T)0);
    }
  }
  tile_fwht<V, J>(v, lds, g, c, lb);

  // vector stores need the row pitch and base aligned to the store width
  constexpr uintptr_t kAlign = sizeof(OutT) == 2 ? 8 : 16;
  const bool vec_ok = ((reinterpret_cast<uintptr_t>(out) |
                        (uintptr_t)(ldo * (int64_t)sizeof(OutT))) & (kAlign - 1)) == 0;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int r = 32 * g + j;
    const int32_t dst = dest[r];
    if (dst >= 0 && cvec) {
      if constexpr (sizeof(OutT) == 2) {
        store_row_bf16(reinterpret_cast<uint16_t*>(out), ldo, dst, col0, d, v[j], (float)scale,
                       vec_ok);
      } else {
        store_row<T>(reinterpret_cast<T*>(out), ldo, dst, col0, d, v[j], (T)scale, vec_ok);
      }
    }
  }
}

// ---------------------------------------------------------------- FP32 two-pass form
// For FP32 A with 1 < n1 <= 2048 the intermediate Z (the tile transforms along i2,
// kept at the Q low indices some sampled row uses) is stored panel-major:
// Z[((p * Qmax + q) * n1 + i1) * 32 + c], p a 32-column panel, so every row a
// first-pass block stores is one whole 128-byte line (64-byte half lines written by
// different blocks moved 3.5 TB/s in a store probe at this size, whole lines 4.7,
// a device copy's rate).  Pass 2 reads each (16-column half of a panel, q) as n1
// rows of 64 bytes at a 128-byte pitch and transforms all of i1 (up to 11 bits) in
// one tile, so Z is read exactly once; the two halves of a panel run on the same
// XCD at the same time, so each line comes from HBM once.
constexpr int kP2Rows = 2048;  // rows of a pass-2 tile
// panels per group in the first pass's work order: 16 when the pass mostly reads
// (few kept low indices), 4 when it also writes an intermediate as large as A
// (the blocks of one XCD then store to 16 different tiles at a time); measured on
// 2^21 x 8192: 21.7 against 24.5 ms at m = 128, 59.0 against 50.9 ms at m = 4096
constexpr int kP1GroupRead = 16;
constexpr int kP1GroupWrite = 4;
constexpr int kP2J = 64;       // rows per thread

// A raw buffer descriptor over `bytes` bytes at `base` (untyped loads; the loads
// below keep every offset inside the region, they do not rely on its range check).
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buf_rsrc(const void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, (int)bytes,
                                           0x00020000);
}

// Block: one (32-column panel, 1024-row tile i1 = tile0 + ...) work item in the
// order of p1_work.
// EDGE = false: tiles whose 1024 rows all lie below n (and n2 = 1024), loaded with
// buffer loads (tile base in scalar registers, one 32-bit lane offset, the row
// group's offset as the scalar offset), so 32 loads in flight cost no address
// registers.  EDGE = true: rows clamped below n.
// Work order: blocks are dispatched to the 8 XCDs in turn, so block L runs on XCD
// L % 8.  XCD j takes the j-th eighth of the work items w (in order), and w runs
// over groups of `pgroup` consecutive panels, all tiles of a group before the next
// (panel fastest inside a group): the blocks one XCD runs together cover pgroup
// column offsets of a few neighbouring tiles.
__device__ __forceinline__ void p1_work(int64_t L, int64_t panels, int64_t ntiles, int pgroup,
                                        int64_t& panel, int64_t& tile) {
  const int64_t W = panels * ntiles;
  const int64_t W8 = W / 8;
  const int64_t w = L < 8 * W8 ? (L % 8) * W8 + L / 8 : L;
  const int64_t G = pgroup;
  const int64_t gsize = G * ntiles;  // items of a full group
  const int64_t grp = w / gsize;
  const int64_t first = grp * G;
  const int64_t gw = panels - first < G ? panels - first : G;  // panels in this group
  const int64_t u = w - grp * gsize;
  tile = u / gw;
  panel = first + u % gw;
}

// One work item (32-column panel, tile) of the first pass, in LDS buffers the caller
// owns.  PROBE: also the learned start's column sums of this tile (ProbeArgs), taken
// from the loaded rows before the sign flip, reduced over the block's 32 row groups
// in the (still unused) transpose buffer.  IDQ: every low index kept in order (q = r,
// Qmax = n2, no qmap read).
template <bool EDGE, bool PROBE, bool IDQ>
__device__ __forceinline__ void p1_item(const float* __restrict__ A, int64_t n, int64_t d,
                                        int64_t lda, const int8_t* __restrict__ signs, int lb,
                                        int64_t n2, int64_t n1, int64_t Qmax,
                                        const int32_t* __restrict__ qmap, float* __restrict__ Z,
                                        int64_t panel, int64_t tile, const ProbeArgs& pa,
                                        float4* lds, int32_t* dest, float* sgn, uint8_t* pbit,
                                        float* bvl, int t) {
  using TT = Tile<float>;
  constexpr int J = TT::J;
  const int c = t & 7;
  const int g = t >> 3;
  const int64_t row0 = tile * n2;
  const int64_t col0 = (panel * TT::CW + c) * 4;
  // columns past d read column 0 and are zeroed (the last panel only)
  const int64_t colr = col0 < d ? col0 : 0;
  float4 v[J];
  if constexpr (!EDGE) {
    const uint32_t rowb = (uint32_t)(lda * 4);
    const __amdgpu_buffer_rsrc_t rs = buf_rsrc(A + row0 * lda, rowb * TT::RT);
    const uint32_t voff = (uint32_t)g * rowb + (uint32_t)colr * 4u;
#pragma unroll
    for (int j = 0; j < J; ++j)
      v[j] = __builtin_bit_cast(float4, __builtin_amdgcn_raw_buffer_load_b128(
                                            rs, voff, (uint32_t)j * 32u * rowb, 0));
  } else {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      int64_t i = row0 + g + 32 * j;
      i = i < n ? i : n - 1;
      v[j] = *reinterpret_cast<const float4*>(A + i * lda + colr);
    }
  }
  // the kept low indices and the signs (zero for tile rows past n2 or n, which then
  // add nothing), loaded behind the tile so that one memory round trip serves both
  static_assert(TT::RT == 4 * 256, "four tile rows per thread");
  int32_t qv[4];
  int8_t sv[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = t + 256 * u;
    const int64_t i = row0 + r;
    qv[u] = IDQ ? r : qmap[r < n2 ? r : 0];
    sv[u] = signs[(r < n2 && i < n) ? i : 0];
  }
  if constexpr (PROBE) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int r = t + 256 * u;
      const int64_t i = row0 + r;
      const bool ok = r < n2 && i < n;
      pbit[r] = ok ? pa.bits[i] : (uint8_t)0;
      bvl[r] = (ok && pa.b) ? pa.b[i] : 0.0f;
    }
  }
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const int r = t + 256 * u;
    const int64_t i = row0 + r;
    dest[r] = (r < n2 && qv[u] < Qmax) ? qv[u] : -1;
    sgn[r] = (r < n2 && i < n) ? (float)sv[u] : 0.0f;
  }
  __syncthreads();  // sgn and dest written
  if constexpr (PROBE) {
    // rows past n2 or n have sign 0 and add nothing; columns past d are masked
    float acc[kProbeCols][4];
#pragma unroll
    for (int k = 0; k < kProbeCols; ++k)
#pragma unroll
      for (int e = 0; e < 4; ++e) acc[k][e] = 0.0f;
    // every row and column of a full tile's panel is inside A except in the last
    // panel: only those blocks and the ragged tiles mask
    auto sums = [&](auto masked) {
      constexpr bool MASK = decltype(masked)::value;
#pragma unroll
      for (int j = 0; j < J; ++j) {
        const int r = g + 32 * j;
        const bool rv = !MASK || sgn[r] != 0.0f;
        const uint32_t bits = pbit[r];
        const float bv = bvl[r];
        // the row's 8 probe signs as +-1.0f (bit k moved to the sign bit of 1.0f),
        // so that each column takes one multiply-add per probe
        float sk[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) sk[k] = __uint_as_float(((bits >> k) << 31) | 0x3f800000u);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const float x = (!MASK || (rv && col0 + e < d)) ? get(v[j], e) : 0.0f;
#pragma unroll
          for (int k = 0; k < 8; ++k) acc[k][e] = fmaf(sk[k], x, acc[k][e]);
          acc[8][e] = fmaf(x, x, acc[8][e]);
          acc[9][e] = fmaf(bv, x, acc[9][e]);
        }
      }
    };
    if (!EDGE && n2 == TT::RT && col0 + 3 < d) sums(std::false_type{});
    else sums(std::true_type{});
    float* red = reinterpret_cast<float*>(lds);  // [32 row groups][10][32 columns]
#pragma unroll
    for (int k = 0; k < kProbeCols; ++k)
#pragma unroll
      for (int e = 0; e < 4; ++e) red[(g * kProbeCols + k) * 32 + c * 4 + e] = acc[k][e];
    __syncthreads();
    for (int q = t; q < kProbeCols * 32; q += 256) {
      const int k = q >> 5, col = q & 31;
      double sum = 0.0;
      for (int gg = 0; gg < 32; ++gg) sum += (double)red[(gg * kProbeCols + k) * 32 + col];
      const int64_t jc = panel * TT::W + col;
      if (jc < d) pa.part[(tile * kProbeCols + k) * pa.dp + jc] = sum;
    }
    __syncthreads();  // the transpose below reuses the buffer
  }
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const float sg = sgn[g + 32 * j];
#pragma unroll
    for (int e = 0; e < 4; ++e) set(v[j], e, get(v[j], e) * (col0 + e < d ? sg : 0.0f));
  }
  tile_fwht<float4, J>(v, lds, g, c, lb);
  // stores through a buffer descriptor over this block's 32-column panel of Z (at
  // most 1024 * 2048 rows of 128 bytes, inside 32-bit offsets): the 8 lanes of a
  // tile row write one whole 128-byte line
  const uint32_t pbytes = (uint32_t)(Qmax * n1 * 128);
  const __amdgpu_buffer_rsrc_t zs = buf_rsrc(Z + panel * Qmax * n1 * 32, pbytes);
  const uint32_t lane_off = (uint32_t)tile * 128u + (uint32_t)c * 16u;
  using U4 = __attribute__((ext_vector_type(4))) unsigned int;
#pragma unroll
  for (int j = 0; j < J; ++j) {
    const int32_t q = dest[32 * g + j];
    if (q >= 0)
      __builtin_amdgcn_raw_buffer_store_b128(__builtin_bit_cast(U4, v[j]), zs,
                                             lane_off + (uint32_t)q * (uint32_t)n1 * 128u, 0, 0);
  }
}

template <bool EDGE, bool PROBE>
__global__ __launch_bounds__(256) void k_srht_p1(const float* __restrict__ A, int64_t n,
                                                 int64_t d, int64_t lda,
                                                 const int8_t* __restrict__ signs, int lb,
                                                 int64_t n2, int64_t n1, int64_t Qmax,
                                                 const int32_t* __restrict__ qmap,
                                                 float* __restrict__ Z, int64_t tile0,
                                                 int64_t ntiles, int64_t panels, int pgroup,
                                                 ProbeArgs pa) {
  using TT = Tile<float>;
  __shared__ float4 lds[TT::RT * TT::CW / 2];
  __shared__ int32_t dest[TT::RT];
  __shared__ float sgn[TT::RT];
  __shared__ uint8_t pbit[PROBE ? TT::RT : 1];
  __shared__ float bvl[PROBE ? TT::RT : 1];
  int64_t panel, tloc;
  p1_work(blockIdx.x, panels, ntiles, pgroup, panel, tloc);
  p1_item<EDGE, PROBE, false>(A, n, d, lda, signs, lb, n2, n1, Qmax, qmap, Z, panel,
                              tile0 + tloc, pa, lds, dest, sgn, pbit, bvl, (int)threadIdx.x);
}

// The probe sketch's first pass (with the sums) and, from the same tile read again
// right after it (then mostly a cache hit, not HBM), the first pass of a second
// SRHT of the same A with its own signs (pa.signs2) and every low index kept, into
// pa.Z2 (the layout of a Qmax = n2 intermediate): a pair's features head and its
// first sketches' transform from one read of A.  Each item is computed exactly as
// k_srht_p1 computes it.
template <bool EDGE>
__global__ __launch_bounds__(256) void k_srht_p1_two(const float* __restrict__ A, int64_t n,
                                                     int64_t d, int64_t lda,
                                                     const int8_t* __restrict__ signs, int lb,
                                                     int64_t n2, int64_t n1, int64_t Qmax,
                                                     const int32_t* __restrict__ qmap,
                                                     float* __restrict__ Z, int64_t tile0,
                                                     int64_t ntiles, int64_t panels, int pgroup,
                                                     ProbeArgs pa) {
  using TT = Tile<float>;
  __shared__ float4 lds[TT::RT * TT::CW / 2];
  __shared__ int32_t dest[TT::RT];
  __shared__ float sgn[TT::RT];
  __shared__ uint8_t pbit[TT::RT];
  __shared__ float bvl[TT::RT];
  int64_t panel, tloc;
  p1_work(blockIdx.x, panels, ntiles, pgroup, panel, tloc);
  const int64_t tile = tile0 + tloc;
  p1_item<EDGE, true, false>(A, n, d, lda, signs, lb, n2, n1, Qmax, qmap, Z, panel, tile, pa,
                             lds, dest, sgn, pbit, bvl, (int)threadIdx.x);
  __syncthreads();  // the first item's stores have read dest
  // the thread index through an empty asm: the second item derives its addresses
  // anew instead of keeping the first item's live across it (they would not fit)
  int t2 = (int)threadIdx.x;
  asm volatile("" : "+v"(t2));
  p1_item<EDGE, false, true>(A, n, d, lda, pa.signs2, lb, n2, n1, n2, nullptr, pa.Z2, panel,
                             tile, pa, lds, dest, sgn, pbit, bvl, t2);
}

__device__ __forceinline__ void bfly2(float2& u, float2& v) {
  const float2 a = u, b = v;
  u = make_float2(a.x + b.x, a.y + b.y);
  v = make_float2(a.x - b.x, a.y - b.y);
}

// Butterflies over register-index bits s < ns; register bit s <-> row bit bit_lo + s.
template <int J, int NS>
__device__ __forceinline__ void reg_fwht2(float2 (&v)[J], int bit_lo, int lb) {
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    if (bit_lo + s < lb) {
#pragma unroll
      for (int j = 0; j < J; ++j)
        if ((j & (1 << s)) == 0) bfly2(v[j], v[j | (1 << s)]);
    }
  }
}

// Transpose slot of (row r, lane c < 4) in float2 units: the row-bit-6..8 XOR
// spreads the 8 row groups a wave reads together over different banks; the rows a
// wave writes together share those bits, so the write stays contiguous.
__device__ __forceinline__ int p2_slot(int r, int c) { return (r * 4 + c) ^ (((r >> 6) & 7) << 2); }

// Pass 2: block (16-column half of a 32-column panel, tile of 2048 rows
// r = qq n1 + i1, i.e. 2048 / n1 consecutive q).  Blocks are dispatched to the 8
// XCDs in turn (block L on XCD L % 8): blocks 16 k + x and 16 k + 8 + x take the
// two halves of the same (panel, tile), work item 8 k + x, so both halves of
// every 128-byte row of Z are read on one XCD at about the same time.
// Thread (g, c) first holds rows g + 32 j (j < 64: row
// bits 5..10 in registers), then after the LDS transpose rows 64 g + j (bits 0..4),
// two columns each.  Row r = (q, r1) of the result goes to SA row kmap[r1 n2 +
// qlist[q]] when that row is sampled, scaled.
// The SA row of every pass-2 tile row (q, r1): kmap[r1 n2 + qlist[q]] for q < Q,
// else -1, stored q-major (q n1 + r1) like the tiles, so pass 2 reads its block's
// destinations as one contiguous run instead of a gather from kmap.
__global__ __launch_bounds__(256) void k_p2_dest(const int32_t* __restrict__ qlist,
                                                 const int32_t* __restrict__ kmap,
                                                 const int32_t* __restrict__ qcount,
                                                 int64_t Qmax, int64_t n1, int64_t n2,
                                                 int32_t* __restrict__ dest2) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;  // q fastest
  if (idx >= Qmax * n1) return;
  const int64_t q = idx % Qmax;
  const int64_t r1 = idx / Qmax;
  int32_t v = -1;
  if (q < (int64_t)*qcount) v = kmap[r1 * n2 + qlist[q]];
  dest2[q * n1 + r1] = v;
}

// DUAL: a second, smaller sketch of the same seed and sketch_id (its rows are a
// subset of this one's) written from the same transformed rows: destination rows
// dest2b (q-major like dest2, -1: not in it), its own output, leading dimension and
// scale.  Both outputs then take their two columns with one store (the host checks
// that each output is aligned for it and has a padding column when d is odd), which
// keeps the kernel's code inside the instruction cache.
struct P2Dual {
  const int32_t* dest2b;
  void* out;
  int64_t ldo;
  float scale;
};

// PST: every output row takes its two columns with one store (the host has checked
// alignment and the padding column); otherwise a row's columns are stored by the
// general path (vector or single stores as alignment and d allow).  DUAL implies PST.
template <typename OutT, bool EDGE, bool DUAL, bool PST>
__global__ __launch_bounds__(256) void k_srht_p2(const float* __restrict__ Z, int64_t Qmax,
                                                 int lb1, int64_t n2, int64_t d,
                                                 const int32_t* __restrict__ dest2,
                                                 const int32_t* __restrict__ qcount,
                                                 OutT* __restrict__ out, int64_t ldo,
                                                 float scale, int64_t ytile0, int64_t np32,
                                                 int64_t ntile, P2Dual du) {
  constexpr int RT = kP2Rows;
  constexpr int J = kP2J;
  __shared__ float2 lds[RT * 4];
  __shared__ int32_t dest[RT];
  const int64_t slot = blockIdx.x >> 3;
  const int64_t item = (slot >> 1) * 8 + (blockIdx.x & 7);
  if (item >= np32 * ntile) return;  // uniform: the grid is rounded up to 16 blocks
  const int64_t p32 = item % np32;
  const int hsel = (int)(slot & 1);
  const int64_t n1 = (int64_t)1 << lb1;
  const int64_t Q = *qcount;
  const int64_t q0 = (ytile0 + item / np32) * (RT >> lb1);
  if (q0 >= Q) return;  // uniform: no sampled low index in this tile
  const int64_t valid = (Q - q0) * n1 < RT ? (Q - q0) * n1 : RT;
  const int t = threadIdx.x;
  const int c = t & 7;
  const int g = t >> 3;
  const int half = c >> 2;
  // rows of q >= Q (whole groups of n1) carry whatever Z holds there: the transform
  // never mixes them with other q and they are not stored, so only the addresses
  // are kept inside this panel's Qmax * n1 rows (EDGE: the tile that reaches past
  // them)
  const float* base = Z + ((p32 * Qmax + q0) * n1 << 5) + 16 * hsel;
  float2 v[J];
  if constexpr (!EDGE) {
    const __amdgpu_buffer_rsrc_t rs = buf_rsrc(base, RT * 128u);
    const uint32_t voff = ((uint32_t)g * 32u + 2u * c) * 4u;
#pragma unroll
    for (int j = 0; j < J; ++j)
      v[j] = __builtin_bit_cast(float2, __builtin_amdgcn_raw_buffer_load_b64(
                                            rs, voff, (uint32_t)j * 32u * 128u, 0));
  } else {
    const int rmax = (int)((Qmax - q0) * n1) - 1;
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int r = g + 32 * j;
      v[j] = *reinterpret_cast<const float2*>(base + ((int64_t)(r < rmax ? r : rmax) << 5) + 2 * c);
    }
  }
  // the SA row of each tile row, loaded behind the tile (one memory round trip)
  static_assert(RT == 8 * 256, "eight tile rows per thread");
  int32_t dv[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int r = t + 256 * u;
    dv[u] = dest2[q0 * n1 + (r < valid ? r : 0)];
  }
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int r = t + 256 * u;
    dest[r] = r < valid ? dv[u] : -1;
  }

  reg_fwht2<J, 6>(v, 5, lb1);
  for (int h = 0; h < 2; ++h) {
    if (half == h) {
#pragma unroll
      for (int j = 0; j < J; ++j) lds[p2_slot(g + 32 * j, c & 3)] = v[j];
    }
    __syncthreads();
    if (half == h) {
#pragma unroll
      for (int j = 0; j < J; ++j) v[j] = lds[p2_slot(64 * g + j, c & 3)];
    }
    __syncthreads();
  }
  reg_fwht2<J, 5>(v, 0, lb1);
  const int64_t col = (2 * p32 + hsel) * 16 + 2 * c;
  if (col >= d) return;
  const bool pair = col + 1 < d;
  constexpr uintptr_t kAlign = sizeof(OutT) == 2 ? 4 : 8;
  // one output row: the two columns scaled, rounded to OutT, stored
  auto put = [&](OutT* base, int64_t ld, int64_t k, float sc, float2 val) {
    const bool vec_ok = pair && ((reinterpret_cast<uintptr_t>(base) |
                                  (uintptr_t)(ld * (int64_t)sizeof(OutT))) & (kAlign - 1)) == 0;
    OutT* o = base + k * ld + col;
    const float a = val.x * sc, b = val.y * sc;
    if constexpr (sizeof(OutT) == 2) {
      if (vec_ok) {
        *reinterpret_cast<uint32_t*>(o) =
            (uint32_t)f32_to_bf16_rne(a) | ((uint32_t)f32_to_bf16_rne(b) << 16);
      } else {
        o[0] = f32_to_bf16_rne(a);
        if (pair) o[1] = f32_to_bf16_rne(b);
      }
    } else {
      if (vec_ok) {
        *reinterpret_cast<float2*>(o) = make_float2(a, b);
      } else {
        o[0] = a;
        if (pair) o[1] = b;
      }
    }
  };
  static_assert(PST || !DUAL, "the dual pass stores paired columns");
  // one store for both columns (alignment and padding checked by the host)
  auto put2 = [&](OutT* base, int64_t ld, int64_t k, float sc, float2 val) {
    OutT* o = base + k * ld + col;
    const float a = val.x * sc, b = val.y * sc;
    if constexpr (sizeof(OutT) == 2)
      *reinterpret_cast<uint32_t*>(o) =
          (uint32_t)f32_to_bf16_rne(a) | ((uint32_t)f32_to_bf16_rne(b) << 16);
    else
      *reinterpret_cast<float2*>(o) = make_float2(a, b);
  };
  if constexpr (!PST) {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int32_t k = dest[64 * g + j];
      if (k >= 0) put(out, ldo, k, scale, v[j]);
    }
  } else {
#pragma unroll
    for (int j = 0; j < J; ++j) {
      const int32_t k = dest[64 * g + j];
      if (k >= 0) put2(out, ldo, k, scale, v[j]);
    }
  }
  if constexpr (DUAL) {
    // the second sketch's rows: destinations read from global memory (the 8 lanes
    // of a row group share each address), no LDS of their own, 16 at a time with
    // 16-byte loads so that one wait covers them (a full tile's 2048 rows lie inside
    // dest2b's Qmax n1 entries; the edge tile reads only rows below valid)
    const int32_t* db = du.dest2b + q0 * n1 + 64 * g;
#pragma unroll
    for (int j0 = 0; j0 < J; j0 += 16) {
      int32_t kb[16];
      if constexpr (!EDGE) {
#pragma unroll
        for (int h = 0; h < 4; ++h) {
          const int4 w4 = *reinterpret_cast<const int4*>(db + j0 + 4 * h);
          kb[4 * h] = w4.x;
          kb[4 * h + 1] = w4.y;
          kb[4 * h + 2] = w4.z;
          kb[4 * h + 3] = w4.w;
        }
      } else {
#pragma unroll
        for (int jj = 0; jj < 16; ++jj) kb[jj] = 64 * g + j0 + jj < valid ? db[j0 + jj] : -1;
      }
#pragma unroll
      for (int jj = 0; jj < 16; ++jj) {
        const int32_t k2 = 64 * g + j0 + jj < valid ? kb[jj] : -1;
        if (k2 >= 0) put2(reinterpret_cast<OutT*>(du.out), du.ldo, k2, du.scale, v[j0 + jj]);
      }
    }
  }
}

size_t srht_zbuf_bytes(rs_dtype a_t, int64_t npad, int64_t d, int64_t Qmax) {
  const int64_t n2 = npad < 1024 ? npad : 1024;
  const int64_t n1 = npad / n2;
  if (n1 <= 1) return 0;
  if (a_t == RS_F32 && n1 <= kP2Rows)  // panel-major, 32-column multiple
    return (size_t)n1 * Qmax * ((d + 31) / 32 * 32) * sizeof(float);
  const int64_t es = a_t == RS_F64 ? 8 : 4;
  const int64_t vec = 16 / es;
  return (size_t)n1 * Qmax * ((d + vec - 1) / vec * vec) * es;
}

// ---------------------------------------------------------------- driver
rs_status srht_select(const SrhtBuffers& B, uint64_t seed, uint32_t sid, int64_t npad, int64_t m,
                      int64_t n2, int64_t* rows, hipStream_t s) {
  const int hist_grid = (int)std::min<int64_t>((npad + 255) / 256, 1024);
  hipLaunchKernelGGL(k_keys_hist, dim3(hist_grid), dim3(256), 0, s, seed, sid, npad, B.hist,
                     B.signs, B.kmap);
  SelectState* st = reinterpret_cast<SelectState*>(B.state);
  hipLaunchKernelGGL(k_select_bin, dim3(1), dim3(1024), 0, s, B.hist, m, st);
  const int nblk = (int)((npad + kCompactBlock - 1) / kCompactBlock);
  hipLaunchKernelGGL(k_collect, dim3(nblk), dim3(256), 0, s, seed, sid, npad, st, B.cand_key,
                     B.cand_idx, B.blk_less);
  // expected boundary-bin population npad / 4096; LDS for 16x that (at least 256,
  // at most 4096 entries = 64 KiB)
  uint32_t cap = 256;
  while ((int64_t)cap < 16 * ((npad + kHistBins - 1) / kHistBins) && cap < 4096u) cap <<= 1;
  hipLaunchKernelGGL(k_cand_sort, dim3(1), dim3(1024), (size_t)cap * 16, s, st, B.cand_key,
                     B.cand_idx, B.blk_less, nblk, cap);
  hipLaunchKernelGGL(k_scatter_rows, dim3(nblk), dim3(256), 0, s, seed, sid, npad, st,
                     B.cand_idx, B.blk_less, rows, B.kmap, B.used, n2 - 1, m);
  hipLaunchKernelGGL(k_qscan, dim3(1), dim3(1024), 0, s, B.used, (int)n2, B.qmap, B.qlist,
                     B.qcount);
  return check_launch("srht select");
}

// The signs of (seed, sid) alone (k_keys_hist writes them with the histogram,
// which must then be consumed by a selection).
__global__ __launch_bounds__(256) void k_signs(uint64_t seed, uint32_t sid, int64_t npad,
                                               int8_t* __restrict__ signs) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < npad;
       i += (int64_t)gridDim.x * blockDim.x)
    signs[i] = (int8_t)sign_of(seed, sid, (uint64_t)i);
}

// Every low index kept, in order: qmap = qlist = identity over n2, qcount = n2.
__global__ __launch_bounds__(1024) void k_iota_q(int32_t* __restrict__ qmap,
                                                 int32_t* __restrict__ qlist,
                                                 int32_t* __restrict__ qcount, int n2) {
  const int i = threadIdx.x;
  if (i < n2) {
    qmap[i] = i;
    qlist[i] = i;
  }
  if (i == 0) *qcount = n2;
}

rs_status srht_pass1_prep(const SrhtBuffers& B, int64_t npad, int64_t lda, uint64_t seed,
                          uint32_t sid, hipStream_t s) {
  if (!srht_panel_path(npad, lda))
    return set_error(RS_ERR_ARG, "srht: the full first pass runs on the panel-major path only");
  const int64_t n2 = npad < 1024 ? npad : 1024;
  const int hist_grid = (int)std::min<int64_t>((npad + 255) / 256, 1024);
  hipLaunchKernelGGL(k_signs, dim3(hist_grid), dim3(256), 0, s, seed, sid, npad, B.signs);
  hipLaunchKernelGGL(k_iota_q, dim3(1), dim3(1024), 0, s, B.qmap, B.qlist, B.qcount, (int)n2);
  return check_launch("srht full first pass set-up");
}

size_t srht_state_bytes() { return sizeof(SelectState); }
int srht_cand_cap() { return kCandCap; }
int srht_compact_block() { return kCompactBlock; }

template <typename T, typename OutT, int MODE>
static void launch_tile(dim3 grid, hipStream_t s, const T* src, int64_t nsrc, int64_t ldsrc,
                        int64_t d, const SrhtBuffers& B, int lb, int64_t n2, int64_t Q, void* out,
                        int64_t ldo, double scale, int hb = 0) {
  if (hb > 0)
    hipLaunchKernelGGL((k_fwht_tile<T, OutT, MODE, true>), grid, dim3(256), 0, s, src, nsrc,
                       ldsrc, d, B.signs, lb, n2, Q, B.qmap, B.qlist, B.kmap, B.qcount,
                       reinterpret_cast<OutT*>(out), ldo, scale, hb);
  else
    hipLaunchKernelGGL((k_fwht_tile<T, OutT, MODE, false>), grid, dim3(256), 0, s, src, nsrc,
                       ldsrc, d, B.signs, lb, n2, Q, B.qmap, B.qlist, B.kmap, B.qcount,
                       reinterpret_cast<OutT*>(out), ldo, scale, hb);
}

bool srht_panel_path(int64_t npad, int64_t lda) {
  const int64_t n2 = npad < 1024 ? npad : 1024;
  const int64_t n1 = npad / n2;
  return n1 > 1 && n1 <= kP2Rows && lda < ((int64_t)1 << 19);
}

// Whether pass 2 may store each row's two columns (col, col + 1; col even) with one
// store into SA: a base aligned to two elements, an even leading dimension, and a
// padding column to take the write past d when d is odd.
static bool pair_store_ok(const void* SA, int64_t ldsa, int64_t d, int es) {
  return (reinterpret_cast<uintptr_t>(SA) % (uintptr_t)(2 * es)) == 0 && ldsa % 2 == 0 &&
         (d % 2 == 0 || ldsa > d);
}

template <typename T>
rs_status srht_transform(const SrhtBuffers& B, const T* A, int64_t n, int64_t d, int64_t lda,
                         int64_t npad, int64_t m, void* SA, rs_dtype sa_t, int64_t ldsa,
                         int64_t Qmax, hipStream_t s, double scale_override,
                         const ProbeArgs* probe, const SrhtDual* dual, const SrhtPre* pre) {
  if (pre && (sizeof(T) != 4 || !srht_panel_path(npad, lda) || probe))
    return set_error(RS_ERR_ARG, "srht: a done first pass rides on the panel-major path only");
  if (probe && (sizeof(T) != 4 || !srht_panel_path(npad, lda)))
    return set_error(RS_ERR_ARG, "srht: the probe sums ride on the panel-major path only");
  if (dual && !(sizeof(T) == 4 && srht_panel_path(npad, lda)))
    return set_error(RS_ERR_ARG, "srht: a second output rides on the panel-major path only");
  if (dual) {
    // the dual pass stores two columns at once in both outputs
    const int es = sa_t == RS_BF16 ? 2 : 4;
    if (!pair_store_ok(SA, ldsa, d, es) || !pair_store_ok(dual->SA2, dual->ldsa2, d, es))
      return set_error(RS_ERR_ARG, "srht: a second output needs paired-column stores");
  }
  using TT = Tile<T>;
  const int64_t n2 = npad < TT::RT ? npad : TT::RT;
  const int64_t n1 = npad / n2;
  int lb2 = 0;
  while (((int64_t)1 << lb2) < n2) ++lb2;
  int lb1 = 0;
  while (((int64_t)1 << lb1) < n1) ++lb1;
  const unsigned panels = (unsigned)((d + TT::W - 1) / TT::W);
  const double scale = scale_override > 0.0 ? scale_override : 1.0 / std::sqrt((double)m);
  const bool bf16 = sa_t == RS_BF16;
  if constexpr (sizeof(T) == 8) {
    if (bf16) return set_error(RS_ERR_UNSUPPORTED, "srht: BF16 output needs FP32 input");
  }
  if (n1 > 4 * TT::RT) return set_error(RS_ERR_SHAPE, "srht: padded n above 2^22 is not supported");
  // pass 2 transforms the low (at most 10) bits of j1 in the tile and folds the rest
  const int lbt = lb1 < 10 ? lb1 : 10;
  const int hb = lb1 - lbt;
  const int64_t n1t = (int64_t)1 << lbt;
  if (n1 == 1) {
    if constexpr (sizeof(T) == 4) {
      if (bf16) {
        launch_tile<T, uint16_t, 1>(dim3(1, panels), s, A, n, lda, d, B, lb2, n2, 0, SA, ldsa, scale);
        return check_launch("srht single pass");
      }
    }
    launch_tile<T, T, 1>(dim3(1, panels), s, A, n, lda, d, B, lb2, n2, 0, SA, ldsa, scale);
    return check_launch("srht single pass");
  }
  // Q (distinct low indices) lives on the device; the intermediate is laid out
  // with the host bound Qmax >= Q and pass 2 reads the device count.
  if constexpr (sizeof(T) == 4) {
    // the panel form addresses a tile of A with 32-bit offsets (1024 rows of lda
    // floats below 2^31 bytes); its intermediate is never smaller than the old
    // layout's, so wider rows fall back to that form in the same buffer
    if (n1 <= kP2Rows && lda < ((int64_t)1 << 19)) {
      // pre: pass 1 already ran with every low index kept (k_srht_p1_two): its
      // intermediate, q = i2 over all n2 low indices
      // (pass 1 writes Zw only without pre; with it pass 2 only reads)
      float* Zw = reinterpret_cast<float*>(pre ? const_cast<void*>(pre->Z) : B.zbuf);
      const int64_t QM = pre ? n2 : Qmax;
      const int32_t* ql = pre ? pre->qlist : B.qlist;
      const int32_t* qc = pre ? pre->qcount : B.qcount;
      const float* Af = reinterpret_cast<const float*>(A);
      // full tiles (all 1024 rows below n), then the rest row-clamped
      const int64_t full = n2 == 1024 ? std::min<int64_t>(n / 1024, n1) : 0;
      const int64_t P = panels;
      const int kP1Group = Qmax >= 512 ? kP1GroupWrite : kP1GroupRead;
      const ProbeArgs pa = probe ? *probe : ProbeArgs{nullptr, nullptr, nullptr, 0};
      auto p1 = [&](auto edge, auto withp, int64_t t0, int64_t nt) {
        constexpr bool E = decltype(edge)::value, PR = decltype(withp)::value;
        if constexpr (PR) {
          if (pa.Z2) {  // the second transform writes an intermediate as large as A
            hipLaunchKernelGGL((k_srht_p1_two<E>), dim3((unsigned)(P * nt)), dim3(256), 0, s,
                               Af, n, d, lda, B.signs, lb2, n2, n1, Qmax, B.qmap, Zw, t0, nt, P,
                               kP1GroupWrite, pa);
            return;
          }
        }
        hipLaunchKernelGGL((k_srht_p1<E, PR>), dim3((unsigned)(P * nt)), dim3(256), 0, s, Af, n,
                           d, lda, B.signs, lb2, n2, n1, Qmax, B.qmap, Zw, t0, nt, P, kP1Group,
                           pa);
      };
      using F_ = std::false_type;
      using T_ = std::true_type;
      if (full > 0 && !pre) {
        if (probe) p1(F_{}, T_{}, (int64_t)0, full);
        else p1(F_{}, F_{}, (int64_t)0, full);
      }
      if (full < n1 && !pre) {
        if (probe) p1(T_{}, T_{}, full, n1 - full);
        else p1(T_{}, F_{}, full, n1 - full);
      }
      if (probe && pa.p1_done) {
        const hipError_t e = hipEventRecord(pa.p1_done, s);
        if (e != hipSuccess) return set_error(RS_ERR_HIP, hipGetErrorString(e));
      }
      hipLaunchKernelGGL(k_p2_dest, dim3((unsigned)((QM * n1 + 255) / 256)), dim3(256), 0, s,
                         ql, B.kmap, qc, QM, n1, n2, B.dest2);
      // the second sketch's rows among this one's transformed rows (its low indices
      // are among this selection's, so this Z holds them all)
      if (dual)
        hipLaunchKernelGGL(k_p2_dest, dim3((unsigned)((QM * n1 + 255) / 256)), dim3(256), 0,
                           s, ql, dual->kmap2, qc, QM, n1, n2, dual->dest2b);
      const P2Dual du = dual ? P2Dual{dual->dest2b, dual->SA2, dual->ldsa2, (float)dual->scale2}
                             : P2Dual{nullptr, nullptr, 0, 0.0f};
      const int64_t t2 = (QM * n1 + kP2Rows - 1) / kP2Rows;  // tiles of 2048 rows
      const int64_t t2full = QM * n1 / kP2Rows;
      const float* Z = Zw;
      // two blocks (the halves of a 32-column panel) per work item, 16 blocks per
      // 8 work items (see k_srht_p2)
      auto p2_grid = [&](int64_t ntile) {
        return dim3((unsigned)((P * ntile + 7) / 8 * 16));
      };
      auto p2 = [&](auto out_tag, auto dual_tag, auto pst_tag) {
        using OutT = decltype(out_tag);
        constexpr bool DU = decltype(dual_tag)::value, PS = decltype(pst_tag)::value;
        OutT* o = reinterpret_cast<OutT*>(SA);
        if (t2full > 0)
          hipLaunchKernelGGL((k_srht_p2<OutT, false, DU, PS>), p2_grid(t2full), dim3(256), 0, s,
                             Z, QM, lb1, n2, d, B.dest2, qc, o, ldsa, (float)scale,
                             (int64_t)0, P, t2full, du);
        if (t2 > t2full)
          hipLaunchKernelGGL((k_srht_p2<OutT, true, DU, PS>), p2_grid(1), dim3(256), 0, s, Z,
                             QM, lb1, n2, d, B.dest2, qc, o, ldsa, (float)scale, t2full,
                             P, (int64_t)1, du);
      };
      using F_ = std::false_type;
      using T_ = std::true_type;
      const bool pst = pair_store_ok(SA, ldsa, d, bf16 ? 2 : 4);
      if (bf16) {
        if (dual) p2(uint16_t{}, T_{}, T_{});
        else if (pst) p2(uint16_t{}, F_{}, T_{});
        else p2(uint16_t{}, F_{}, F_{});
      } else {
        if (dual) p2(float{}, T_{}, T_{});
        else if (pst) p2(float{}, F_{}, T_{});
        else p2(float{}, F_{}, F_{});
      }
      return check_launch("srht two pass");
    }
  }
  const int64_t ldz = ((d + TT::VEC - 1) / TT::VEC) * TT::VEC;
  launch_tile<T, T, 0>(dim3((unsigned)n1, panels), s, A, n, lda, d, B, lb2, n2, Qmax, B.zbuf, ldz,
                       1.0);
  const int64_t tiles2 = (Qmax * n1t + TT::RT - 1) / TT::RT;
  const T* Z = reinterpret_cast<const T*>(B.zbuf);
  const dim3 grid2((unsigned)tiles2, panels, 1u << hb);
  if constexpr (sizeof(T) == 4) {
    if (bf16) {
      launch_tile<T, uint16_t, 2>(grid2, s, Z, n1 * Qmax, ldz, d, B, lbt, n2, Qmax, SA, ldsa,
                                  scale, hb);
      return check_launch("srht two pass");
    }
  }
  launch_tile<T, T, 2>(grid2, s, Z, n1 * Qmax, ldz, d, B, lbt, n2, Qmax, SA, ldsa, scale, hb);
  return check_launch("srht two pass");
}

template rs_status srht_transform<float>(const SrhtBuffers&, const float*, int64_t, int64_t,
                                         int64_t, int64_t, int64_t, void*, rs_dtype, int64_t,
                                         int64_t, hipStream_t, double, const ProbeArgs*,
                                         const SrhtDual*, const SrhtPre*);
template rs_status srht_transform<double>(const SrhtBuffers&, const double*, int64_t, int64_t,
                                          int64_t, int64_t, int64_t, void*, rs_dtype, int64_t,
                                          int64_t, hipStream_t, double, const ProbeArgs*,
                                          const SrhtDual*, const SrhtPre*);

// ---------------------------------------------------------------- nested gather
// SA[k] = scale * HDA[rows[k]] for the cached transform of the whole padded A
// (nested resampling keeps signs and keys, so every level's rows index the same
// H D A).  One block per row; the product and rounding are those of the direct
// transform's output stage.
template <typename T, typename OutT>
__global__ __launch_bounds__(256) void k_gather_rows(const T* __restrict__ H, int64_t ldh,
                                                     const int64_t* __restrict__ rows,
                                                     int64_t d, double scale,
                                                     OutT* __restrict__ SA, int64_t ldsa) {
  const int64_t k = blockIdx.x;
  const T* src = H + rows[k] * ldh;
  OutT* dst = SA + k * ldsa;
  for (int64_t c = threadIdx.x; c < d; c += 256) {
    if constexpr (sizeof(OutT) == 2)
      dst[c] = f32_to_bf16_rne((float)src[c] * (float)scale);
    else
      dst[c] = (OutT)(src[c] * (T)scale);
  }
}

rs_status srht_gather(const void* H, rs_dtype h_t, int64_t ldh, const int64_t* rows, int64_t m,
                      int64_t d, double scale, void* SA, rs_dtype sa_t, int64_t ldsa,
                      hipStream_t s) {
  const dim3 g((unsigned)m);
  if (h_t == RS_F64) {
    if (sa_t != RS_F64) return set_error(RS_ERR_UNSUPPORTED, "gather: F64 data needs F64 SA");
    hipLaunchKernelGGL((k_gather_rows<double, double>), g, dim3(256), 0, s,
                       reinterpret_cast<const double*>(H), ldh, rows, d, scale,
                       reinterpret_cast<double*>(SA), ldsa);
  } else if (sa_t == RS_BF16) {
    hipLaunchKernelGGL((k_gather_rows<float, uint16_t>), g, dim3(256), 0, s,
                       reinterpret_cast<const float*>(H), ldh, rows, d, scale,
                       reinterpret_cast<uint16_t*>(SA), ldsa);
  } else if (sa_t == RS_F32) {
    hipLaunchKernelGGL((k_gather_rows<float, float>), g, dim3(256), 0, s,
                       reinterpret_cast<const float*>(H), ldh, rows, d, scale,
                       reinterpret_cast<float*>(SA), ldsa);
  } else {
    return set_error(RS_ERR_UNSUPPORTED, "gather: SA dtype not supported");
  }
  return check_launch("srht gather");
}

}  // namespace rs
