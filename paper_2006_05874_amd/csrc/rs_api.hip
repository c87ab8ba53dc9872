// C ABI of librs: argument checks, per-device scratch, and the host side of the
// adaptive controller (Algorithm 1).  Every numeric step runs in the kernels.
#include <array>
#include <atomic>
#include <cstdio>
#include <cstring>
#include <iterator>
#include <memory>
#include <mutex>
#include <string>
#include <condition_variable>
#include <functional>
#include <thread>
#include <vector>

#include "rs_internal.hpp"

namespace rs {

static thread_local std::string g_err;

rs_status set_error(rs_status st, const char* msg) {
  g_err = msg ? msg : "";
  return st;
}

rs_status check_launch(const char* what) {
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    g_err = std::string(what) + ": " + hipGetErrorString(e);
    return RS_ERR_HIP;
  }
  return RS_OK;
}

#define RS_HIP(call)                                                                \
  do {                                                                              \
    hipError_t e_ = (call);                                                         \
    if (e_ != hipSuccess) {                                                         \
      g_err = std::string(#call) + ": " + hipGetErrorString(e_);                    \
      return e_ == hipErrorOutOfMemory ? RS_ERR_OOM : RS_ERR_HIP;                   \
    }                                                                               \
  } while (0)

#define RS_TRY(expr)                   \
  do {                                 \
    rs_status st_ = (expr);            \
    if (st_ != RS_OK) return st_;      \
  } while (0)

int device_cus() {
  static std::atomic<int> cus[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cus[dev] == 0) {
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
      v = 256;
    cus[dev] = v;
  }
  return cus[dev];
}

// ------------------------------------------------------------------ timing
// Launches bracketed while profiling: event pairs plus a device flag per launch
// that the kernel sets when it does its work (launches queued behind a raised
// status flag return at once and are not counted).
// Worker threads of a batch launch concurrently: the slot counter and the event
// list are guarded by g_prof_mu, and each launch keeps its own slot.  The events
// are updated by the profiled launch itself with the kernel's start and stop.
static std::mutex g_prof_mu;
static std::atomic<bool> g_prof_on{false};
static std::vector<hipEvent_t> g_prof_ev;  // begin/end pairs
static size_t g_prof_pairs = 0;            // launches bracketed
static int* g_prof_ran = nullptr;          // device flags, one per launch
static constexpr size_t kProfCap = 1 << 16;

ProfSlot prof_begin() {
  ProfSlot ps;
  if (!g_prof_on.load(std::memory_order_relaxed)) return ps;
  std::lock_guard<std::mutex> g(g_prof_mu);
  if (!g_prof_on || g_prof_pairs >= kProfCap) return ps;
  while (g_prof_ev.size() < 2 * (g_prof_pairs + 1)) {
    hipEvent_t ne;
    if (hipEventCreate(&ne) != hipSuccess) return ps;
    g_prof_ev.push_back(ne);
  }
  ps.slot = (int64_t)g_prof_pairs++;
  ps.begin = g_prof_ev[2 * ps.slot];
  ps.end = g_prof_ev[2 * ps.slot + 1];
  ps.ran = g_prof_ran ? g_prof_ran + ps.slot : nullptr;
  return ps;
}

// ------------------------------------------------------------------ scratch
// While a batch runs, its worker threads do not free device memory: hipFree
// synchronizes the whole device, stalling every other worker's stream, and it
// would run concurrently with the other workers' launches.  A buffer that must
// grow on a worker thread hands its old block to the thread's retire list (set by
// the batch for the worker's lifetime in the call); the calling thread frees them
// after every worker has finished and its stream is synchronized.  Growth on such
// a thread is at least 1.5x, so a worker retires few blocks per batch.
static thread_local std::vector<void*>* t_retire = nullptr;

static void release_block(void* p) {
  if (!p) return;
  if (t_retire)
    t_retire->push_back(p);
  else
    (void)hipFree(p);
}

struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  // grow-only
  rs_status ensure(size_t want) {
    if (want <= bytes && p) return RS_OK;
    size_t sz = want ? want : 256;
    if (t_retire && p) sz = std::max(sz, bytes + bytes / 2);
    if (p) {
      release_block(p);
      p = nullptr;
      bytes = 0;
    }
    hipError_t e = hipMalloc(&p, sz);
    if (e != hipSuccess) {
      p = nullptr;
      g_err = std::string("hipMalloc: ") + hipGetErrorString(e);
      return e == hipErrorOutOfMemory ? RS_ERR_OOM : RS_ERR_HIP;
    }
    bytes = sz;
    return RS_OK;
  }
  // grow-only; fresh memory is zero-filled on stream s, the stream whose kernels
  // read it (a plain hipMemset runs on the null stream, which the library's
  // non-blocking streams do not wait for: their kernels could read the block
  // before the fill lands)
  rs_status ensure_zeroed(size_t want, hipStream_t s) {
    if (want <= bytes && p) return RS_OK;
    RS_TRY(ensure(want));
    RS_HIP(hipMemsetAsync(p, 0, bytes, s));
    return RS_OK;
  }
  // grow-only, keeping the first `keep` bytes (copied on the stream, which is
  // synchronized before the old block is released)
  rs_status grow_keep(size_t want, size_t keep, hipStream_t s) {
    if (want <= bytes && p) return RS_OK;
    void* np = nullptr;
    hipError_t e = hipMalloc(&np, want);
    if (e != hipSuccess) {
      g_err = std::string("hipMalloc: ") + hipGetErrorString(e);
      return e == hipErrorOutOfMemory ? RS_ERR_OOM : RS_ERR_HIP;
    }
    if (p && keep) {
      e = hipMemcpyAsync(np, p, keep, hipMemcpyDeviceToDevice, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) {
        (void)hipFree(np);
        return set_error(RS_ERR_HIP, "grow_keep: copy failed");
      }
    }
    release_block(p);
    p = np;
    bytes = want;
    return RS_OK;
  }
  template <typename T>
  T* as() const {
    return reinterpret_cast<T*>(p);
  }
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() {
    if (p) (void)hipFree(p);
  }
};

// the solvers apply H_S^-1 through Cw = L^-1 SA (m < d) only above this width
constexpr int64_t kWoodburyApplyMinD = 2048;

struct DeviceScratch {
  std::mutex mu;
  // SRHT
  DevBuf hist, signs, kmap, state, cand_key, cand_idx, blk_less, used, qmap, qlist, qcount, zbuf, rows,
      dest2;
  // a second, smaller sketch formed by the same transform (srht_run's dual output):
  // its own selection's row map and low-index lists, and its pass-2 destinations
  DevBuf kmap2, qmap2, qlist2, qcount2, rows2, dest2b;
  // identity low-index lists of a full first pass run ahead of its selection
  // (srht_pretransform): qmap, qlist (1024 each) and the count
  DevBuf qid;
  // gradient partials, vectors, control
  DevBuf partial, vecs, rpart, ctl, ev, info, rvec;
  // solver-owned sketch and factor (wbuf: scratch of the Woodbury-form apply)
  DevBuf sa, fM, fLinv, fHinv, fCw, fGram, wbuf;
  // FP8 staging: FP32 sketch, column maxima, per-column scales
  DevBuf sa_tmp, colmax, sa_scale;
  // nested resampling: H D A of the whole padded A, and the unscaled Gaussian rows
  DevBuf hda, graw;
  // split partial products of the Gaussian sketch
  DevBuf gpart;
  // dual problem: the data matrix A^T, a zero right-hand side, b in FP64
  DevBuf dM, dzero, dc;
  // sparse A: its column-major copy, the gradient's residuals, the sketch's sort
  SparseWork spw;
  // learned form: probe sketch and its factor, probe sums, features
  DevBuf psa, pM, pLinv, pHinv, pCw, pGram, pinfo, ppart, pU, pY, prp, pr, pfeat, py, pbits;
  // nu grid: per-slot state, candidate blocks, multi-RHS products, batched
  // factors, uploads, and the per-level sketch / Gram cache
  DevBuf g_vec, g_ctl, g_ev, g_hinv, g_rpart, g_xc, g_gc, g_gtc, g_nu2, g_up, g_R, g_Gp, g_M, g_L,
      g_Cw, g_xt;
  std::vector<std::unique_ptr<DevBuf>> lv_sa, lv_scale, lv_gram;
  void* g_pinned = nullptr;
  size_t g_pinned_bytes = 0;
  void* host_pinned = nullptr;
  hipEvent_t done_ev = nullptr;
  // side stream (default priority) for work that runs beside the caller's stream
  hipStream_t aux = nullptr;
  hipEvent_t fork_ev = nullptr, join_ev = nullptr;
  DeviceScratch() = default;
  ~DeviceScratch() {
    if (g_pinned) (void)hipHostFree(g_pinned);
    if (host_pinned) (void)hipHostFree(host_pinned);
    if (done_ev) (void)hipEventDestroy(done_ev);
    if (fork_ev) (void)hipEventDestroy(fork_ev);
    if (join_ev) (void)hipEventDestroy(join_ev);
    if (aux) (void)hipStreamDestroy(aux);
  }
  rs_status ensure_aux() {
    if (!aux) RS_HIP(hipStreamCreateWithFlags(&aux, hipStreamNonBlocking));
    if (!fork_ev) RS_HIP(hipEventCreateWithFlags(&fork_ev, hipEventDisableTiming));
    if (!join_ev) RS_HIP(hipEventCreateWithFlags(&join_ev, hipEventDisableTiming));
    return RS_OK;
  }
};

static DeviceScratch* scratch_for_current() {
  static std::mutex mu;
  static std::vector<DeviceScratch*> all;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  std::lock_guard<std::mutex> g(mu);
  if ((int)all.size() <= dev) all.resize(dev + 1, nullptr);
  if (!all[dev]) {
    all[dev] = new DeviceScratch();
    // the side stream of single solves is created with the scratch, before any
    // batch creates its worker streams: streams share the device's few hardware
    // queues in creation order, and a side stream created later can land on the
    // caller's queue, which serializes the work meant to overlap
    (void)all[dev]->ensure_aux();
  }
  return all[dev];
}

// Worker streams (default priority) with private scratch for batched solves.  A
// worker past the first also keeps a host thread of its own (started on first use,
// current device set once), which runs the tasks a batch hands it; the pool is never
// destroyed, so its threads wait for work until the process ends.
struct BatchWorker {
  DeviceScratch S;
  hipStream_t s = nullptr;
  hipEvent_t join = nullptr;
  hipEvent_t step_ev = nullptr;  // a pair's shared steps (drive_pair)
  std::thread th;
  std::mutex m;
  std::condition_variable cv;
  std::function<void()> task;  // set by the batch, cleared by the thread when done
  bool started = false;

  // start the thread if needed; false if it cannot be started
  bool ensure_thread(int dev) {
    if (started) return true;
    try {
      th = std::thread([this, dev] {
        (void)hipSetDevice(dev);
        std::unique_lock<std::mutex> lk(m);
        for (;;) {
          cv.wait(lk, [this] { return (bool)task; });
          std::function<void()> f = task;  // task stays set until f has run
          lk.unlock();
          f();
          lk.lock();
          task = nullptr;
          cv.notify_all();
        }
      });
    } catch (...) {
      return false;
    }
    th.detach();
    started = true;
    return true;
  }
  void post(std::function<void()> f) {
    std::lock_guard<std::mutex> g(m);
    task = std::move(f);
    cv.notify_all();
  }
  void wait_idle() {
    std::unique_lock<std::mutex> lk(m);
    cv.wait(lk, [this] { return !task; });
  }
};
struct WorkerPool {
  std::mutex mu;
  std::vector<std::unique_ptr<BatchWorker>> w;
  hipEvent_t entry = nullptr;
};

static WorkerPool* pool_for_current() {
  static std::mutex mu;
  static std::vector<WorkerPool*> all;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) dev = 0;
  std::lock_guard<std::mutex> g(mu);
  if ((int)all.size() <= dev) all.resize(dev + 1, nullptr);
  if (!all[dev]) all[dev] = new WorkerPool();
  return all[dev];
}

static int64_t next_pow2(int64_t n) {
  int64_t p = 1;
  while (p < n) p <<= 1;
  return p;
}

static size_t dtype_size(rs_dtype t) {
  switch (t) {
    case RS_F64: return 8;
    case RS_F32: return 4;
    case RS_BF16: return 2;
    case RS_FP8E4M3: return 1;
  }
  return 0;
}

static rs_status check_matrix(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda,
                              const char* who) {
  if (!A) return set_error(RS_ERR_ARG, (std::string(who) + ": A is null").c_str());
  if (a_t != RS_F32 && a_t != RS_F64)
    return set_error(RS_ERR_ARG, (std::string(who) + ": A must be F32 or F64").c_str());
  if (n < 1 || d < 1) return set_error(RS_ERR_SHAPE, (std::string(who) + ": empty matrix").c_str());
  const int64_t vec = 16 / (int64_t)dtype_size(a_t);
  if (lda < d || lda % vec != 0)
    return set_error(RS_ERR_ARG,
                     (std::string(who) + ": lda must be >= d and a multiple of 16 bytes").c_str());
  if (reinterpret_cast<uintptr_t>(A) % 16 != 0)
    return set_error(RS_ERR_ARG, (std::string(who) + ": A must be 16-byte aligned").c_str());
  return RS_OK;
}

// hist and used must be zero on entry to the selection (its kernels leave them
// zero): fresh blocks are cleared on s, the selection's stream
static rs_status ensure_srht(DeviceScratch& S, int64_t npad, int64_t zbytes, SrhtBuffers& B,
                             hipStream_t s) {
  RS_TRY(S.hist.ensure_zeroed(4096 * sizeof(uint32_t), s));
  RS_TRY(S.signs.ensure((size_t)npad));
  RS_TRY(S.kmap.ensure((size_t)npad * sizeof(int32_t)));
  RS_TRY(S.state.ensure(srht_state_bytes()));
  RS_TRY(S.cand_key.ensure((size_t)srht_cand_cap() * sizeof(uint64_t)));
  RS_TRY(S.cand_idx.ensure((size_t)srht_cand_cap() * sizeof(int64_t)));
  RS_TRY(S.blk_less.ensure((size_t)((npad + srht_compact_block() - 1) / srht_compact_block()) *
                           sizeof(uint32_t)));
  RS_TRY(S.used.ensure_zeroed(1024 * sizeof(int32_t), s));
  RS_TRY(S.qmap.ensure(1024 * sizeof(int32_t)));
  RS_TRY(S.qlist.ensure(1024 * sizeof(int32_t)));
  RS_TRY(S.qcount.ensure(sizeof(int32_t)));
  RS_TRY(S.zbuf.ensure((size_t)std::max<int64_t>(zbytes, 256)));
  RS_TRY(S.dest2.ensure((size_t)npad * sizeof(int32_t)));
  B = SrhtBuffers{S.hist.as<uint32_t>(), S.signs.as<int8_t>(),   S.kmap.as<int32_t>(),
                  S.state.p,             S.cand_key.as<uint64_t>(), S.cand_idx.as<int64_t>(),
                  S.blk_less.as<uint32_t>(), S.used.as<int32_t>(), S.qmap.as<int32_t>(),
                  S.qlist.as<int32_t>(), S.qcount.as<int32_t>(), S.zbuf.p, S.dest2.as<int32_t>()};
  return RS_OK;
}

// SRHT into SA (no argument checks).
// A second SRHT of the same seed and sketch_id with m2 <= m rows (its rows are
// among this one's) written by the same transform: SA2 (ldsa2, the dtype of SA).
struct SrhtSecond {
  int64_t m2;
  void* SA2;
  int64_t ldsa2;
  const SrhtPre* pre = nullptr;  // pass 1 already run with every low index kept
};

// Whether srht_run can carry a SrhtSecond for this problem and sketch dtype.
static bool srht_second_ok(rs_dtype a_t, int64_t n, int64_t lda, rs_dtype sa_t) {
  return a_t == RS_F32 && (sa_t == RS_F32 || sa_t == RS_BF16) &&
         srht_panel_path(next_pow2(n), lda);
}

static rs_status srht_run(DeviceScratch& S, const void* A, rs_dtype a_t, int64_t n, int64_t d,
                          int64_t lda, int64_t m, uint64_t seed, uint32_t sid, void* SA,
                          rs_dtype sa_t, int64_t ldsa, float* scale_out, int64_t* rows_out,
                          int8_t* signs_out, hipStream_t s, const ProbeArgs* probe = nullptr,
                          const SrhtSecond* second = nullptr) {
  const int64_t npad = next_pow2(n);
  const int64_t n2 = std::min<int64_t>(npad, 1024);
  const int64_t Qmax = std::min<int64_t>(m, n2);
  const size_t zbytes = srht_zbuf_bytes(a_t, npad, d, Qmax);
  SrhtBuffers B;
  RS_TRY(ensure_srht(S, npad, zbytes, B, s));
  int64_t* rows = rows_out;
  if (!rows) {
    RS_TRY(S.rows.ensure((size_t)m * sizeof(int64_t)));
    rows = S.rows.as<int64_t>();
  }
  SrhtDual dual{};
  if (second) {
    if (!srht_second_ok(a_t, n, lda, sa_t) || second->m2 < 1 || second->m2 > m)
      return set_error(RS_ERR_ARG, "srht: no second output for this shape");
    // the second sketch's own selection first (its row map and low-index lists in
    // buffers of their own; the shared histogram and flags are left zero), then
    // this one's, whose lists the transform uses
    RS_TRY(S.kmap2.ensure((size_t)npad * sizeof(int32_t)));
    RS_TRY(S.qmap2.ensure(1024 * sizeof(int32_t)));
    RS_TRY(S.qlist2.ensure(1024 * sizeof(int32_t)));
    RS_TRY(S.qcount2.ensure(sizeof(int32_t)));
    RS_TRY(S.rows2.ensure((size_t)second->m2 * sizeof(int64_t)));
    RS_TRY(S.dest2b.ensure((size_t)(second->pre ? n2 : Qmax) * (npad / n2) * sizeof(int32_t)));
    SrhtBuffers B2 = B;
    B2.kmap = S.kmap2.as<int32_t>();
    B2.qmap = S.qmap2.as<int32_t>();
    B2.qlist = S.qlist2.as<int32_t>();
    B2.qcount = S.qcount2.as<int32_t>();
    RS_TRY(srht_select(B2, seed, sid, npad, second->m2, n2, S.rows2.as<int64_t>(), s));
    dual = SrhtDual{S.kmap2.as<int32_t>(), S.dest2b.as<int32_t>(), second->SA2, second->ldsa2,
                    1.0 / std::sqrt((double)second->m2)};
  }
  RS_TRY(srht_select(B, seed, sid, npad, m, n2, rows, s));
  if (a_t == RS_F32 && sa_t == RS_FP8E4M3) {
    RS_TRY(S.sa_tmp.ensure((size_t)m * d * sizeof(float)));
    RS_TRY(S.colmax.ensure((size_t)d * sizeof(uint32_t)));
    RS_TRY(srht_transform<float>(B, reinterpret_cast<const float*>(A), n, d, lda, npad, m,
                                 S.sa_tmp.p, RS_F32, d, Qmax, s));
    RS_TRY(quantize_fp8(S.sa_tmp.as<float>(), m, d, d, S.colmax.as<uint32_t>(), scale_out,
                        reinterpret_cast<uint8_t*>(SA), ldsa, s));
  } else if (a_t == RS_F32)
    RS_TRY(srht_transform<float>(B, reinterpret_cast<const float*>(A), n, d, lda, npad, m, SA, sa_t,
                                 ldsa, Qmax, s, 0.0, probe, second ? &dual : nullptr,
                                 second ? second->pre : nullptr));
  else
    RS_TRY(srht_transform<double>(B, reinterpret_cast<const double*>(A), n, d, lda, npad, m, SA,
                                  sa_t, ldsa, Qmax, s));
  if (signs_out) RS_HIP(hipMemcpyAsync(signs_out, B.signs, (size_t)npad, hipMemcpyDeviceToDevice, s));
  return RS_OK;
}

// Set-up of the SRHT of (seed, sid) whose first pass, with every low index kept,
// rides in another job's probe sketch pass (ProbeArgs::signs2 / Z2, *two): its
// signs and identity lists in S, on stream s; *pre then describes the intermediate
// for srht_run (a pair's first sketches: that pass needs only A and the signs, so it
// shares the learned features' read of A).
static rs_status srht_pretransform(DeviceScratch& S, rs_dtype a_t, int64_t n, int64_t d,
                                   int64_t lda, uint64_t seed, uint32_t sid, hipStream_t s,
                                   SrhtPre* pre, ProbeArgs* two) {
  const int64_t npad = next_pow2(n);
  const int64_t n2 = std::min<int64_t>(npad, 1024);
  if (a_t != RS_F32 || !srht_panel_path(npad, lda))
    return set_error(RS_ERR_ARG, "srht: no full first pass for this shape");
  SrhtBuffers B;
  RS_TRY(ensure_srht(S, npad, (int64_t)srht_zbuf_bytes(a_t, npad, d, n2), B, s));
  RS_TRY(S.qid.ensure((2 * 1024 + 1) * sizeof(int32_t)));
  B.qmap = S.qid.as<int32_t>();
  B.qlist = B.qmap + 1024;
  B.qcount = B.qmap + 2048;
  RS_TRY(srht_pass1_prep(B, npad, lda, seed, sid, s));
  *pre = SrhtPre{S.zbuf.p, B.qlist, B.qcount};
  two->signs2 = B.signs;
  two->Z2 = reinterpret_cast<float*>(S.zbuf.p);
  return RS_OK;
}

static rs_status check_sa_type(rs_dtype a_t, rs_dtype sa_t) {
  if (a_t == RS_F64 && sa_t != RS_F64) return set_error(RS_ERR_UNSUPPORTED, "F64 A needs F64 SA");
  if (a_t == RS_F32 && !(sa_t == RS_F32 || sa_t == RS_BF16 || sa_t == RS_FP8E4M3))
    return set_error(RS_ERR_UNSUPPORTED, "F32 A supports F32, BF16 or FP8E4M3 SA");
  return RS_OK;
}

// Gaussian sketch into SA (no argument checks); FP8 goes through an FP32 stage.
static rs_status gauss_run(DeviceScratch& S, const void* A, rs_dtype a_t, int64_t n, int64_t d,
                           int64_t lda, int64_t m, uint64_t seed, uint32_t sid, void* SA,
                           rs_dtype sa_t, int64_t ldsa, float* scale_out, hipStream_t s) {
  RS_TRY(S.gpart.ensure(std::max<size_t>(gauss_split_bytes(n, d, m, a_t), 256)));
  if (sa_t != RS_FP8E4M3)
    return gauss_launch(A, a_t, n, d, lda, m, seed, sid, SA, sa_t, ldsa, s, 0, 0.0, S.gpart.p,
                        S.gpart.bytes);
  RS_TRY(S.sa_tmp.ensure((size_t)m * d * sizeof(float)));
  RS_TRY(S.colmax.ensure((size_t)d * sizeof(uint32_t)));
  RS_TRY(gauss_launch(A, a_t, n, d, lda, m, seed, sid, S.sa_tmp.p, RS_F32, d, s, 0, 0.0,
                      S.gpart.p, S.gpart.bytes));
  return quantize_fp8(S.sa_tmp.as<float>(), m, d, d, S.colmax.as<uint32_t>(), scale_out,
                      reinterpret_cast<uint8_t*>(SA), ldsa, s);
}

// Nested resampling keeps the sketch's randomness from level to level: the
// SRHT's signs and keys (so H D A is computed once, at the first level, and every
// level gathers its sampled rows from it) and the Gaussian's rows (each level
// computes only its new rows, unscaled, and scales all of them by 1/sqrt(m)).
// The values are those of the direct sketch: the same products and roundings.
struct NestedCache {
  bool hda_ready = false;
  int64_t graw_rows = 0;
  // a path's solves share the scratch: the sketch of size gram_m and its split
  // Gram partials are still in it (0: none)
  int64_t gram_m = 0;
};

static rs_status nested_sketch(DeviceScratch& S, NestedCache& C, bool srht, const void* A,
                               rs_dtype a_t, int64_t n, int64_t d, int64_t lda, int64_t m,
                               uint64_t seed, uint32_t sid, void* SA, rs_dtype sa_t,
                               int64_t ldsa, float* scale_out, hipStream_t s) {
  const int64_t es = (int64_t)dtype_size(a_t);
  void* dst = SA;
  rs_dtype dst_t = sa_t;
  int64_t ldd = ldsa;
  if (sa_t == RS_FP8E4M3) {  // through an FP32 stage and the per-column quantizer
    RS_TRY(S.sa_tmp.ensure((size_t)m * d * sizeof(float)));
    RS_TRY(S.colmax.ensure((size_t)d * sizeof(uint32_t)));
    dst = S.sa_tmp.p;
    dst_t = RS_F32;
    ldd = d;
  }
  const double scale = 1.0 / std::sqrt((double)m);
  if (srht) {
    const int64_t npad = next_pow2(n);
    const int64_t n2 = std::min<int64_t>(npad, 1024);
    const int64_t vec = 16 / es;
    const int64_t ldh = (d + vec - 1) / vec * vec;
    SrhtBuffers B;
    RS_TRY(S.rows.ensure((size_t)npad * sizeof(int64_t)));
    if (!C.hda_ready) {
      RS_TRY(ensure_srht(S, npad, (int64_t)srht_zbuf_bytes(a_t, npad, d, n2), B, s));
      RS_TRY(S.hda.ensure((size_t)npad * ldh * es));
      RS_TRY(srht_select(B, seed, sid, npad, npad, n2, S.rows.as<int64_t>(), s));
      if (a_t == RS_F32)
        RS_TRY(srht_transform<float>(B, reinterpret_cast<const float*>(A), n, d, lda, npad, npad,
                                     S.hda.p, RS_F32, ldh, n2, s, 1.0));
      else
        RS_TRY(srht_transform<double>(B, reinterpret_cast<const double*>(A), n, d, lda, npad,
                                      npad, S.hda.p, RS_F64, ldh, n2, s, 1.0));
      C.hda_ready = true;
    } else {
      RS_TRY(ensure_srht(S, npad, 0, B, s));
    }
    RS_TRY(srht_select(B, seed, sid, npad, m, n2, S.rows.as<int64_t>(), s));
    RS_TRY(srht_gather(S.hda.p, a_t, ldh, S.rows.as<int64_t>(), m, d, scale, dst, dst_t, ldd, s));
  } else {
    if (m > C.graw_rows) {
      RS_TRY(S.graw.grow_keep((size_t)m * d * es, (size_t)C.graw_rows * d * es, s));
      RS_TRY(S.gpart.ensure(std::max<size_t>(gauss_split_bytes(n, d, m - C.graw_rows, a_t), 256)));
      RS_TRY(gauss_launch(A, a_t, n, d, lda, m, seed, sid, S.graw.p, a_t, d, s, C.graw_rows,
                          1.0, S.gpart.p, S.gpart.bytes));
      C.graw_rows = m;
    }
    RS_TRY(gauss_scale_rows(S.graw.p, a_t, m, d, scale, dst, dst_t, ldd, s));
  }
  if (sa_t == RS_FP8E4M3)
    return quantize_fp8(S.sa_tmp.as<float>(), m, d, d, S.colmax.as<uint32_t>(), scale_out,
                        reinterpret_cast<uint8_t*>(SA), ldsa, s);
  return RS_OK;
}

}  // namespace rs

using namespace rs;

// ==================================================================== ABI
struct rs_factor {
  int64_t m, d, p, pp, dp;
  double nu2;
  bool wood;  // m < d: applied through Cw = L^-1 SA, no d x d inverse
  DevBuf M, Linv, Hinv, Cw, info, rpart, gram, wbuf;
  rs_dtype sa_t;
};

// gtilde = H_S^-1 G of a factor handle (either route), partial sums into rpart
// (apply_blocks(d) blocks).
static rs_status factor_apply_any(const rs_factor* F, const double* G, int k, double* GT,
                                  double* rpart, const int* status, hipStream_t s) {
  if (F->wood)
    return wapply_launch(F->Cw.as<double>(), F->dp, F->m, F->d, F->nu2, G, k, GT, rpart,
                         apply_blocks(F->d), F->wbuf.as<double>(), status, s);
  return apply_launch(F->Hinv.as<double>(), F->dp, F->d, G, k, GT, rpart, status, s);
}

extern "C" {

const char* rs_last_error(void) { return g_err.c_str(); }
const char* rs_version(void) { return "librs 0.1 (gfx950)"; }

rs_status rs_profile_enable(int on) {
  std::lock_guard<std::mutex> g(g_prof_mu);
  if (on && !g_prof_ran) {
    RS_HIP(hipMalloc(&g_prof_ran, kProfCap * sizeof(int)));
    RS_HIP(hipMemset(g_prof_ran, 0, kProfCap * sizeof(int)));
    // the launches that set these flags run on streams that do not wait for the
    // null stream's fill
    RS_HIP(hipDeviceSynchronize());
  }
  g_prof_on = on != 0;
  return RS_OK;
}

rs_status rs_profile_read(int64_t* launches, double* total_ms) {
  if (!launches || !total_ms) return set_error(RS_ERR_ARG, "rs_profile_read: null argument");
  std::lock_guard<std::mutex> g(g_prof_mu);
  double tot = 0.0;
  int64_t cnt = 0;
  const size_t pairs = g_prof_pairs;
  std::vector<int> ran(pairs, 1);
  if (g_prof_ran && pairs) {
    RS_HIP(hipDeviceSynchronize());
    RS_HIP(hipMemcpy(ran.data(), g_prof_ran, pairs * sizeof(int), hipMemcpyDeviceToHost));
    RS_HIP(hipMemset(g_prof_ran, 0, kProfCap * sizeof(int)));
    RS_HIP(hipDeviceSynchronize());
  }
  for (size_t i = 0; i < pairs; ++i) {
    RS_HIP(hipEventSynchronize(g_prof_ev[2 * i + 1]));
    if (!ran[i]) continue;
    float ms = 0.0f;
    RS_HIP(hipEventElapsedTime(&ms, g_prof_ev[2 * i], g_prof_ev[2 * i + 1]));
    tot += ms;
    ++cnt;
  }
  g_prof_pairs = 0;
  *launches = cnt;
  *total_ms = tot;
  return RS_OK;
}

rs_status rs_params(rs_sketch_kind kind, double rho, double eta, rs_ihs_params* out) {
  if (!out) return set_error(RS_ERR_ARG, "rs_params: out is null");
  double lam, Lam;
  if (kind == RS_SKETCH_SRHT || kind == RS_SKETCH_COUNT) {
    // the CountSketch takes the SRHT's bounds (the paper gives none for it)
    if (!(rho > 0.0 && rho < 1.0)) return set_error(RS_ERR_ARG, "rs_params: SRHT needs rho in (0,1)");
    lam = 1.0 - std::sqrt(rho);
    Lam = 1.0 + std::sqrt(rho);
  } else if (kind == RS_SKETCH_GAUSSIAN) {
    if (!(rho > 0.0 && rho <= 0.18 && eta > 0.0 && eta <= 0.01))
      return set_error(RS_ERR_ARG, "rs_params: Gaussian needs rho in (0,0.18], eta in (0,0.01]");
    const double ceta = (1.0 + 3.0 * std::sqrt(eta)) * (1.0 + 3.0 * std::sqrt(eta));
    const double sq = std::sqrt(ceta * rho);
    lam = (1.0 - sq) * (1.0 - sq);
    Lam = (1.0 + sq) * (1.0 + sq);
  } else {
    return set_error(RS_ERR_ARG, "rs_params: unknown sketch kind");
  }
  const double sl = std::sqrt(lam), sL = std::sqrt(Lam);
  out->mu_gd = 2.0 / (1.0 / lam + 1.0 / Lam);
  out->cbar_gd = ((Lam - lam) / (Lam + lam)) * ((Lam - lam) / (Lam + lam));
  out->mu_p = 4.0 / ((1.0 / sl + 1.0 / sL) * (1.0 / sl + 1.0 / sL));
  out->beta_p = ((sL - sl) / (sL + sl)) * ((sL - sl) / (sL + sl));
  out->cbar_p = out->beta_p;
  return RS_OK;
}

static int32_t rule_code(int st) {
  switch (st) {
    case RS_CTL_RUNNING: return RS_RULE_RUNNING;
    case RS_CTL_CONVERGED: return RS_RULE_CONVERGED;
    case RS_CTL_DOUBLE: return RS_RULE_DOUBLE;
    case RS_CTL_STUCK: return RS_RULE_STUCK;
    case RS_CTL_NONFINITE: return RS_RULE_NONFINITE;
    default: return RS_RULE_INDEFINITE;
  }
}

int32_t rs_step_rule(int32_t polyak, double r_p, double r_gd, double r_t, double r_1, int64_t t,
                     int32_t at_cap, double cbar_p, double cbar_gd) {
  int st = RS_CTL_RUNNING;
  const int c = step_rule(polyak != 0, r_p, r_gd, r_t, r_1, t, at_cap, cbar_p, cbar_gd, &st);
  if (c == 0) return RS_RULE_ACCEPT_POLYAK;
  if (c == 1) return RS_RULE_ACCEPT_GD;
  return rule_code(st);
}

int32_t rs_start_rule(double r, double r_ref, double tol, int32_t at_cap) {
  return rule_code(start_rule(r, r_ref, tol, at_cap));
}

rs_status rs_sketch_srht(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda, int64_t m,
                         uint64_t seed, uint32_t sketch_id, void* SA, rs_dtype sa_t, int64_t ldsa,
                         float* sa_col_scale, int64_t* rows_out, int8_t* signs_out,
                         hipStream_t stream) {
  RS_TRY(check_matrix(A, a_t, n, d, lda, "rs_sketch_srht"));
  if (!SA) return set_error(RS_ERR_ARG, "rs_sketch_srht: SA is null");
  RS_TRY(check_sa_type(a_t, sa_t));
  if (sa_t == RS_FP8E4M3 && !sa_col_scale)
    return set_error(RS_ERR_ARG, "rs_sketch_srht: FP8 output needs sa_col_scale");
  const int64_t npad = next_pow2(n);
  if (npad > (int64_t)1 << 22) return set_error(RS_ERR_SHAPE, "rs_sketch_srht: padded n above 2^22");
  if (m < 1 || m > npad) return set_error(RS_ERR_SHAPE, "rs_sketch_srht: need 1 <= m <= padded n");
  if (ldsa < d) return set_error(RS_ERR_ARG, "rs_sketch_srht: ldsa < d");
  DeviceScratch* S = scratch_for_current();
  std::lock_guard<std::mutex> g(S->mu);
  return srht_run(*S, A, a_t, n, d, lda, m, seed, sketch_id, SA, sa_t, ldsa, sa_col_scale, rows_out,
                  signs_out, stream);
}

rs_status rs_sketch_gaussian(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda,
                             int64_t m, uint64_t seed, uint32_t sketch_id, void* SA, rs_dtype sa_t,
                             int64_t ldsa, float* sa_col_scale, hipStream_t stream) {
  RS_TRY(check_matrix(A, a_t, n, d, lda, "rs_sketch_gaussian"));
  if (!SA) return set_error(RS_ERR_ARG, "rs_sketch_gaussian: SA is null");
  RS_TRY(check_sa_type(a_t, sa_t));
  if (sa_t == RS_FP8E4M3 && !sa_col_scale)
    return set_error(RS_ERR_ARG, "rs_sketch_gaussian: FP8 output needs sa_col_scale");
  if (m < 1 || m > n) return set_error(RS_ERR_SHAPE, "rs_sketch_gaussian: need 1 <= m <= n");
  if (ldsa < d) return set_error(RS_ERR_ARG, "rs_sketch_gaussian: ldsa < d");
  DeviceScratch* S = scratch_for_current();
  std::lock_guard<std::mutex> g(S->mu);
  return gauss_run(*S, A, a_t, n, d, lda, m, seed, sketch_id, SA, sa_t, ldsa, sa_col_scale, stream);
}

static rs_status factor_alloc(rs_factor* F, int64_t m, int64_t d, double nu2) {
  F->m = m;
  F->d = d;
  F->wood = m < d;
  F->p = F->wood ? m : d;
  F->pp = (F->p + 63) / 64 * 64;
  F->dp = (d + 63) / 64 * 64;
  F->nu2 = nu2;
  RS_TRY(F->M.ensure(factor_bytes_M(m, d)));
  RS_TRY(F->Linv.ensure(factor_bytes_M(m, d)));
  if (!F->wood) RS_TRY(F->Hinv.ensure(factor_bytes_Hinv(d)));
  RS_TRY(F->Cw.ensure(factor_bytes_Cw(m, d)));
  if (F->wood) RS_TRY(F->wbuf.ensure(wapply_scratch_doubles(m, d) * sizeof(double)));
  RS_TRY(F->info.ensure(sizeof(int)));  // cleared on the stream before each use
  RS_TRY(F->rpart.ensure((size_t)apply_blocks(d) * 4 * sizeof(double)));
  RS_TRY(F->gram.ensure(factor_bytes_gram(m, d, F->sa_t)));
  return RS_OK;
}

rs_status rs_factor_woodbury(const void* SA, rs_dtype sa_t, const float* sa_col_scale, int64_t m,
                             int64_t d, int64_t ldsa, double nu2, rs_factor** out,
                             hipStream_t stream) {
  if (!SA || !out) return set_error(RS_ERR_ARG, "rs_factor_woodbury: null argument");
  if (sa_t == RS_FP8E4M3 && !sa_col_scale)
    return set_error(RS_ERR_ARG, "rs_factor_woodbury: FP8 SA needs sa_col_scale");
  if (m < 1 || d < 1 || ldsa < d) return set_error(RS_ERR_SHAPE, "rs_factor_woodbury: bad shape");
  if (!(nu2 > 0.0) || !std::isfinite(nu2))
    return set_error(RS_ERR_NOT_SPD, "rs_factor_woodbury: nu^2 must be positive");
  if (sa_t != RS_F32 && sa_t != RS_F64 && sa_t != RS_BF16 && sa_t != RS_FP8E4M3)
    return set_error(RS_ERR_UNSUPPORTED, "rs_factor_woodbury: SA dtype not supported");
  *out = nullptr;
  rs_factor* F = new rs_factor();
  F->sa_t = sa_t;
  rs_status st = factor_alloc(F, m, d, nu2);
  if (st == RS_OK) {
    FactorBuffers B{F->M.as<double>(), F->Linv.as<double>(),
                    F->wood ? nullptr : F->Hinv.as<double>(), F->Cw.as<double>(),
                    F->info.as<int>(), F->gram.p, F->gram.bytes, F->Cw.bytes};
    B.cw_only = F->wood;
    hipError_t e = hipMemsetAsync(B.info, 0, sizeof(int), stream);
    if (e != hipSuccess) st = set_error(RS_ERR_HIP, "hipMemsetAsync failed");
    if (st == RS_OK) st = factor_build(B, SA, sa_t, sa_col_scale, m, d, ldsa, nu2, stream);
    int info = 0;
    if (st == RS_OK) {
      e = hipMemcpyAsync(&info, B.info, sizeof(int), hipMemcpyDeviceToHost, stream);
      if (e == hipSuccess) e = hipStreamSynchronize(stream);
      if (e != hipSuccess) st = set_error(RS_ERR_HIP, hipGetErrorString(e));
    }
    if (st == RS_OK && info) st = set_error(RS_ERR_NOT_SPD, "rs_factor_woodbury: pivot not positive");
  }
  if (st != RS_OK) {
    delete F;
    return st;
  }
  *out = F;
  return RS_OK;
}

rs_status rs_factor_apply(const rs_factor* F, const double* g, double* gtilde, double* r, int64_t k,
                          hipStream_t stream) {
  if (!F || !g || !gtilde || !r) return set_error(RS_ERR_ARG, "rs_factor_apply: null argument");
  if (k < 1 || k > 4) return set_error(RS_ERR_ARG, "rs_factor_apply: k must be in 1..4");
  RS_TRY(factor_apply_any(F, g, (int)k, gtilde, F->rpart.as<double>(), nullptr, stream));
  return rsum_launch(F->rpart.as<double>(), apply_blocks(F->d), (int)k, r, stream);
}

void rs_factor_destroy(rs_factor* F) {
  delete F;  // the buffers free themselves
}

rs_status rs_gradient(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda, const void* b,
                      double nu2, const double* X, int64_t k, double* G, hipStream_t stream) {
  RS_TRY(check_matrix(A, a_t, n, d, lda, "rs_gradient"));
  if (!b || !X || !G) return set_error(RS_ERR_ARG, "rs_gradient: null argument");
  if (k < 1 || k > 4) return set_error(RS_ERR_ARG, "rs_gradient: k must be in 1..4");
  DeviceScratch* S = scratch_for_current();
  std::lock_guard<std::mutex> g(S->mu);
  const int grid = grad_partial_blocks_max(n);
  RS_TRY(S->partial.ensure((size_t)grid * k * d * sizeof(double)));
  if (a_t == RS_F32)
    return gradient_launch<float>(reinterpret_cast<const float*>(A), n, d, lda,
                                  reinterpret_cast<const float*>(b), nu2, X, (int)k, G,
                                  S->partial.as<double>(), grid, nullptr, stream);
  return gradient_launch<double>(reinterpret_cast<const double*>(A), n, d, lda,
                                 reinterpret_cast<const double*>(b), nu2, X, (int)k, G,
                                 S->partial.as<double>(), grid, nullptr, stream);
}

rs_status rs_gradient_two(const float* A, int64_t n, int64_t d, int64_t lda, const float* b,
                          const double* nu2, const double* X0, const double* X1, double* G0,
                          double* G1, hipStream_t stream) {
  RS_TRY(check_matrix(A, RS_F32, n, d, lda, "rs_gradient_two"));
  if (!b || !nu2 || !X0 || !X1 || !G0 || !G1)
    return set_error(RS_ERR_ARG, "rs_gradient_two: null argument");
  DeviceScratch* S = scratch_for_current();
  std::lock_guard<std::mutex> g(S->mu);
  const int grid = grad_partial_blocks_max(n);
  if (!gradient_two_fits(n, d, lda, grid))
    return set_error(RS_ERR_UNSUPPORTED,
                     "rs_gradient_two: the k = 2 plan for this shape is not on the 512-thread kernel");
  RS_TRY(S->partial.ensure((size_t)grid * 4 * d * sizeof(double)));
  double* p0 = S->partial.as<double>();
  const double* X[2] = {X0, X1};
  double* G[2] = {G0, G1};
  double* P[2] = {p0, p0 + (size_t)grid * 2 * d};
  const int* st[2] = {nullptr, nullptr};
  return gradient_two_launch(A, n, d, lda, b, nu2, X, G, P, grid, st, stream);
}

static rs_status grad_any(DeviceScratch& S, const void* A, rs_dtype a_t, int64_t n, int64_t d,
                          int64_t lda, const void* b, double nu2, const double* X, int k, double* G,
                          const int* status, hipStream_t s, const double* c = nullptr) {
  const int grid = grad_partial_blocks_max(n);
  RS_TRY(S.partial.ensure((size_t)grid * 4 * d * sizeof(double)));
  if (a_t == RS_F32)
    return gradient_launch<float>(reinterpret_cast<const float*>(A), n, d, lda,
                                  reinterpret_cast<const float*>(b), nu2, X, k, G,
                                  S.partial.as<double>(), grid, status, s, c);
  return gradient_launch<double>(reinterpret_cast<const double*>(A), n, d, lda,
                                 reinterpret_cast<const double*>(b), nu2, X, k, G,
                                 S.partial.as<double>(), grid, status, s, c);
}

rs_status rs_gradient_autotune(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda,
                               const void* b, int64_t k, int32_t* plan, hipStream_t stream) {
  RS_TRY(check_matrix(A, a_t, n, d, lda, "rs_gradient_autotune"));
  if (!b) return set_error(RS_ERR_ARG, "rs_gradient_autotune: b is null");
  if (k < 1 || k > 4) return set_error(RS_ERR_ARG, "rs_gradient_autotune: k must be in 1..4");
  DeviceScratch* S = scratch_for_current();
  std::lock_guard<std::mutex> g(S->mu);
  const int grid = grad_partial_blocks_max(n);
  RS_TRY(S->partial.ensure((size_t)grid * 4 * d * sizeof(double)));
  RS_TRY(S->rvec.ensure((size_t)2 * 4 * d * sizeof(double)));
  double* X = S->rvec.as<double>();
  double* G = X + 4 * d;
  RS_HIP(hipMemsetAsync(X, 0, (size_t)4 * d * sizeof(double), stream));
  GradPlan pl;
  if (a_t == RS_F32)
    RS_TRY(gradient_autotune<float>(reinterpret_cast<const float*>(A), n, d, lda,
                                    reinterpret_cast<const float*>(b), X, (int)k, G,
                                    S->partial.as<double>(), grid, stream, &pl));
  else
    RS_TRY(gradient_autotune<double>(reinterpret_cast<const double*>(A), n, d, lda,
                                     reinterpret_cast<const double*>(b), X, (int)k, G,
                                     S->partial.as<double>(), grid, stream, &pl));
  if (plan) {
    plan[0] = pl.tpr;
    plan[1] = pl.nv;
    plan[2] = pl.grid;
    plan[3] = pl.r;
  }
  return RS_OK;
}

rs_status rs_gradient_set_plan(rs_dtype a_t, int64_t n, int64_t d, int64_t k,
                               const int32_t* plan) {
  if (!plan) return set_error(RS_ERR_ARG, "rs_gradient_set_plan: plan is null");
  if (a_t != RS_F32 && a_t != RS_F64)
    return set_error(RS_ERR_ARG, "rs_gradient_set_plan: F32 or F64");
  if (n < 1 || d < 1 || k < 1 || k > 4)
    return set_error(RS_ERR_SHAPE, "rs_gradient_set_plan: bad shape");
  GradPlan pl;
  pl.tpr = plan[0];
  pl.nv = plan[1];
  pl.grid = plan[2];
  pl.r = plan[3];
  return a_t == RS_F32 ? gradient_set_plan<float>(n, d, (int)k, pl)
                       : gradient_set_plan<double>(n, d, (int)k, pl);
}

rs_status rs_gradient_plan(rs_dtype a_t, int64_t n, int64_t d, int64_t k, int32_t* plan) {
  if (!plan) return set_error(RS_ERR_ARG, "rs_gradient_plan: plan is null");
  if (a_t != RS_F32 && a_t != RS_F64) return set_error(RS_ERR_ARG, "rs_gradient_plan: F32 or F64");
  if (n < 1 || d < 1 || k < 1 || k > 4) return set_error(RS_ERR_SHAPE, "rs_gradient_plan: bad shape");
  const GradPlan pl = a_t == RS_F32 ? grad_plan<float>(n, d, (int)k) : grad_plan<double>(n, d, (int)k);
  plan[0] = pl.tpr;
  plan[1] = pl.nv;
  plan[2] = pl.grid;
  plan[3] = pl.r;
  return RS_OK;
}

rs_status rs_ihs_step(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda, const void* b,
                      double nu2, const rs_factor* F, const rs_ihs_params* p, rs_variant variant,
                      rs_ihs_state* st, rs_step_result* out, hipStream_t stream) {
  RS_TRY(check_matrix(A, a_t, n, d, lda, "rs_ihs_step"));
  if (!b || !F || !p || !st || !out || !st->x || !st->x_prev || !st->g || !st->gtilde)
    return set_error(RS_ERR_ARG, "rs_ihs_step: null argument");
  if (F->d != d) return set_error(RS_ERR_SHAPE, "rs_ihs_step: factor built for another d");
  if (st->t < 1) return set_error(RS_ERR_ARG, "rs_ihs_step: t must start at 1");
  if (!(st->r_t >= 0.0) || !(st->r_1 >= 0.0))
    return set_error(RS_ERR_ARG, "rs_ihs_step: r_t and r_1 must be >= 0 (Lemma 1)");
  const int K = variant == RS_VARIANT_POLYAK ? 2 : 1;
  DeviceScratch* S = scratch_for_current();
  std::lock_guard<std::mutex> g(S->mu);
  RS_TRY(S->vecs.ensure((size_t)6 * d * sizeof(double)));
  const int nrp = apply_blocks(d);
  RS_TRY(S->rpart.ensure((size_t)nrp * 4 * sizeof(double)));
  RS_TRY(S->ctl.ensure(sizeof(DevCtl)));
  RS_TRY(S->ev.ensure(sizeof(int32_t) * 4));
  double* X = S->vecs.as<double>();
  double* G = X + 2 * d;
  double* GT = X + 4 * d;
  DevCtl h{};
  h.r_t = st->r_t;
  h.r_1 = st->r_1;
  h.r_ref = 1.0;
  h.t = st->t;
  h.status = RS_CTL_RUNNING;
  h.at_cap = 0;
  DevCtl* dctl = S->ctl.as<DevCtl>();
  RS_HIP(hipMemcpyAsync(dctl, &h, sizeof(DevCtl), hipMemcpyHostToDevice, stream));
  CtlParams cp{p->mu_p, p->beta_p, p->mu_gd, p->cbar_p, p->cbar_gd, -1.0, INT64_MAX};
  const int* status = &dctl->status;
  RS_TRY(candidates_launch(K, d, st->x, st->x_prev, st->gtilde, X, p->mu_p, p->beta_p, p->mu_gd,
                           status, stream));
  RS_TRY(grad_any(*S, A, a_t, n, d, lda, b, nu2, X, K, G, status, stream));
  RS_TRY(factor_apply_any(F, G, K, GT, S->rpart.as<double>(), status, stream));
  RS_TRY(decide_launch(K, dctl, S->rpart.as<double>(), nrp, cp, d, X, G, GT, st->x, st->x_prev,
                       st->g, st->gtilde, S->ev.as<int32_t>(), 0, stream));
  RS_HIP(hipMemcpyAsync(&h, dctl, sizeof(DevCtl), hipMemcpyDeviceToHost, stream));
  RS_HIP(hipStreamSynchronize(stream));
  if (h.status == RS_CTL_NONFINITE) return set_error(RS_ERR_NONFINITE, "rs_ihs_step: non-finite decrement");
  if (h.last_r[1] < 0.0 || (K == 2 && h.last_r[0] < 0.0))
    return set_error(RS_ERR_NOT_SPD, "rs_ihs_step: negative decrement (H_S^-1 of F indefinite)");
  out->r_p = K == 2 ? h.last_r[0] : std::nan("");
  out->r_gd = h.last_r[1];
  if (h.status == RS_CTL_DOUBLE) {
    out->accepted = -1;
  } else {
    out->accepted = (h.polyak > 0) ? 0 : 1;
    st->r_t = h.r_t;
    st->t = h.t;
  }
  return RS_OK;
}

void rs_solve_opts_default(rs_solve_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->kind = RS_SKETCH_SRHT;
  o->variant = RS_VARIANT_POLYAK;
  o->resample = RS_RESAMPLE_FRESH;
  o->sketch_dtype = RS_F32;
  o->rho = 0.1;
  o->eta = 0.01;
  o->m_init = 1;
  o->m_max = 0;
  o->tol = 1e-7;
  o->max_iter = 200;
  o->seed = 0;
  o->check_every = 4;
}

}  // extern "C"

namespace rs {

// The 16 features of (A, nu^2) into feat (device), on stream; no argument checks.
// With b (device, n values of a_t; may be null) the same pass over A also leaves
// A^T b in column kFeatAtbCol of S.pU.
// The learned start's features (Section 5's predictor inputs) come in two parts.
// The head is one pass over A: the 256-row probe sketch and the probe sums A^T w_k,
// the squared column norms and A^T b (none of them depends on nu).  The tail
// factors the probe sketch at nu, forms the probe quadratic forms and the final
// features.  Jobs on the same A and b can share one head (features_copy_head).
static int64_t features_m0(int64_t n) { return std::min<int64_t>(256, next_pow2(n)); }

static rs_status features_buffers(DeviceScratch& S, rs_dtype a_t, int64_t n, int64_t d,
                                  hipStream_t stream) {
  const int64_t m0 = features_m0(n);
  const rs_dtype sa_t = a_t == RS_F64 ? RS_F64 : RS_F32;
  const int64_t es = a_t == RS_F64 ? 8 : 4;
  RS_TRY(S.psa.ensure((size_t)m0 * d * es));
  RS_TRY(S.pM.ensure(factor_bytes_M(m0, d)));
  RS_TRY(S.pLinv.ensure(factor_bytes_M(m0, d)));
  if (!(m0 < d)) RS_TRY(S.pHinv.ensure(factor_bytes_Hinv(d)));
  RS_TRY(S.pGram.ensure(factor_bytes_gram(m0, d, sa_t)));
  RS_TRY(S.pinfo.ensure_zeroed(sizeof(int), stream));
  RS_TRY(S.pU.ensure((size_t)(kFeatAtbCol + 1) * d * sizeof(double)));
  return RS_OK;
}

// The head; *join: the tail must wait for S.join_ev (the sums on the side stream).
// two: the first pass of another SRHT to run in the probe sketch's read of A (or null).
static rs_status features_head(DeviceScratch& S, const void* A, rs_dtype a_t, int64_t n,
                               int64_t d, int64_t lda, const void* b, uint64_t seed,
                               hipStream_t stream, bool* join, const ProbeArgs* two = nullptr) {
  const int64_t npad = next_pow2(n);
  const int64_t m0 = features_m0(n);
  const rs_dtype sa_t = a_t == RS_F64 ? RS_F64 : RS_F32;
  // one pass over A for the 8 probes A^T w_k, the squared column norms and A^T b
  // (they do not depend on the probe sketch).  FP32 A on the panel-major SRHT
  // path: the probe sketch's first pass takes these sums from the tiles it reads
  // anyway (one read of A for both).  Otherwise a pass of its own on the side
  // stream, beside the sketch.
  const bool fused = a_t == RS_F32 && srht_panel_path(npad, lda);
  if (two && !fused) return set_error(RS_ERR_ARG, "features: no shared first pass for this shape");
  *join = true;  // either way the side stream finishes the sums
  RS_TRY(S.ensure_aux());
  if (fused) {
    const int64_t ntiles = npad / 1024, dp = (d + 31) / 32 * 32;
    RS_TRY(S.pbits.ensure((size_t)n));
    RS_TRY(S.ppart.ensure((size_t)ntiles * kProbeCols * dp * sizeof(double)));
    RS_TRY(probe_bits(seed, n, S.pbits.as<uint8_t>(), stream));
    // the per-tile sums are complete after the first pass: the side stream adds them
    // up while the probe sketch's second pass runs
    const ProbeArgs pa{S.pbits.as<uint8_t>(), reinterpret_cast<const float*>(b),
                       S.ppart.as<double>(), dp, two ? two->signs2 : nullptr,
                       two ? two->Z2 : nullptr, S.fork_ev};
    RS_TRY(srht_run(S, A, a_t, n, d, lda, m0, seed, 0x7FFF0000u, S.psa.p, sa_t, d, nullptr,
                    nullptr, nullptr, stream, &pa));
    RS_HIP(hipStreamWaitEvent(S.aux, S.fork_ev, 0));
    RS_TRY(probe_tiles_finish(S.ppart.as<double>(), ntiles, d, dp, S.pU.as<double>(), S.aux));
    RS_HIP(hipEventRecord(S.join_ev, S.aux));
    return RS_OK;
  }
  const int nch = feature_chunks(n, d, a_t == RS_F32 ? 4 : 2);
  RS_TRY(S.ppart.ensure((size_t)nch * (kFeatAtbCol + 1) * d * sizeof(double)));
  RS_HIP(hipEventRecord(S.fork_ev, stream));
  RS_HIP(hipStreamWaitEvent(S.aux, S.fork_ev, 0));
  if (a_t == RS_F32)
    RS_TRY(features_pass<float>(reinterpret_cast<const float*>(A), n, d, lda,
                                reinterpret_cast<const float*>(b), seed, S.ppart.as<double>(),
                                S.pU.as<double>(), S.aux));
  else
    RS_TRY(features_pass<double>(reinterpret_cast<const double*>(A), n, d, lda,
                                 reinterpret_cast<const double*>(b), seed, S.ppart.as<double>(),
                                 S.pU.as<double>(), S.aux));
  RS_HIP(hipEventRecord(S.join_ev, S.aux));
  return srht_run(S, A, a_t, n, d, lda, m0, seed, 0x7FFF0000u, S.psa.p, sa_t, d, nullptr,
                  nullptr, nullptr, stream);
}

// Another job's head (same A, b and seed) into S: the probe sketch and the sums
// copied on `stream`, which must already wait for the head's work.
static rs_status features_copy_head(DeviceScratch& S, const DeviceScratch& from, rs_dtype a_t,
                                    int64_t n, int64_t d, hipStream_t stream) {
  const int64_t es = a_t == RS_F64 ? 8 : 4;
  RS_HIP(hipMemcpyAsync(S.psa.p, from.psa.p, (size_t)features_m0(n) * d * es,
                        hipMemcpyDeviceToDevice, stream));
  RS_HIP(hipMemcpyAsync(S.pU.p, from.pU.p, (size_t)(kFeatAtbCol + 1) * d * sizeof(double),
                        hipMemcpyDeviceToDevice, stream));
  return RS_OK;
}

static rs_status features_tail(DeviceScratch& S, rs_dtype a_t, int64_t n, int64_t d, double nu2,
                               float* feat, bool join, hipStream_t stream) {
  const int64_t m0 = features_m0(n);
  const rs_dtype sa_t = a_t == RS_F64 ? RS_F64 : RS_F32;
  // the probe sketch's factor (when m0 < d only L and L^-1 of the m0 x m0 Woodbury
  // matrix are needed)
  const bool wood = m0 < d;
  FactorBuffers FB{S.pM.as<double>(), S.pLinv.as<double>(), wood ? nullptr : S.pHinv.as<double>(),
                   nullptr, S.pinfo.as<int>(), S.pGram.p, S.pGram.bytes};
  RS_TRY(factor_build(FB, S.psa.p, sa_t, nullptr, m0, d, d, nu2, stream));
  if (join) RS_HIP(hipStreamWaitEvent(stream, S.join_ev, 0));
  // r_k = q_k / 2 with q_k = u_k^T H_S0^-1 u_k
  RS_TRY(S.pr.ensure(8 * sizeof(double)));
  if (wood) {
    RS_TRY(S.pY.ensure((size_t)8 * m0 * sizeof(double)));
    RS_TRY(probe_quads(S.psa.p, sa_t, m0, d, d, S.pLinv.as<double>(), (m0 + 63) / 64 * 64,
                       S.pU.as<double>(), nu2, S.pY.as<double>(), S.pr.as<double>(), stream));
  } else {
    const int nrp = apply_blocks(d);
    const int64_t dp = (d + 63) / 64 * 64;
    RS_TRY(S.pY.ensure((size_t)8 * d * sizeof(double)));
    RS_TRY(S.prp.ensure((size_t)nrp * 4 * sizeof(double)));
    for (int h = 0; h < 2; ++h) {
      RS_TRY(apply_launch(S.pHinv.as<double>(), dp, d, S.pU.as<double>() + (int64_t)4 * h * d, 4,
                          S.pY.as<double>() + (int64_t)4 * h * d, S.prp.as<double>(), nullptr,
                          stream));
      RS_TRY(rsum_launch(S.prp.as<double>(), nrp, 4, S.pr.as<double>() + 4 * h, stream));
    }
  }
  return features_final(S.pU.as<double>(), d, S.pr.as<double>(), n, nu2, feat, stream);
}

static rs_status features_run(DeviceScratch& S, const void* A, rs_dtype a_t, int64_t n,
                              int64_t d, int64_t lda, const void* b, double nu2, uint64_t seed,
                              float* feat, hipStream_t stream, const ProbeArgs* two = nullptr) {
  RS_TRY(features_buffers(S, a_t, n, d, stream));
  bool join = false;
  RS_TRY(features_head(S, A, a_t, n, d, lda, b, seed, stream, &join, two));
  return features_tail(S, a_t, n, d, nu2, feat, join, stream);
}

// m_init from the predicted log2 m: 2^floor(pred), clamped to [1, m_max].
static int64_t learned_m_init(float pred, const rs_solve_opts& o, int64_t n) {
  const int64_t cap = o.kind == RS_SKETCH_SRHT ? next_pow2(n) : n;
  const int64_t mmax = o.m_max > 0 ? std::min<int64_t>(o.m_max, cap) : cap;
  int64_t m0 = 1;
  if (std::isfinite(pred) && pred > 0.0f) {
    const int e = (int)std::floor(std::min(pred, 40.0f));
    m0 = (int64_t)1 << e;
  }
  return std::max<int64_t>(1, std::min<int64_t>(m0, mmax));
}

static rs_status check_features_args(rs_dtype a_t, int64_t n, int64_t d, double nu2,
                                     const char* who) {
  if (d > 8192) return set_error(RS_ERR_UNSUPPORTED, (std::string(who) + ": d above 8192").c_str());
  if (!(nu2 > 0.0))
    return set_error(RS_ERR_NOT_SPD, (std::string(who) + ": nu^2 must be positive").c_str());
  if (next_pow2(n) > (int64_t)1 << 22)
    return set_error(RS_ERR_SHAPE, (std::string(who) + ": padded n above 2^22").c_str());
  (void)a_t;
  return RS_OK;
}

// The info record of one run.  Event log: the doublings recorded at step t come
// before the step accepted at t; kinds[t] is the accepted candidate of step t.
static void fill_info(rs_solve_info* info, rs_status result, const DevCtl& h,
                      const int32_t* kinds, int64_t nkinds, const std::vector<int32_t>& dbl_t,
                      const std::vector<int64_t>& dbl_m, int64_t m_start, int64_t m_final,
                      int64_t applies) {
  const int64_t tfin = h.t;
  int64_t ne = 0;
  size_t di = 0;
  int64_t m_now = m_start;
  auto push = [&](int kind, int64_t t, int64_t mm) {
    if (ne < RS_MAX_EVENTS) {
      info->event_kind[ne] = kind;
      info->event_t[ne] = (int32_t)t;
      info->event_m[ne] = mm;
    }
    ++ne;
  };
  for (int64_t t = 1; t <= tfin; ++t) {
    while (di < dbl_t.size() && dbl_t[di] == t) {
      m_now = dbl_m[di];
      push(RS_EVENT_DOUBLE, t, m_now);
      ++di;
    }
    if (t < tfin && t < nkinds && kinds[t] >= 0)
      push(kinds[t] == 0 ? RS_EVENT_POLYAK : RS_EVENT_GD, t, m_now);
  }
  info->status = result;
  info->m_final = m_final;
  info->doublings = (int64_t)dbl_t.size();
  info->steps = h.steps;
  info->grad_passes = h.passes;
  info->applies = applies + h.passes;
  info->accepted_polyak = h.polyak;
  info->accepted_gd = h.gd;
  info->r_final = h.r_t;
  info->r_ref = h.r_ref;
  info->n_events = std::min<int64_t>(ne, RS_MAX_EVENTS);
}

static rs_status ctl_result(int status) {
  if (status == RS_CTL_CONVERGED) return RS_OK;
  if (status == RS_CTL_NONFINITE)
    return set_error(RS_ERR_NONFINITE, "solve: non-finite decrement");
  if (status == RS_CTL_INDEFINITE)
    return set_error(RS_ERR_NOT_SPD, "solve: negative decrement at m_max (H_S^-1 indefinite)");
  return set_error(RS_ERR_NO_CONVERGENCE, status == RS_CTL_STUCK ? "solve: no progress at m_max"
                                                                 : "solve: max_iter reached");
}

// One run of Algorithm 1 as a resumable job: start() enqueues the first sketch,
// factor and g_1; every later advance() is called once the previous batch of
// device work has finished (its event completed), reads the control record and
// enqueues the next batch (queued steps, or a resampling).  A single solve
// drives one job synchronously; rs_solve_batch multiplexes many jobs over
// several streams.
struct SolveJob {
  const void* A = nullptr;
  rs_dtype a_t = RS_F32;
  int64_t n = 0, d = 0, lda = 0;
  const void* b = nullptr;
  double nu2 = 0.0;
  double* x = nullptr;
  rs_solve_opts o{};
  rs_solve_info* info = nullptr;
  hipStream_t stream = nullptr;
  DeviceScratch* S = nullptr;

  rs_ihs_params prm{};
  bool srht = true;
  int64_t m_cap = 0, m = 0, ldsa = 0, dp = 0;
  int K = 2, check_every = 4, nrp = 0, ev_cap = 0;
  rs_dtype sa_t = RS_F32;
  size_t sa_es = 4;
  uint32_t sid = 0;
  CtlParams cp{};
  double *x_prev = nullptr, *g = nullptr, *gt = nullptr, *gref = nullptr;
  double *X = nullptr, *G = nullptr, *GT = nullptr;
  DevCtl* dctl = nullptr;
  int* finfo = nullptr;
  const int* status = nullptr;
  const double* Hinv = nullptr;  // m >= d: explicit inverse of the d x d factor
  bool wood = false;             // m < d: apply through Cw = L^-1 SA
  const double* Cw = nullptr;
  std::vector<int32_t> dbl_t;  // step index of each doubling
  std::vector<int64_t> dbl_m;  // m after it
  DevCtl h{};
  int64_t applies = 1;
  rs_status result = RS_OK;
  int queue = 1;
  bool done = false;
  // learned start: features and the prediction come first (phase 0)
  const float* lp_params = nullptr;
  const float* lp_mu = nullptr;
  const float* lp_sd = nullptr;
  int phase = 1;
  int64_t m_init_used = 0;
  bool atb_ready = false;  // the features pass left A^T b in S->pU
  bool defer = false;      // steps and reads left to a pair driver
  // the learned features' head taken from a partner's scratch (feat_wait: recorded
  // on the partner's stream after it)
  const DeviceScratch* feat_from = nullptr;
  hipEvent_t feat_wait = nullptr;
  // a partner's first pass to run in this job's probe sketch pass (or null)
  const ProbeArgs* feat_two = nullptr;
  // the first sketch shared within a pair (same seed and sketch_id, m2 <= m): the
  // job with the larger m forms both (sa_for: the partner, sa_done: recorded on
  // this stream after the transform); the partner's SA is then given (sa_given,
  // its stream waits for sa_wait) and it only factors
  SolveJob* sa_for = nullptr;
  int64_t sa_m2 = 0;
  const SrhtPre* sa_pre = nullptr;  // its first pass, already run (or null)
  hipEvent_t sa_done = nullptr;
  bool sa_given = false;
  hipEvent_t sa_wait = nullptr;
  int pend_q = 0;
  bool pend_read = false;
  // queued steps replayed from HIP graphs (one for a single step, one for
  // check_every steps), captured on first use under the current factor and
  // dropped when the job refactors (the apply's route and buffers follow m)
  bool use_graph = false;
  hipGraphExec_t gx[2] = {nullptr, nullptr};
  NestedCache ncache;
  NestedCache* nc_shared = nullptr;  // a path's cache, kept across its solves
  // phase timing (RS_SOLVE_TIMING): events around every sketch and factor, and
  // the first and last work of the run
  std::vector<hipEvent_t> tev;  // triples: before sketch, after sketch, after factor
  hipEvent_t tbeg = nullptr, tend = nullptr;
  bool timing() const { return (o.flags & RS_SOLVE_TIMING) != 0; }
  rs_status tmark(hipEvent_t* e) {
    if (!*e) RS_HIP(hipEventCreate(e));
    RS_HIP(hipEventRecord(*e, stream));
    return RS_OK;
  }
  // the dual problem: A holds the data matrix A^T of the dual, b a zero vector,
  // and the gradient subtracts cvec (the primal b, FP64)
  const double* cvec = nullptr;
  // sparse A (CSR, CountSketch): the gradient and the sketch take these instead
  const SparseA* sp = nullptr;

  SolveJob() = default;
  SolveJob(const SolveJob&) = delete;
  SolveJob& operator=(const SolveJob&) = delete;
  ~SolveJob() {
    for (hipGraphExec_t& g : gx)
      if (g) (void)hipGraphExecDestroy(g);
    for (hipEvent_t e : tev) (void)hipEventDestroy(e);
    if (tbeg) (void)hipEventDestroy(tbeg);
    if (tend) (void)hipEventDestroy(tend);
  }

  rs_status grad(const double* Xin, int k, double* Gout, const int* st, hipStream_t s) {
    if (sp) return sparse_gradient(S->spw, *sp, b, nu2, Xin, k, Gout, st, s, cvec);
    return grad_any(*S, A, a_t, n, d, lda, b, nu2, Xin, k, Gout, st, s, cvec);
  }

  // gtilde = H_S^-1 G under the current factor (either route)
  rs_status apply(const double* Gin, int k, double* GTout, const int* st) {
    if (wood)
      return wapply_launch(Cw, dp, m, d, nu2, Gin, k, GTout, S->rpart.as<double>(), nrp,
                           S->wbuf.as<double>(), st, stream);
    return apply_launch(Hinv, dp, d, Gin, k, GTout, S->rpart.as<double>(), st, stream);
  }

  // one step = the gradient pass over the candidates (left in X by the previous
  // decision, or by the start / resample kernels), the apply, and the decision,
  // which also writes the next step's candidates
  rs_status after_grad() {
    RS_TRY(apply(G, K, GT, status));
    return decide_launch(K, dctl, S->rpart.as<double>(), nrp, cp, d, X, G, GT, x, x_prev, g, gt,
                         S->ev.as<int32_t>(), ev_cap, stream, true, snap());
  }
  rs_status enqueue_steps(int q) {
    for (int it = 0; it < q; ++it) {
      RS_TRY(grad(X, K, G, status, stream));
      RS_TRY(after_grad());
    }
    return RS_OK;
  }

  NextCand next_cand() { return NextCand{X, prm.mu_p, prm.beta_p, prm.mu_gd, K}; }

  rs_status steps(int q) {
    if (defer) {
      pend_q = q;
      return RS_OK;
    }
    if (!use_graph || g_prof_on || (q != 1 && q != check_every)) return enqueue_steps(q);
    hipGraphExec_t& ex = gx[q == 1 ? 0 : 1];
    if (!ex) {
      RS_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
      const rs_status st = enqueue_steps(q);
      hipGraph_t gr = nullptr;
      const hipError_t e = hipStreamEndCapture(stream, &gr);
      if (st != RS_OK) {
        if (gr) (void)hipGraphDestroy(gr);
        return st;
      }
      if (e != hipSuccess) return set_error(RS_ERR_HIP, hipGetErrorString(e));
      const hipError_t e2 = hipGraphInstantiate(&ex, gr, nullptr, nullptr, 0);
      (void)hipGraphDestroy(gr);
      if (e2 != hipSuccess) {
        ex = nullptr;
        return set_error(RS_ERR_HIP, hipGetErrorString(e2));
      }
    }
    RS_HIP(hipGraphLaunch(ex, stream));
    return RS_OK;
  }

  rs_status validate() {
    if (!sp) RS_TRY(check_matrix(A, a_t, n, d, lda, "rs_adaptive_solve"));
    if ((o.kind == RS_SKETCH_COUNT) != (sp != nullptr))
      return set_error(RS_ERR_UNSUPPORTED,
                       "rs_adaptive_solve: the CountSketch is for sparse A (and sparse A for it)");
    if (!b || !x || !info) return set_error(RS_ERR_ARG, "rs_adaptive_solve: null argument");
    if (n < d) return set_error(RS_ERR_SHAPE, "rs_adaptive_solve: needs n >= d");
    if (!(nu2 > 0.0) || !std::isfinite(nu2))
      return set_error(RS_ERR_NOT_SPD, "rs_adaptive_solve: nu^2 must be positive");
    if (!(o.tol >= 0.0)) return set_error(RS_ERR_ARG, "rs_adaptive_solve: tol must be >= 0");
    if (o.max_iter < 1) return set_error(RS_ERR_ARG, "rs_adaptive_solve: max_iter must be >= 1");
    RS_TRY(check_sa_type(a_t, o.sketch_dtype));
    RS_TRY(rs_params(o.kind, o.rho, o.eta, &prm));
    srht = o.kind == RS_SKETCH_SRHT;
    const int64_t npad = next_pow2(n);
    if (srht && npad > (int64_t)1 << 22)
      return set_error(RS_ERR_SHAPE, "rs_adaptive_solve: SRHT padded n above 2^22");
    m_cap = srht ? npad : n;
    if (o.m_max > 0) m_cap = std::min<int64_t>(m_cap, o.m_max);
    m = std::min<int64_t>(std::max<int64_t>(o.m_init, 1), m_cap);
    K = o.variant == RS_VARIANT_POLYAK ? 2 : 1;
    check_every = std::max(1, (int)o.check_every);
    sa_t = o.sketch_dtype;
    sa_es = dtype_size(sa_t);
    // SA rows padded to a multiple of 64 columns: the low-precision Gram reads
    // whole 64-column segments
    ldsa = (d + 63) / 64 * 64;
    dp = (d + 63) / 64 * 64;
    nrp = apply_blocks(d);
    ev_cap = (int)std::min<int64_t>(o.max_iter + 1, 1 << 20);
    cp = CtlParams{prm.mu_p, prm.beta_p, prm.mu_gd, prm.cbar_p, prm.cbar_gd, o.tol, o.max_iter};
    return RS_OK;
  }

  rs_status sketch_and_factor(int64_t mm, uint32_t id) {
    // along a path a solve starts at the sketch its predecessor ended with: that
    // sketch and its Gram do not depend on nu, only the shifted factor is new
    const bool reuse = nc_shared && nc_shared->gram_m == mm;
    if (nc_shared) nc_shared->gram_m = 0;
    RS_TRY(S->sa.ensure((size_t)mm * ldsa * sa_es));
    RS_TRY(S->sa_scale.ensure((size_t)d * sizeof(float)));
    float* scl = sa_t == RS_FP8E4M3 ? S->sa_scale.as<float>() : nullptr;
    const size_t tk = tev.size();
    if (timing()) {
      tev.resize(tk + 3, nullptr);
      RS_TRY(tmark(&tev[tk]));
    }
    if (sa_given) {
      // a partner's transform wrote this sketch into S->sa
      RS_HIP(hipStreamWaitEvent(stream, sa_wait, 0));
      sa_given = false;
    } else if (reuse)
      ;  // SA (and its FP8 column scales) already hold this sketch
    else if (sa_for) {
      const SrhtSecond sec{sa_m2, sa_for->S->sa.p, sa_for->ldsa, sa_pre};
      RS_TRY(srht_run(*S, A, a_t, n, d, lda, mm, o.seed, id, S->sa.p, sa_t, ldsa, scl, nullptr,
                      nullptr, stream, nullptr, &sec));
      RS_HIP(hipEventRecord(sa_done, stream));
      sa_for = nullptr;
      sa_pre = nullptr;
    } else if (sp)  // nested: the same hash at 2m splits every bucket in two
      RS_TRY(count_sketch_run(S->spw, *sp, mm, o.seed, id, S->sa.p, sa_t, ldsa, stream));
    else if (o.resample == RS_RESAMPLE_NESTED)
      RS_TRY(nested_sketch(*S, nc_shared ? *nc_shared : ncache, srht, A, a_t, n, d, lda, mm,
                           o.seed, id, S->sa.p, sa_t, ldsa, scl, stream));
    else if (srht)
      RS_TRY(srht_run(*S, A, a_t, n, d, lda, mm, o.seed, id, S->sa.p, sa_t, ldsa, scl, nullptr,
                      nullptr, stream));
    else
      RS_TRY(gauss_run(*S, A, a_t, n, d, lda, mm, o.seed, id, S->sa.p, sa_t, ldsa, scl, stream));
    // step graphs captured under the previous factor hold its route, sizes and
    // buffers: they are captured again on next use (the job's queued work has
    // finished whenever it refactors)
    for (hipGraphExec_t& gxe : gx)
      if (gxe) {
        (void)hipGraphExecDestroy(gxe);
        gxe = nullptr;
      }
    // m < d and d > 2048: the Woodbury route keeps the whitened sketch
    // Cw = L^-1 SA and applies H_S^-1 through it (O(m d) per apply, m d doubles);
    // otherwise the explicit d x d inverse (at d <= 2048 it holds at most 32 MiB
    // and its apply is one launch instead of three, which the small solves of a
    // batch, bound by launches, feel: 1761 against 2178 solves/s on 256 uneven
    // problems with d <= 1024)
    const bool w = mm < d && d > kWoodburyApplyMinD;
    RS_TRY(S->fM.ensure(factor_bytes_M(mm, d)));
    RS_TRY(S->fLinv.ensure(factor_bytes_M(mm, d)));
    if (!w) RS_TRY(S->fHinv.ensure(factor_bytes_Hinv(d)));
    RS_TRY(S->fCw.ensure(factor_bytes_Cw(mm, d)));
    RS_TRY(S->fGram.ensure(factor_bytes_gram(mm, d, sa_t)));
    if (w) RS_TRY(S->wbuf.ensure(wapply_scratch_doubles(mm, d) * sizeof(double)));
    FactorBuffers FB{S->fM.as<double>(), S->fLinv.as<double>(),
                     w ? nullptr : S->fHinv.as<double>(), S->fCw.as<double>(), finfo,
                     S->fGram.p, S->fGram.bytes, S->fCw.bytes};
    FB.cw_only = w;
    if (timing()) RS_TRY(tmark(&tev[tk + 1]));
    if (reuse)
      RS_TRY(factor_finish(FB, S->sa.p, sa_t, scl, mm, d, ldsa, nu2, 1, FactorBatch{}, stream));
    else
      RS_TRY(factor_build(FB, S->sa.p, sa_t, scl, mm, d, ldsa, nu2, stream));
    if (timing()) RS_TRY(tmark(&tev[tk + 2]));
    if (nc_shared) nc_shared->gram_m = mm;
    wood = w;
    Hinv = w ? nullptr : S->fHinv.as<double>();
    Cw = S->fCw.as<double>();
    return RS_OK;
  }

  // the control record and the factor's pivot flag reach pinned host memory from
  // the kernels that change them (CtlSnap); the host waits for this event
  rs_status enqueue_read() {
    if (defer) {
      pend_read = true;
      return RS_OK;
    }
    RS_HIP(hipEventRecord(S->done_ev, stream));
    return RS_OK;
  }
  // deferred mode (a pair of jobs driven together): the steps and the read a
  // decision asks for are left to the driver, which queues them after the partner's
  // decision (the steps both jobs have share their gradient passes)
  rs_status flush_read() {
    pend_q = 0;
    if (!pend_read) return RS_OK;
    pend_read = false;
    RS_HIP(hipEventRecord(S->done_ev, stream));
    return RS_OK;
  }
  CtlSnap snap() const { return CtlSnap{S->host_pinned, finfo}; }

  rs_status start() {
    std::memset(info, 0, sizeof(*info));
    RS_TRY(S->vecs.ensure((size_t)(4 + 3 * 2) * d * sizeof(double)));
    RS_TRY(S->rpart.ensure((size_t)nrp * 4 * sizeof(double)));
    RS_TRY(S->ctl.ensure(kSnapFlagOff + 16));
    RS_TRY(S->ev.ensure((size_t)ev_cap * sizeof(int32_t)));
    if (!S->host_pinned) RS_HIP(hipHostMalloc(&S->host_pinned, 4096, hipHostMallocCoherent));
    if (!S->done_ev) RS_HIP(hipEventCreateWithFlags(&S->done_ev, hipEventDisableTiming));
    x_prev = S->vecs.as<double>();
    g = x_prev + d;
    gt = g + d;
    gref = gt + d;
    X = gref + d;
    G = X + 2 * d;
    GT = G + 2 * d;
    dctl = S->ctl.as<DevCtl>();
    finfo = reinterpret_cast<int*>(S->ctl.as<char>() + kSnapFlagOff);
    status = &dctl->status;
    RS_HIP(hipMemsetAsync(finfo, 0, sizeof(int), stream));
    // g_1 at x_0 needs no sketch: it runs on the side stream beside the sketch and
    // the factor (its scratch is not theirs)
    // (with the origin as the stop test's reference, the gradient at 0 rides in
    // the same pass as a second column: [x_1, 0] -> [g_1, g(0)])
    const int cols = (o.flags & RS_SOLVE_REF_AT_ZERO) ? 2 : 1;
    RS_TRY(S->ensure_aux());
    RS_HIP(hipEventRecord(S->fork_ev, stream));
    RS_HIP(hipStreamWaitEvent(S->aux, S->fork_ev, 0));
    const double* gin = x;
    if (cols == 2) {
      RS_HIP(hipMemcpyAsync(X, x, (size_t)d * sizeof(double), hipMemcpyDeviceToDevice, S->aux));
      RS_HIP(hipMemsetAsync(X + d, 0, (size_t)d * sizeof(double), S->aux));
      gin = X;
    }
    // after a learned prediction, a start at the origin takes g_1 = -A^T b from the
    // features pass (the same read of A) and its own gradient pass returns at once
    const int* gskip = nullptr;
    if (atb_ready && cols == 1 && !cvec) {
      int* fl = reinterpret_cast<int*>(S->ctl.as<char>() + kSnapFlagOff + 8);
      RS_TRY(start_from_atb(x, S->pU.as<double>() + (int64_t)kFeatAtbCol * d, d, G, fl, S->aux));
      gskip = fl;
    }
    RS_TRY(grad(gin, cols, G, gskip, S->aux));
    RS_HIP(hipEventRecord(S->join_ev, S->aux));
    RS_TRY(sketch_and_factor(m, sid));
    RS_HIP(hipStreamWaitEvent(stream, S->join_ev, 0));
    // gtilde_1, r_1 (and r_ref from g(0))
    RS_TRY(apply(G, cols, GT, nullptr));
    RS_TRY(init_state_launch(dctl, S->rpart.as<double>(), nrp, o.tol, o.max_iter, d, G, GT, x,
                             x_prev, g, gt, gref, m == m_cap ? 1 : 0, stream, next_cand(),
                             snap(), cols));
    if (lp_params) {
      // a predicted starting m is usually large enough for the first steps to be
      // accepted: queue check_every of them now instead of reading the state first
      // (a rejection turns the rest into no-ops, as in any queued batch)
      RS_TRY(steps(check_every));
      queue = check_every;
    }
    return enqueue_read();
  }

  bool ready() const { return hipEventQuery(S->done_ev) == hipSuccess; }

  // first work of the job: the learned prediction if a model is given, else start()
  rs_status begin() {
    if (timing()) RS_TRY(tmark(&tbeg));
    if (!lp_params) {
      m_init_used = m;
      return start();
    }
    phase = 0;
    if (!S->host_pinned) RS_HIP(hipHostMalloc(&S->host_pinned, 4096, hipHostMallocCoherent));
    if (!S->done_ev) RS_HIP(hipEventCreateWithFlags(&S->done_ev, hipEventDisableTiming));
    RS_TRY(S->pfeat.ensure(16 * sizeof(float)));
    if (feat_from) {
      // a partner on the same A, b and seed formed the features' head: copy it and
      // finish at this job's nu
      RS_TRY(features_buffers(*S, a_t, n, d, stream));
      RS_HIP(hipStreamWaitEvent(stream, feat_wait, 0));
      RS_TRY(features_copy_head(*S, *feat_from, a_t, n, d, stream));
      RS_TRY(features_tail(*S, a_t, n, d, nu2, S->pfeat.as<float>(), false, stream));
    } else {
      RS_TRY(features_run(*S, A, a_t, n, d, lda, sp ? nullptr : b, nu2, o.seed,
                          S->pfeat.as<float>(), stream, feat_two));
    }
    atb_ready = !sp;
    // the prediction goes straight to pinned host memory
    RS_TRY(mlp_forward(lp_params, S->pfeat.as<float>(), 1, lp_mu, lp_sd,
                       reinterpret_cast<float*>((char*)S->host_pinned + 1024), nullptr, stream));
    RS_HIP(hipEventRecord(S->done_ev, stream));
    return RS_OK;
  }

  // the starting m of a learned job whose prediction has reached host memory
  int64_t predicted_m() const {
    float pred = 0.0f;
    std::memcpy(&pred, (char*)S->host_pinned + 1024, sizeof(float));
    return std::min<int64_t>(std::max<int64_t>(learned_m_init(pred, o, n), 1), m_cap);
  }

  // the previous batch has finished: decide what to enqueue next
  rs_status advance() {
    if (phase == 0) {
      float pred = 0.0f;
      std::memcpy(&pred, (char*)S->host_pinned + 1024, sizeof(float));
      o.m_init = learned_m_init(pred, o, n);
      m = std::min<int64_t>(std::max<int64_t>(o.m_init, 1), m_cap);
      m_init_used = m;
      phase = 1;
      return start();
    }
    std::memcpy(&h, S->host_pinned, sizeof(DevCtl));
    int fbad = 0;
    std::memcpy(&fbad, (char*)S->host_pinned + kSnapFlagOff, sizeof(int));
    if (fbad) {
      result = set_error(RS_ERR_NOT_SPD, "rs_adaptive_solve: sketched Hessian factor failed");
      return conclude();
    }
    if (h.status == RS_CTL_RUNNING) {
      // one step right after a resample (the next step is often rejected again
      // while m is small), check_every steps after accepted ones; with accepted
      // steps behind it and no resample yet, as many as the observed contraction
      // (r_t / r_1)^(1 / (t - 1)) needs to reach tol * r_ref (queued steps past
      // convergence are no-ops, a shortfall only costs one more read)
      int q = queue;
      if (queue == check_every && dbl_t.empty() && h.t > 1 && h.r_t > 0.0 && h.r_t < h.r_1) {
        const double rho = std::pow(h.r_t / h.r_1, 1.0 / (double)(h.t - 1));
        const double need = std::log(o.tol * h.r_ref / h.r_t) / std::log(rho);
        if (std::isfinite(need) && need > 0.0)
          q = (int)std::min<double>(std::ceil(need), 2.0 * check_every);
      }
      RS_TRY(steps(q));
      queue = check_every;
      return enqueue_read();
    }
    if (h.status == RS_CTL_DOUBLE) {
      m = std::min<int64_t>(2 * m, m_cap);
      if (o.resample == RS_RESAMPLE_FRESH) ++sid;
      dbl_t.push_back((int32_t)h.t);
      dbl_m.push_back(m);
      RS_TRY(sketch_and_factor(m, sid));
      RS_TRY(pack2_launch(d, g, gref, X, stream));
      RS_TRY(apply(X, 2, GT, nullptr));
      RS_TRY(post_resample_launch(dctl, S->rpart.as<double>(), nrp, o.tol, d, GT, gt,
                                  m == m_cap ? 1 : 0, stream, next_cand(), x, x_prev, snap()));
      applies += 1;
      queue = 1;
      return enqueue_read();
    }
    if (h.status == RS_CTL_CONVERGED) result = RS_OK;
    else if (h.status == RS_CTL_NONFINITE)
      result = set_error(RS_ERR_NONFINITE, "rs_adaptive_solve: non-finite decrement");
    else if (h.status == RS_CTL_INDEFINITE)
      result = set_error(RS_ERR_NOT_SPD,
                         "rs_adaptive_solve: negative decrement at m_max (H_S^-1 indefinite)");
    else
      result = set_error(RS_ERR_NO_CONVERGENCE,
                         h.status == RS_CTL_STUCK ? "rs_adaptive_solve: no progress at m_max"
                                                  : "rs_adaptive_solve: max_iter reached");
    return conclude();
  }

  rs_status conclude() {
    done = true;
    double ms_sk = 0.0, ms_fa = 0.0, ms_all = 0.0;
    if (timing() && tbeg) {
      RS_TRY(tmark(&tend));
      RS_HIP(hipEventSynchronize(tend));
      float v = 0.0f;
      RS_HIP(hipEventElapsedTime(&v, tbeg, tend));
      ms_all = v;
      for (size_t i = 0; i + 2 < tev.size(); i += 3) {
        RS_HIP(hipEventElapsedTime(&v, tev[i], tev[i + 1]));
        ms_sk += v;
        RS_HIP(hipEventElapsedTime(&v, tev[i + 1], tev[i + 2]));
        ms_fa += v;
      }
    }
    const int64_t tfin = h.t;
    std::vector<int32_t> kinds((size_t)std::max<int64_t>(tfin, 1), -1);
    if (tfin > 1) {
      const int64_t cnt = std::min<int64_t>(tfin, ev_cap);
      RS_HIP(hipMemcpyAsync(kinds.data(), S->ev.p, (size_t)cnt * sizeof(int32_t),
                            hipMemcpyDeviceToHost, stream));
      RS_HIP(hipStreamSynchronize(stream));
    }
    fill_info(info, result, h, kinds.data(), (int64_t)kinds.size(), dbl_t, dbl_m,
              std::min<int64_t>(std::max<int64_t>(o.m_init, 1), m_cap), m, applies);
    info->ms_sketch = ms_sk;
    info->ms_factor = ms_fa;
    info->ms_iterate = ms_all > 0.0 ? std::max(0.0, ms_all - ms_sk - ms_fa) : 0.0;
    return result;
  }
};

}  // namespace rs

extern "C" {

rs_status rs_adaptive_solve(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda,
                            const void* b, double nu2, const rs_solve_opts* opts, double* x,
                            rs_solve_info* info, hipStream_t stream) {
  if (!opts) return set_error(RS_ERR_ARG, "rs_adaptive_solve: null argument");
  SolveJob J;
  J.A = A; J.a_t = a_t; J.n = n; J.d = d; J.lda = lda; J.b = b; J.nu2 = nu2; J.x = x;
  J.o = *opts; J.info = info; J.stream = stream;
  RS_TRY(J.validate());
  DeviceScratch* S = scratch_for_current();
  std::lock_guard<std::mutex> lock(S->mu);
  J.S = S;
  RS_TRY(J.begin());
  while (!J.done) {
    RS_HIP(hipEventSynchronize(S->done_ev));
    const rs_status st = J.advance();
    if (st != RS_OK && !J.done) return st;
  }
  return J.result;
}

rs_status rs_adaptive_solve_csr(const int64_t* rowptr, const int32_t* col, const void* val,
                                rs_dtype a_t, int64_t n, int64_t d, int64_t nnz, const void* b,
                                double nu2, const rs_solve_opts* opts, double* x,
                                rs_solve_info* info, hipStream_t stream) {
  if (!rowptr || !opts || !b || !x || !info || (nnz > 0 && (!col || !val)))
    return set_error(RS_ERR_ARG, "rs_adaptive_solve_csr: null argument");
  if (a_t != RS_F32 && a_t != RS_F64)
    return set_error(RS_ERR_ARG, "rs_adaptive_solve_csr: values must be F32 or F64");
  if (n < 1 || d < 1 || nnz < 0)
    return set_error(RS_ERR_SHAPE, "rs_adaptive_solve_csr: empty matrix");
  if (n >= ((int64_t)1 << 31) || nnz >= ((int64_t)1 << 31) || d > 8192)
    return set_error(RS_ERR_SHAPE, "rs_adaptive_solve_csr: needs n, nnz < 2^31 and d <= 8192");
  if (opts->kind != RS_SKETCH_COUNT)
    return set_error(RS_ERR_UNSUPPORTED, "rs_adaptive_solve_csr: sparse A takes the CountSketch");
  if (opts->sketch_dtype == RS_FP8E4M3)
    return set_error(RS_ERR_UNSUPPORTED, "rs_adaptive_solve_csr: no FP8 CountSketch");
  SparseA spa;
  spa.rowptr = rowptr; spa.col = col; spa.val = val; spa.a_t = a_t;
  spa.n = n; spa.d = d; spa.nnz = nnz;
  SolveJob J;
  J.a_t = a_t; J.n = n; J.d = d; J.lda = d; J.b = b; J.nu2 = nu2; J.x = x;
  J.o = *opts; J.o.flags &= ~RS_SOLVE_GRAPH_STEPS; J.info = info; J.stream = stream;
  J.sp = &spa;
  RS_TRY(J.validate());
  DeviceScratch* S = scratch_for_current();
  std::lock_guard<std::mutex> lock(S->mu);
  int bad = 0;
  RS_TRY(sparse_check(S->spw, spa, stream, &bad));
  if (bad)
    return set_error(RS_ERR_ARG,
                     "rs_adaptive_solve_csr: rowptr must run from 0 to nnz without decreasing "
                     "and columns must lie in [0, d)");
  RS_TRY(sparse_to_csc(S->spw, spa, stream));
  J.S = S;
  RS_TRY(J.begin());
  while (!J.done) {
    RS_HIP(hipEventSynchronize(S->done_ev));
    const rs_status st = J.advance();
    if (st != RS_OK && !J.done) return st;
  }
  return J.result;
}

rs_status rs_refreshed_ihs(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda,
                           const void* b, double nu2, const rs_solve_opts* opts, double* x,
                           double* r_hist, rs_solve_info* info, hipStream_t stream) {
  if (!opts || !info) return set_error(RS_ERR_ARG, "rs_refreshed_ihs: null argument");
  SolveJob J;
  J.A = A; J.a_t = a_t; J.n = n; J.d = d; J.lda = lda; J.b = b; J.nu2 = nu2; J.x = x;
  J.o = *opts; J.o.resample = RS_RESAMPLE_FRESH; J.info = info; J.stream = stream;
  RS_TRY(J.validate());
  const int64_t m = J.m;  // fixed: m_init clamped to [1, m_cap]
  const bool polyak = J.o.variant == RS_VARIANT_POLYAK;
  const double mu = polyak ? J.prm.mu_p : J.prm.mu_gd;
  const double beta = polyak ? J.prm.beta_p : 0.0;
  const int64_t rcap = J.o.max_iter + 1;
  DeviceScratch* S = scratch_for_current();
  std::lock_guard<std::mutex> lock(S->mu);
  J.S = S;
  std::memset(info, 0, sizeof(*info));
  RS_TRY(S->vecs.ensure((size_t)3 * d * sizeof(double)));
  RS_TRY(S->rpart.ensure((size_t)J.nrp * 4 * sizeof(double)));
  RS_TRY(S->ctl.ensure(kSnapFlagOff + 16));
  RS_TRY(S->rvec.ensure((size_t)rcap * sizeof(double)));
  double* xp = S->vecs.as<double>();
  double* G = xp + d;
  double* GT = G + d;
  double* rhist = S->rvec.as<double>();
  DevCtl* dctl = S->ctl.as<DevCtl>();
  J.finfo = reinterpret_cast<int*>(S->ctl.as<char>() + kSnapFlagOff);
  DevCtl h{};
  h.t = 1;
  RS_HIP(hipMemcpyAsync(dctl, &h, sizeof(DevCtl), hipMemcpyHostToDevice, stream));
  RS_HIP(hipMemsetAsync(J.finfo, 0, sizeof(int), stream));
  RS_HIP(hipMemcpyAsync(xp, x, (size_t)d * sizeof(double), hipMemcpyDeviceToDevice, stream));
  rs_status result = RS_OK;
  for (;;) {
    // a new sketch (sketch_id t - 1) and factor every step, then one step
    RS_TRY(J.sketch_and_factor(m, (uint32_t)(h.t - 1)));
    RS_TRY(grad_any(*S, A, a_t, n, d, lda, b, nu2, x, 1, G, nullptr, stream));
    RS_TRY(J.apply(G, 1, GT, nullptr));
    RS_TRY(refresh_step_launch(dctl, S->rpart.as<double>(), J.nrp, d, GT, x, xp, mu, beta,
                               J.o.tol, J.o.max_iter, rhist, rcap, stream));
    int fbad = 0;
    RS_HIP(hipMemcpyAsync(&h, dctl, sizeof(DevCtl), hipMemcpyDeviceToHost, stream));
    RS_HIP(hipMemcpyAsync(&fbad, J.finfo, sizeof(int), hipMemcpyDeviceToHost, stream));
    RS_HIP(hipStreamSynchronize(stream));
    if (fbad) {
      result = set_error(RS_ERR_NOT_SPD, "rs_refreshed_ihs: sketched Hessian factor failed");
      break;
    }
    if (h.status == RS_CTL_RUNNING) continue;
    if (h.status == RS_CTL_NONFINITE)
      result = set_error(RS_ERR_NONFINITE, "rs_refreshed_ihs: non-finite decrement");
    else if (h.status == RS_CTL_INDEFINITE)
      result = set_error(RS_ERR_NOT_SPD, "rs_refreshed_ihs: negative decrement (H_S^-1 indefinite)");
    else if (h.status == RS_CTL_MAXITER)
      result = set_error(RS_ERR_NO_CONVERGENCE, "rs_refreshed_ihs: max_iter reached");
    break;
  }
  const int64_t evals = std::min<int64_t>(h.passes, rcap);
  if (r_hist && evals > 0)
    RS_HIP(hipMemcpy(r_hist, rhist, (size_t)evals * sizeof(double), hipMemcpyDeviceToHost));
  info->status = result;
  info->m_final = m;
  info->steps = h.steps;
  info->grad_passes = h.passes;
  info->applies = h.passes;
  info->r_final = h.r_t;
  info->r_ref = h.r_1;
  return result;
}

rs_status rs_adaptive_solve_dual(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda,
                                 const void* b, double nu2, const rs_solve_opts* opts, double* z,
                                 double* x, rs_solve_info* info, hipStream_t stream) {
  if (!opts || !z || !x || !info || !b)
    return set_error(RS_ERR_ARG, "rs_adaptive_solve_dual: null argument");
  RS_TRY(check_matrix(A, a_t, n, d, lda, "rs_adaptive_solve_dual"));
  if (n > d) return set_error(RS_ERR_SHAPE, "rs_adaptive_solve_dual: needs n <= d");
  const int64_t es = (int64_t)dtype_size(a_t);
  const int64_t ldm = (n * es + 15) / 16 * 16 / es;  // rows of A^T: 16-byte multiples
  DeviceScratch* S = scratch_for_current();
  std::lock_guard<std::mutex> lock(S->mu);
  SolveJob J;
  J.a_t = a_t; J.n = d; J.d = n; J.lda = ldm; J.nu2 = nu2; J.x = z;
  J.o = *opts; J.o.flags &= ~RS_SOLVE_GRAPH_STEPS; J.info = info; J.stream = stream;
  // argument checks of the dual job (shape, nu, options) before any allocation
  J.A = A; J.b = b;
  RS_TRY(J.validate());
  RS_TRY(S->dM.ensure((size_t)d * ldm * es));
  RS_TRY(S->dzero.ensure((size_t)d * es));
  RS_TRY(S->dc.ensure((size_t)n * sizeof(double)));
  RS_TRY(dual_transpose(A, a_t, n, d, lda, S->dM.p, ldm, stream));
  RS_HIP(hipMemsetAsync(S->dzero.p, 0, (size_t)d * es, stream));
  RS_TRY(dual_widen(b, a_t, n, S->dc.as<double>(), stream));
  J.A = S->dM.p;
  J.b = S->dzero.p;
  J.cvec = S->dc.as<double>();
  J.S = S;
  RS_TRY(J.begin());
  while (!J.done) {
    RS_HIP(hipEventSynchronize(S->done_ev));
    const rs_status st = J.advance();
    if (st != RS_OK && !J.done) return st;
  }
  // x = A^T z, also for a solve that ended without convergence (last iterate)
  if (J.result == RS_OK || J.result == RS_ERR_NO_CONVERGENCE) {
    RS_TRY(dual_rowdot(S->dM.p, a_t, d, n, ldm, z, x, stream));
    RS_HIP(hipStreamSynchronize(stream));
  }
  return J.result;
}

rs_status rs_solve_path(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda,
                        const void* b, const double* nu2, int64_t count,
                        const rs_solve_opts* opts, double* X, rs_solve_info* infos,
                        hipStream_t stream) {
  if (!opts || !nu2 || !X || !infos) return set_error(RS_ERR_ARG, "rs_solve_path: null argument");
  if (count < 0) return set_error(RS_ERR_ARG, "rs_solve_path: count < 0");
  if (count == 0) return RS_OK;
  for (int64_t j = 0; j < count; ++j) {
    if (!(nu2[j] > 0.0) || !std::isfinite(nu2[j]))
      return set_error(RS_ERR_NOT_SPD, "rs_solve_path: nu^2 must be positive");
    if (j && nu2[j] > nu2[j - 1])
      return set_error(RS_ERR_ARG, "rs_solve_path: nu^2 must not increase along the path");
  }
  rs_solve_opts o = *opts;
  o.resample = RS_RESAMPLE_NESTED;
  o.flags = (o.flags | RS_SOLVE_REF_AT_ZERO) & ~RS_SOLVE_GRAPH_STEPS;
  {  // argument errors before any work
    SolveJob J0;
    J0.A = A; J0.a_t = a_t; J0.n = n; J0.d = d; J0.lda = lda; J0.b = b; J0.nu2 = nu2[0];
    J0.x = X; J0.o = o; J0.info = infos;
    RS_TRY(J0.validate());
  }
  DeviceScratch* S = scratch_for_current();
  std::lock_guard<std::mutex> lock(S->mu);
  NestedCache cache;  // one nested sketch family (and its transformed A) for the path
  for (int64_t j = 0; j < count; ++j) {
    double* xj = X + j * d;
    if (j)
      RS_HIP(hipMemcpyAsync(xj, xj - d, (size_t)d * sizeof(double), hipMemcpyDeviceToDevice,
                            stream));
    SolveJob J;
    J.A = A; J.a_t = a_t; J.n = n; J.d = d; J.lda = lda; J.b = b; J.nu2 = nu2[j]; J.x = xj;
    J.o = o; J.info = &infos[j]; J.stream = stream; J.nc_shared = &cache;
    RS_TRY(J.validate());
    J.S = S;
    RS_TRY(J.begin());
    while (!J.done) {
      RS_HIP(hipEventSynchronize(S->done_ev));
      const rs_status st = J.advance();
      if (st != RS_OK && !J.done) return st;
    }
    if (J.result != RS_OK && J.result != RS_ERR_NO_CONVERGENCE) return J.result;
    o.m_init = infos[j].m_final;
  }
  return RS_OK;
}

}  // extern "C"

namespace rs {

// Whether two jobs of a batch can run as a pair: the same FP32 A and b (pointers,
// shape, leading dimension), two candidates per step, no step graphs, and a k = 2
// gradient plan on the kernel that has a two-job form.
static bool pairable(const SolveJob& a, const SolveJob& b) {
  return a.A == b.A && a.b == b.b && a.a_t == RS_F32 && b.a_t == RS_F32 && a.n == b.n &&
         a.d == b.d && a.lda == b.lda && a.K == 2 && b.K == 2 && !a.use_graph && !b.use_graph &&
         !a.sp && !b.sp && !a.cvec && !b.cvec &&
         gradient_two_fits(a.n, a.d, a.lda, grad_partial_blocks_max(a.n));
}

// Two jobs on the same A and b, each on its own stream and scratch, driven by one
// host thread in rounds.  A round waits for both jobs' control records, lets each
// decide its next work (resample, steps, or the end) with its steps and read held
// back, then queues the steps both have as shared steps: one gradient pass for the
// two (gradient_two_launch, each job's result bit for bit its own pass) on job 0's
// stream once job 1's last decision is in, then each job's apply and decision on its
// own stream.  A job's extra steps run alone, and each read follows its job's last
// step.  The device decides every step as in a solve alone (queued steps past a
// rejection or the stop are no-ops), so trajectories and solutions are the jobs' own.
// With learned starts the features' head (its pass over A) is formed once, by job 0.
static void drive_pair(SolveJob* J[2], hipEvent_t ev[2]) {
  auto fail = [](SolveJob& j, rs_status st) {
    if (!j.done) {
      j.done = true;
      j.result = st;
      j.info->status = st;
    }
  };
  // learned starts: job 1 takes the features' head (one pass over A, independent
  // of nu) from job 0's scratch and finishes them at its own nu
  const bool share_head = J[0]->lp_params && J[1]->lp_params && !J[0]->sp && !J[1]->sp &&
                          J[0]->o.seed == J[1]->o.seed;
  // and the first sketches' pass 1 (sketch_id 0, every low index kept, into job 1's
  // scratch) runs in job 0's probe sketch pass: it needs only A and the signs, so one
  // read of A serves both
  const bool pre_first = share_head && J[0]->srht && J[0]->o.resample == RS_RESAMPLE_FRESH &&
                         J[0]->sid == J[1]->sid && J[0]->sa_t == J[1]->sa_t &&
                         srht_second_ok(J[0]->a_t, J[0]->n, J[0]->lda, J[0]->sa_t);
  SrhtPre pre{};
  ProbeArgs two{};
  bool pre_ok = false;
  if (pre_first) {
    // job 1's scratch is written on job 0's stream: after job 1's earlier work on it
    pre_ok = hipEventRecord(ev[1], J[1]->stream) == hipSuccess &&
             hipStreamWaitEvent(J[0]->stream, ev[1], 0) == hipSuccess &&
             srht_pretransform(*J[1]->S, J[1]->a_t, J[1]->n, J[1]->d, J[1]->lda, J[1]->o.seed,
                               J[1]->sid, J[0]->stream, &pre, &two) == RS_OK;
    if (pre_ok) J[0]->feat_two = &two;
  }
  for (int k = 0; k < 2; ++k) {
    J[k]->defer = true;
    if (k == 1 && share_head && !J[0]->done) {
      const hipError_t e = hipEventRecord(ev[0], J[0]->stream);
      if (e != hipSuccess) {
        fail(*J[1], set_error(RS_ERR_HIP, hipGetErrorString(e)));
        continue;
      }
      J[1]->feat_from = J[0]->S;
      J[1]->feat_wait = ev[0];
    }
    const rs_status st = J[k]->begin();
    J[k]->feat_two = nullptr;  // (points into this frame)
    if (st != RS_OK) fail(*J[k], st);
  }
  const int grid = grad_partial_blocks_max(J[0]->n);
  auto issue = [&]() -> rs_status {
    const bool both = !J[0]->done && !J[1]->done;
    const int common = both ? std::min(J[0]->pend_q, J[1]->pend_q) : 0;
    if (common > 0) {
      const size_t pbytes = (size_t)grid * 4 * J[0]->d * sizeof(double);
      RS_TRY(J[0]->S->partial.ensure(pbytes));
      RS_TRY(J[1]->S->partial.ensure(pbytes));
      const double nu2[2] = {J[0]->nu2, J[1]->nu2};
      const double* X[2] = {J[0]->X, J[1]->X};
      double* G[2] = {J[0]->G, J[1]->G};
      double* P[2] = {J[0]->S->partial.as<double>(), J[1]->S->partial.as<double>()};
      const int* stt[2] = {J[0]->status, J[1]->status};
      for (int it = 0; it < common; ++it) {
        RS_HIP(hipEventRecord(ev[1], J[1]->stream));
        RS_HIP(hipStreamWaitEvent(J[0]->stream, ev[1], 0));
        RS_TRY(gradient_two_launch(reinterpret_cast<const float*>(J[0]->A), J[0]->n, J[0]->d,
                                   J[0]->lda, reinterpret_cast<const float*>(J[0]->b), nu2, X, G,
                                   P, grid, stt, J[0]->stream));
        RS_HIP(hipEventRecord(ev[0], J[0]->stream));
        RS_HIP(hipStreamWaitEvent(J[1]->stream, ev[0], 0));
        RS_TRY(J[0]->after_grad());
        RS_TRY(J[1]->after_grad());
      }
    }
    for (int k = 0; k < 2; ++k) {
      if (J[k]->done) continue;
      if (J[k]->pend_q > common) RS_TRY(J[k]->enqueue_steps(J[k]->pend_q - common));
      RS_TRY(J[k]->flush_read());
    }
    return RS_OK;
  };
  for (;;) {
    const rs_status st = issue();
    if (st != RS_OK) {
      for (int k = 0; k < 2; ++k) fail(*J[k], st);
      return;
    }
    if (J[0]->done && J[1]->done) return;
    for (int k = 0; k < 2; ++k) {
      if (J[k]->done) continue;
      const hipError_t e = hipEventSynchronize(J[k]->S->done_ev);
      if (e != hipSuccess) fail(*J[k], set_error(RS_ERR_HIP, hipGetErrorString(e)));
    }
    // both learned predictions in: their first sketches have the same seed and
    // sketch_id, so the job with the larger m forms both in one transform
    int order[2] = {0, 1};
    int prod = -1;
    if (!J[0]->done && !J[1]->done && J[0]->phase == 0 && J[1]->phase == 0 && J[0]->srht &&
        !J[0]->sp && J[0]->o.resample == RS_RESAMPLE_FRESH && J[0]->sid == J[1]->sid &&
        J[0]->sa_t == J[1]->sa_t && srht_second_ok(J[0]->a_t, J[0]->n, J[0]->lda, J[0]->sa_t)) {
      const int64_t mk[2] = {J[0]->predicted_m(), J[1]->predicted_m()};
      const int p = mk[0] >= mk[1] ? 0 : 1, c = 1 - p;
      if (J[c]->S->sa.ensure((size_t)mk[c] * J[c]->ldsa * J[c]->sa_es) == RS_OK) {
        J[p]->sa_for = J[c];
        J[p]->sa_m2 = mk[c];
        // the full first pass ran in job 0's features pass, which the host has seen
        // finish (its prediction came after it)
        J[p]->sa_pre = pre_ok ? &pre : nullptr;
        J[p]->sa_done = ev[p];
        J[c]->sa_given = true;
        J[c]->sa_wait = ev[p];
        order[0] = p;
        order[1] = c;
        prod = p;
      }
    }
    for (int i = 0; i < 2; ++i) {
      const int k = order[i];
      if (J[k]->done) continue;
      const rs_status r = J[k]->advance();
      if (r != RS_OK) fail(*J[k], r);
      if (k == prod && J[k]->sa_for) {
        // the transform was not queued: the partner forms its own sketch
        J[k]->sa_for = nullptr;
        J[k]->sa_pre = nullptr;
        J[1 - k]->sa_given = false;
      }
    }
  }
}

static rs_status solve_batch_impl(const rs_problem* probs, int64_t count, const rs_solve_opts* opts,
                                  rs_solve_info* infos, int32_t workers, hipStream_t stream,
                                  const float* params, const float* mu, const float* sd,
                                  int64_t* m_init_used) {
  if (!probs || !opts || !infos) return set_error(RS_ERR_ARG, "rs_solve_batch: null argument");
  if (count < 0) return set_error(RS_ERR_ARG, "rs_solve_batch: count < 0");
  if (count == 0) return RS_OK;
  std::vector<SolveJob> jobs((size_t)count);
  for (int64_t i = 0; i < count; ++i) {
    SolveJob& J = jobs[i];
    const rs_problem& P = probs[i];
    J.A = P.A; J.a_t = P.a_t; J.n = P.n; J.d = P.d; J.lda = P.lda; J.b = P.b; J.nu2 = P.nu2;
    J.x = P.x; J.o = *opts; J.info = &infos[i];
    J.lp_params = params; J.lp_mu = mu; J.lp_sd = sd;
    J.use_graph = (opts->flags & RS_SOLVE_GRAPH_STEPS) != 0;
    RS_TRY(J.validate());
    if (params) RS_TRY(check_features_args(P.a_t, P.n, P.d, P.nu2, "rs_learned_solve_batch"));
  }
  const int W = (int)std::max<int64_t>(1, std::min<int64_t>(workers > 0 ? workers : 8, count));
  int dev = 0;
  RS_HIP(hipGetDevice(&dev));
  // worker streams and scratch: a per-device pool kept across calls (its lock is
  // held for the whole call)
  WorkerPool* pool = pool_for_current();
  std::lock_guard<std::mutex> plock(pool->mu);
  while ((int)pool->w.size() < W) {
    std::unique_ptr<BatchWorker> nw(new BatchWorker());
    RS_HIP(hipStreamCreateWithFlags(&nw->s, hipStreamNonBlocking));
    RS_HIP(hipEventCreateWithFlags(&nw->join, hipEventDisableTiming));
    pool->w.push_back(std::move(nw));
  }
  if (!pool->entry) RS_HIP(hipEventCreateWithFlags(&pool->entry, hipEventDisableTiming));
  RS_HIP(hipEventRecord(pool->entry, stream));
  for (int i = 0; i < W; ++i) RS_HIP(hipStreamWaitEvent(pool->w[i]->s, pool->entry, 0));
  // Each worker runs on a host thread of its own (worker 0 on the caller's, the
  // others on their persistent threads): it
  // takes the next unstarted job, drives it to the end on its stream (queue work,
  // wait for the job's completion event, read the control record, queue more),
  // then takes the next.  One host thread per stream keeps every stream fed while
  // another thread waits or launches.
  std::atomic<int64_t> next{0};
  std::mutex emu;
  rs_status first_err = RS_OK;
  std::string first_msg;
  auto note = [&](rs_status st) {
    std::lock_guard<std::mutex> g(emu);
    if (first_err == RS_OK) {
      first_err = st;
      first_msg = rs_last_error();
    }
  };
  // Jobs on the same FP32 A and b form pairs (pairable); a pair shares its
  // gradient passes (drive_pair) and takes two workers' streams and scratch:
  // worker 2t drives the pairs of team t one after another while worker 2t + 1
  // lends its set, then both take single jobs.
  std::vector<char> in_pair((size_t)count, 0);
  std::vector<std::array<int64_t, 2>> pairs;
  if (W >= 2)
    for (int64_t i = 0; i < count; ++i) {
      if (in_pair[i]) continue;
      for (int64_t j = i + 1; j < count; ++j)
        if (!in_pair[j] && pairable(jobs[i], jobs[j])) {
          pairs.push_back({i, j});
          in_pair[i] = in_pair[j] = 1;
          break;
        }
    }
  std::vector<int64_t> singles;
  for (int64_t i = 0; i < count; ++i)
    if (!in_pair[i]) singles.push_back(i);
  const int teams = (int)std::min<int64_t>(W / 2, (int64_t)pairs.size());
  for (int t = 0; t < 2 * teams; ++t)
    if (!pool->w[t]->step_ev)
      RS_HIP(hipEventCreateWithFlags(&pool->w[t]->step_ev, hipEventDisableTiming));
  std::atomic<int64_t> next_pair{0};
  std::mutex tmu;
  std::condition_variable tcv;
  std::vector<char> team_done((size_t)teams, 0);
  std::vector<std::vector<void*>> retired((size_t)W);
  auto run = [&](int wi) {
    BatchWorker& w = *pool->w[wi];
    t_retire = &retired[(size_t)wi];
    struct Reset {
      ~Reset() { t_retire = nullptr; }
    } reset;
    if (wi < 2 * teams) {
      const int t = wi / 2;
      if (wi % 2 == 0) {
        BatchWorker& w1 = *pool->w[wi + 1];
        for (;;) {
          const int64_t pid = next_pair.fetch_add(1);
          if (pid >= (int64_t)pairs.size()) break;
          SolveJob* J[2] = {&jobs[pairs[pid][0]], &jobs[pairs[pid][1]]};
          J[0]->S = &w.S;
          J[0]->stream = w.s;
          J[1]->S = &w1.S;
          J[1]->stream = w1.s;
          hipEvent_t ev[2] = {w.step_ev, w1.step_ev};
          drive_pair(J, ev);
          for (SolveJob* j : J)
            if (j->result != RS_OK && j->result != RS_ERR_NO_CONVERGENCE) note(j->result);
        }
        {
          std::lock_guard<std::mutex> g(tmu);
          team_done[t] = 1;
        }
        tcv.notify_all();
      } else {
        std::unique_lock<std::mutex> lk(tmu);
        tcv.wait(lk, [&] { return team_done[t] != 0; });
      }
    }
    for (;;) {
      const int64_t sid_ = next.fetch_add(1);
      if (sid_ >= (int64_t)singles.size()) return;
      SolveJob& J = jobs[singles[sid_]];
      J.S = &w.S;
      J.stream = w.s;
      rs_status st = J.begin();
      while (st == RS_OK && !J.done) {
        const hipError_t e = hipEventSynchronize(w.S.done_ev);
        if (e != hipSuccess) {
          st = set_error(RS_ERR_HIP, hipGetErrorString(e));
          break;
        }
        st = J.advance();
      }
      if (!J.done) {
        J.done = true;
        J.result = st;
        J.info->status = st;
      }
      if (J.result != RS_OK && J.result != RS_ERR_NO_CONVERGENCE) note(J.result);
    }
  };
  std::vector<BatchWorker*> posted;
  for (int i = 1; i < W; ++i) {
    BatchWorker* wp = pool->w[i].get();
    if (!wp->ensure_thread(dev)) break;  // the remaining jobs go to the workers that run
    wp->post([&run, i] { run(i); });
    posted.push_back(wp);
  }
  run(0);
  for (BatchWorker* wp : posted) wp->wait_idle();
  // the caller's stream waits for every worker
  for (int i = 0; i < W; ++i) {
    BatchWorker* wp = pool->w[i].get();
    RS_HIP(hipEventRecord(wp->join, wp->s));
    RS_HIP(hipStreamWaitEvent(stream, wp->join, 0));
    RS_HIP(hipStreamSynchronize(wp->s));
    if (wp->S.aux) RS_HIP(hipStreamSynchronize(wp->S.aux));
  }
  // the blocks the workers retired while growing their scratch
  for (std::vector<void*>& lst : retired)
    for (void* p : lst) (void)hipFree(p);
  if (first_err != RS_OK) set_error(first_err, first_msg.c_str());
  if (m_init_used)
    for (int64_t i = 0; i < count; ++i) m_init_used[i] = jobs[i].m_init_used;
  return first_err;
}

}  // namespace rs

extern "C" {

rs_status rs_solve_batch(const rs_problem* probs, int64_t count, const rs_solve_opts* opts,
                         rs_solve_info* infos, int32_t workers, hipStream_t stream) {
  return solve_batch_impl(probs, count, opts, infos, workers, stream, nullptr, nullptr, nullptr,
                          nullptr);
}

rs_status rs_learned_solve_batch(const rs_problem* probs, int64_t count, const rs_solve_opts* opts,
                                 const float* params, const float* mu, const float* sd,
                                 rs_solve_info* infos, int64_t* m_init_used, int32_t workers,
                                 hipStream_t stream) {
  if (!params || !mu || !sd)
    return set_error(RS_ERR_ARG, "rs_learned_solve_batch: null model argument");
  return solve_batch_impl(probs, count, opts, infos, workers, stream, params, mu, sd,
                          m_init_used);
}

}  // extern "C"


// ==================================================================== nu grid
namespace rs {

// Algorithm 1 for count values of nu^2 on one (A, b).  Level L of the doubling
// ladder has m_L = min(m_init 2^L, m_cap) rows and sketch_id L (fresh) or 0
// (nested): exactly the sketch a single solve at that level draws, shared here by
// every nu at that level together with its Gram partial products.  Each round
// the host reads the control records of all nu, refactors the ones that asked
// for a larger sketch (one batched factor launch per level), and queues
// check_every steps for the whole list: per step one candidate launch, one
// multi-RHS gradient (both candidates of every listed nu), one apply and one
// decision launch.  Slots that are not running skip their share on the device.
struct NuGrid {
  SolveJob base;  // argument checks and derived sizes (nu of slot 0)
  NestedCache ncache;
  const double* nu2h = nullptr;
  int64_t count = 0;
  double* X = nullptr;
  rs_solve_info* infos = nullptr;
  DeviceScratch* S = nullptr;
  hipStream_t s = nullptr;
  int64_t pp_max = 0;
  std::vector<int64_t> m_lv;             // m of each level
  std::vector<int> lvl;                  // level of each slot
  std::vector<std::vector<int32_t>> dbl_t;
  std::vector<std::vector<int64_t>> dbl_m;
  std::vector<int64_t> applies;
  std::vector<DevCtl> h;
  std::vector<char> finished;
  std::vector<int> at_cap;
  GridPtrs P{};
  // uploads: bump allocation in the pinned staging area and the device mirror
  size_t up_off = 0, up_cap = 0;
  char* up_host = nullptr;

  int64_t level_m(int L) {
    while ((int)m_lv.size() <= L) {
      const int64_t prev = m_lv.empty() ? base.m : std::min<int64_t>(2 * m_lv.back(), base.m_cap);
      m_lv.push_back(prev);
    }
    return m_lv[L];
  }

  template <typename V>
  rs_status upload(const V* src, size_t n, const V** dev) {
    const size_t bytes = (n * sizeof(V) + 255) / 256 * 256;
    if (up_off + bytes > up_cap) return set_error(RS_ERR_ARG, "nu grid: upload area exhausted");
    std::memcpy(up_host + up_off, src, n * sizeof(V));
    char* d = reinterpret_cast<char*>(S->g_up.p) + up_off;
    RS_HIP(hipMemcpyAsync(d, up_host + up_off, n * sizeof(V), hipMemcpyHostToDevice, s));
    *dev = reinterpret_cast<const V*>(d);
    up_off += bytes;
    return RS_OK;
  }

  rs_status ensure_level(int L) {
    const int64_t mL = level_m(L);
    while ((int)S->lv_sa.size() <= L) {
      S->lv_sa.emplace_back(new DevBuf());
      S->lv_scale.emplace_back(new DevBuf());
      S->lv_gram.emplace_back(new DevBuf());
    }
    DevBuf& sa = *S->lv_sa[L];
    DevBuf& sc = *S->lv_scale[L];
    DevBuf& gr = *S->lv_gram[L];
    RS_TRY(sa.ensure((size_t)mL * base.ldsa * base.sa_es));
    RS_TRY(sc.ensure((size_t)base.d * sizeof(float)));
    RS_TRY(gr.ensure(factor_bytes_gram(mL, base.d, base.sa_t)));
    const uint32_t sid = base.o.resample == RS_RESAMPLE_FRESH ? (uint32_t)L : 0u;
    float* scl = base.sa_t == RS_FP8E4M3 ? sc.as<float>() : nullptr;
    if (base.o.resample == RS_RESAMPLE_NESTED)
      RS_TRY(nested_sketch(*S, ncache, base.srht, base.A, base.a_t, base.n, base.d, base.lda, mL,
                           base.o.seed, sid, sa.p, base.sa_t, base.ldsa, scl, s));
    else if (base.srht)
      RS_TRY(srht_run(*S, base.A, base.a_t, base.n, base.d, base.lda, mL, base.o.seed, sid, sa.p,
                      base.sa_t, base.ldsa, scl, nullptr, nullptr, s));
    else
      RS_TRY(gauss_run(*S, base.A, base.a_t, base.n, base.d, base.lda, mL, base.o.seed, sid, sa.p,
                       base.sa_t, base.ldsa, scl, s));
    FactorBuffers FB{nullptr, nullptr, nullptr, nullptr, nullptr, gr.p, gr.bytes};
    return gram_partials(FB, sa.p, base.sa_t, scl, mL, base.d, base.ldsa, s);
  }

  // shifted factors of level L for the given slots, in batches that fit the scratch
  rs_status factor_level(int L, const std::vector<int>& slots) {
    const int64_t mL = level_m(L), d = base.d;
    const int64_t p = mL < d ? mL : d;
    const int64_t pp = (p + 63) / 64 * 64, dp = base.dp;
    const bool wood = mL < d;
    const size_t per = (size_t)pp * pp * 16 + (wood ? (size_t)pp * dp * 8 : 0);
    const size_t cap_bytes = (size_t)4 << 30;
    const int64_t bmax = std::max<int64_t>(1, (int64_t)(cap_bytes / per));
    float* scl = base.sa_t == RS_FP8E4M3 ? S->lv_scale[L]->as<float>() : nullptr;
    for (size_t i0 = 0; i0 < slots.size(); i0 += (size_t)bmax) {
      const int B = (int)std::min<size_t>(slots.size() - i0, (size_t)bmax);
      RS_TRY(S->g_M.ensure((size_t)B * pp * pp * 8));
      RS_TRY(S->g_L.ensure((size_t)B * pp * pp * 8));
      if (wood) RS_TRY(S->g_Cw.ensure((size_t)B * pp * dp * 8));
      std::vector<double> nu(B);
      std::vector<int> hz(B);
      for (int j = 0; j < B; ++j) {
        hz[j] = slots[i0 + j];
        nu[j] = nu2h[hz[j]];
      }
      const double* nud;
      const int* hzd;
      RS_TRY(upload(nu.data(), (size_t)B, &nud));
      RS_TRY(upload(hz.data(), (size_t)B, &hzd));
      DevBuf& gr = *S->lv_gram[L];
      FactorBuffers FB{S->g_M.as<double>(), S->g_L.as<double>(), S->g_hinv.as<double>(),
                       S->g_Cw.as<double>(), S->info.as<int>(), gr.p, gr.bytes};
      FactorBatch zb;
      zb.sM = pp * pp;
      zb.sL = pp * pp;
      zb.sH = dp * dp;
      zb.sC = pp * dp;
      zb.nu2 = nud;
      zb.hz = hzd;
      RS_TRY(factor_finish(FB, S->lv_sa[L]->p, base.sa_t, scl, mL, d, base.ldsa, 0.0, B, zb, s));
    }
    return RS_OK;
  }

  rs_status gradient(const double* Xsrc, int64_t Kc, int kper, const int* zl) {
    if (base.a_t == RS_F32)
      return mr_gradient<float>(reinterpret_cast<const float*>(base.A), base.n, base.d, base.lda,
                                reinterpret_cast<const float*>(base.b), Xsrc, Kc, kper,
                                S->g_nu2.as<double>(), zl, S->g_R.as<float>(), ldr(),
                                S->g_Gp.as<double>(), S->g_gc.as<double>(),
                                S->g_xt.as<float>(), s);
    return mr_gradient<double>(reinterpret_cast<const double*>(base.A), base.n, base.d, base.lda,
                               reinterpret_cast<const double*>(base.b), Xsrc, Kc, kper,
                               S->g_nu2.as<double>(), zl, S->g_R.as<double>(), ldr(),
                               S->g_Gp.as<double>(), S->g_gc.as<double>(),
                               S->g_xt.as<double>(), s);
  }
  int64_t ldr() const { return (2 * count + 3) / 4 * 4; }

  // check_every steps of the listed nu in one cooperative launch
  rs_status steps_persistent(const GridPtrs& Q, int nl, int K) {
    const DecideParams dpar{base.prm.mu_p, base.prm.beta_p, base.prm.mu_gd, base.prm.cbar_p,
                            base.prm.cbar_gd, base.o.tol, base.o.max_iter};
    if (base.a_t == RS_F32)
      return grid_steps<float>(Q, nl, K, reinterpret_cast<const float*>(base.A), base.n, base.d,
                               base.lda, reinterpret_cast<const float*>(base.b),
                               S->g_nu2.as<double>(), S->g_R.as<float>(), ldr(),
                               S->g_Gp.as<double>(), S->g_xt.as<float>(), base.prm.mu_p,
                               base.prm.beta_p, base.prm.mu_gd, dpar, base.check_every, s);
    return grid_steps<double>(Q, nl, K, reinterpret_cast<const double*>(base.A), base.n, base.d,
                              base.lda, reinterpret_cast<const double*>(base.b),
                              S->g_nu2.as<double>(), S->g_R.as<double>(), ldr(),
                              S->g_Gp.as<double>(), S->g_xt.as<double>(), base.prm.mu_p,
                              base.prm.beta_p, base.prm.mu_gd, dpar, base.check_every, s);
  }

  rs_status read_ctl() {
    RS_HIP(hipMemcpyAsync(S->g_pinned, S->g_ctl.p, (size_t)count * sizeof(DevCtl),
                          hipMemcpyDeviceToHost, s));
    RS_HIP(hipMemcpyAsync((char*)S->g_pinned + count * sizeof(DevCtl), S->info.p, sizeof(int),
                          hipMemcpyDeviceToHost, s));
    RS_HIP(hipEventRecord(S->done_ev, s));
    RS_HIP(hipEventSynchronize(S->done_ev));
    std::memcpy(h.data(), S->g_pinned, (size_t)count * sizeof(DevCtl));
    int bad = 0;
    std::memcpy(&bad, (char*)S->g_pinned + count * sizeof(DevCtl), sizeof(int));
    if (bad) return set_error(RS_ERR_NOT_SPD, "rs_solve_nu_grid: sketched Hessian factor failed");
    up_off = 0;
    return RS_OK;
  }

  rs_status setup() {
    const int64_t d = base.d, dp = base.dp;
    const int64_t es = base.a_t == RS_F32 ? 4 : 8;
    RS_TRY(S->g_vec.ensure((size_t)count * 4 * d * 8));
    RS_TRY(S->g_ctl.ensure((size_t)count * sizeof(DevCtl)));
    RS_TRY(S->g_ev.ensure((size_t)count * base.ev_cap * 4));
    RS_TRY(S->g_hinv.ensure((size_t)count * dp * dp * 8));
    RS_TRY(S->g_rpart.ensure((size_t)count * base.nrp * 2 * 8));
    RS_TRY(S->g_xc.ensure((size_t)count * 2 * d * 8));
    RS_TRY(S->g_gc.ensure((size_t)count * 2 * d * 8));
    RS_TRY(S->g_gtc.ensure((size_t)count * 2 * d * 8));
    RS_TRY(S->g_xt.ensure((size_t)count * 2 * d * 8));
    RS_TRY(S->g_nu2.ensure((size_t)count * 8));
    RS_TRY(S->g_R.ensure((size_t)base.n * ldr() * es));
    int64_t rps = 0;
    const int ns = mr_splits(base.n, d, 1, rps);
    RS_TRY(S->g_Gp.ensure((size_t)ns * d * ldr() * 8));
    RS_TRY(S->info.ensure(sizeof(int)));  // cleared on the stream before each use
    up_cap = (size_t)64 * count + 65536;
    RS_TRY(S->g_up.ensure(up_cap));
    const size_t pin = (size_t)count * sizeof(DevCtl) + 256 + up_cap;
    if (S->g_pinned_bytes < pin) {
      if (S->g_pinned) RS_HIP(hipHostFree(S->g_pinned));
      S->g_pinned = nullptr;
      S->g_pinned_bytes = 0;
      RS_HIP(hipHostMalloc(&S->g_pinned, pin, hipHostMallocDefault));
      S->g_pinned_bytes = pin;
    }
    up_host = (char*)S->g_pinned + count * sizeof(DevCtl) + 256;
    if (!S->done_ev) RS_HIP(hipEventCreateWithFlags(&S->done_ev, hipEventDisableTiming));
    RS_HIP(hipMemcpyAsync(S->g_nu2.p, nu2h, (size_t)count * 8, hipMemcpyHostToDevice, s));
    RS_HIP(hipMemsetAsync(S->info.p, 0, sizeof(int), s));
    P.x = X;
    P.vec = S->g_vec.as<double>();
    P.ctl = S->g_ctl.as<DevCtl>();
    P.ev = S->g_ev.as<int32_t>();
    P.ev_cap = base.ev_cap;
    P.Hinv = S->g_hinv.as<double>();
    P.sH = dp * dp;
    P.ldh = dp;
    P.rpart = S->g_rpart.as<double>();
    P.nrp = base.nrp;
    P.Xc = S->g_xc.as<double>();
    P.Gc = S->g_gc.as<double>();
    P.GTc = S->g_gtc.as<double>();
    lvl.assign(count, 0);
    dbl_t.assign(count, {});
    dbl_m.assign(count, {});
    applies.assign(count, 1);
    h.assign(count, DevCtl{});
    finished.assign(count, 0);
    at_cap.assign(count, base.m == base.m_cap ? 1 : 0);
    return RS_OK;
  }

  rs_status run() {
    RS_TRY(setup());
    const int64_t d = base.d;
    const int K = base.K;
    // level 0 for everyone: sketch, Gram, factors, g_1, gtilde_1, r_1
    std::vector<int> all(count);
    for (int64_t z = 0; z < count; ++z) all[z] = (int)z;
    RS_TRY(ensure_level(0));
    RS_TRY(factor_level(0, all));
    const int* zl;
    const int* capd;
    RS_TRY(upload(all.data(), all.size(), &zl));
    RS_TRY(upload(at_cap.data(), at_cap.size(), &capd));
    P.zl = zl;
    RS_TRY(grid_pack(P, (int)count, d, 0, s));
    RS_TRY(gradient(P.Xc, count, 1, zl));
    RS_TRY(grid_apply(P, (int)count, 1, d, P.Gc, 1, s));
    RS_TRY(grid_init(P, (int)count, base.o.tol, base.o.max_iter, d, capd, s));
    const DecideParams dpar{base.prm.mu_p, base.prm.beta_p, base.prm.mu_gd, base.prm.cbar_p,
                            base.prm.cbar_gd, base.o.tol, base.o.max_iter};
    for (;;) {
      RS_TRY(read_ctl());
      std::vector<int> run_list, dbl;
      for (int64_t z = 0; z < count; ++z) {
        if (h[z].status == RS_CTL_RUNNING) run_list.push_back((int)z);
        else if (h[z].status == RS_CTL_DOUBLE) dbl.push_back((int)z);
      }
      if (run_list.empty() && dbl.empty()) break;
      if (!dbl.empty()) {
        // group the doublings by their new level
        std::vector<std::vector<int>> by_level;
        for (int z : dbl) {
          const int L = ++lvl[z];
          const int64_t mL = level_m(L);
          dbl_t[z].push_back((int32_t)h[z].t);
          dbl_m[z].push_back(mL);
          applies[z] += 1;
          at_cap[z] = mL == base.m_cap ? 1 : 0;
          if ((int)by_level.size() <= L) by_level.resize(L + 1);
          by_level[L].push_back(z);
        }
        for (int L = 0; L < (int)by_level.size(); ++L) {
          if (by_level[L].empty()) continue;
          if (built.size() <= (size_t)L || !built[L]) {
            RS_TRY(ensure_level(L));
            if (built.size() <= (size_t)L) built.resize(L + 1, 0);
            built[L] = 1;
          }
          RS_TRY(factor_level(L, by_level[L]));
        }
        const int* dz;
        RS_TRY(upload(dbl.data(), dbl.size(), &dz));
        RS_TRY(upload(at_cap.data(), at_cap.size(), &capd));
        GridPtrs Q = P;
        Q.zl = dz;
        RS_TRY(grid_pack(Q, (int)dbl.size(), d, 1, s));
        RS_TRY(grid_apply(Q, (int)dbl.size(), 2, d, Q.Xc, 1, s));
        RS_TRY(grid_post_resample(Q, (int)dbl.size(), base.o.tol, d, capd, s));
      }
      // queue steps for every slot that may run
      std::vector<int> lst;
      lst.reserve(run_list.size() + dbl.size());
      std::merge(run_list.begin(), run_list.end(), dbl.begin(), dbl.end(),
                 std::back_inserter(lst));
      const int* sz;
      RS_TRY(upload(lst.data(), lst.size(), &sz));
      GridPtrs Q = P;
      Q.zl = sz;
      const int nl = (int)lst.size();
      if (base.o.flags & RS_SOLVE_PERSISTENT) {
        RS_TRY(steps_persistent(Q, nl, K));
        continue;
      }
      for (int it = 0; it < base.check_every; ++it) {
        RS_TRY(grid_candidates(Q, nl, K, d, base.prm.mu_p, base.prm.beta_p, base.prm.mu_gd, s));
        RS_TRY(gradient(Q.Xc, (int64_t)nl * K, K, sz));
        RS_TRY(grid_apply(Q, nl, K, d, Q.Gc, 0, s));
        RS_TRY(grid_decide(Q, nl, K, dpar, d, s));
      }
    }
    // event logs and info records
    std::vector<int32_t> kinds((size_t)count * base.ev_cap);
    RS_HIP(hipMemcpyAsync(kinds.data(), S->g_ev.p, kinds.size() * 4, hipMemcpyDeviceToHost, s));
    RS_HIP(hipStreamSynchronize(s));
    rs_status first = RS_OK;
    for (int64_t z = 0; z < count; ++z) {
      std::memset(&infos[z], 0, sizeof(rs_solve_info));
      const rs_status r = ctl_result(h[z].status);
      if (r != RS_OK && r != RS_ERR_NO_CONVERGENCE && first == RS_OK) first = r;
      fill_info(&infos[z], r, h[z], kinds.data() + z * base.ev_cap, base.ev_cap, dbl_t[z],
                dbl_m[z], level_m(0), level_m(lvl[z]), applies[z]);
    }
    return first;
  }
  std::vector<char> built{1};
};

}  // namespace rs

extern "C" {

rs_status rs_solve_nu_grid(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda,
                           const void* b, const double* nu2, int64_t count,
                           const rs_solve_opts* opts, double* X, rs_solve_info* infos,
                           hipStream_t stream) {
  if (!opts || !nu2 || !X || !infos) return set_error(RS_ERR_ARG, "rs_solve_nu_grid: null argument");
  if (count < 1 || count > 4096) return set_error(RS_ERR_ARG, "rs_solve_nu_grid: count in 1..4096");
  for (int64_t k = 0; k < count; ++k)
    if (!(nu2[k] > 0.0) || !std::isfinite(nu2[k]))
      return set_error(RS_ERR_NOT_SPD, "rs_solve_nu_grid: every nu^2 must be positive");
  NuGrid G;
  SolveJob& J = G.base;
  J.A = A; J.a_t = a_t; J.n = n; J.d = d; J.lda = lda; J.b = b; J.nu2 = nu2[0]; J.x = X;
  J.o = *opts; J.info = infos; J.stream = stream;
  RS_TRY(J.validate());
  DeviceScratch* S = scratch_for_current();
  std::lock_guard<std::mutex> lock(S->mu);
  G.nu2h = nu2;
  G.count = count;
  G.X = X;
  G.infos = infos;
  G.S = S;
  G.s = stream;
  // levels are rebuilt for every call (the sketch depends on A)
  return G.run();
}

}  // extern "C"

// ==================================================================== learned form
extern "C" {

rs_status rs_features(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda, double nu2,
                      uint64_t seed, float* feat, hipStream_t stream) {
  RS_TRY(check_matrix(A, a_t, n, d, lda, "rs_features"));
  if (!feat) return set_error(RS_ERR_ARG, "rs_features: feat is null");
  if (d > 8192) return set_error(RS_ERR_UNSUPPORTED, "rs_features: d above 8192");
  if (!(nu2 > 0.0)) return set_error(RS_ERR_NOT_SPD, "rs_features: nu^2 must be positive");
  const int64_t npad = next_pow2(n);
  if (npad > (int64_t)1 << 22) return set_error(RS_ERR_SHAPE, "rs_features: padded n above 2^22");
  DeviceScratch* S = scratch_for_current();
  std::lock_guard<std::mutex> g(S->mu);
  return features_run(*S, A, a_t, n, d, lda, nullptr, nu2, seed, feat, stream);
}

rs_status rs_mlp_forward(const float* params, const float* X, int64_t B, const float* mu,
                         const float* sd, float* y, float* cache, hipStream_t stream) {
  if (!params || !X || !mu || !sd || !y) return set_error(RS_ERR_ARG, "rs_mlp_forward: null argument");
  if (B < 1) return set_error(RS_ERR_SHAPE, "rs_mlp_forward: empty batch");
  return mlp_forward(params, X, B, mu, sd, y, cache, stream);
}

rs_status rs_mlp_backward(const float* params, const float* cache, const float* t, int64_t B,
                          float* grad, float* loss, float* work, hipStream_t stream) {
  if (!params || !cache || !t || !grad || !work)
    return set_error(RS_ERR_ARG, "rs_mlp_backward: null argument");
  if (B < 1) return set_error(RS_ERR_SHAPE, "rs_mlp_backward: empty batch");
  return mlp_backward(params, cache, t, B, grad, loss, work, stream);
}

rs_status rs_mlp_adam_step(float* params, const float* grad, float* m, float* v, int64_t count,
                           int64_t step, float lr, float beta1, float beta2, float eps,
                           hipStream_t stream) {
  if (!params || !grad || !m || !v) return set_error(RS_ERR_ARG, "rs_mlp_adam_step: null argument");
  if (count < 1 || step < 1) return set_error(RS_ERR_ARG, "rs_mlp_adam_step: count, step >= 1");
  return mlp_adam(params, grad, m, v, count, step, lr, beta1, beta2, eps, stream);
}

rs_status rs_learned_solve(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda,
                           const void* b, double nu2, const rs_solve_opts* opts,
                           const float* params, const float* mu, const float* sd, double* x,
                           rs_solve_info* info, int64_t* m_init_used, hipStream_t stream) {
  if (!opts || !params || !mu || !sd) return set_error(RS_ERR_ARG, "rs_learned_solve: null argument");
  SolveJob J;
  J.A = A; J.a_t = a_t; J.n = n; J.d = d; J.lda = lda; J.b = b; J.nu2 = nu2; J.x = x;
  J.o = *opts; J.info = info; J.stream = stream;
  J.lp_params = params; J.lp_mu = mu; J.lp_sd = sd;
  RS_TRY(J.validate());
  RS_TRY(check_features_args(a_t, n, d, nu2, "rs_learned_solve"));
  DeviceScratch* S = scratch_for_current();
  std::lock_guard<std::mutex> lock(S->mu);
  J.S = S;
  RS_TRY(J.begin());
  while (!J.done) {
    RS_HIP(hipEventSynchronize(S->done_ev));
    const rs_status st = J.advance();
    if (st != RS_OK && !J.done) return st;
  }
  if (m_init_used) *m_init_used = J.m_init_used;
  return J.result;
}

}  // extern "C"
