// Internal declarations shared by the librs translation units.
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <type_traits>

#include "rs.h"
#include "rs_device.hpp"

namespace rs {

rs_status set_error(rs_status st, const char* msg);
rs_status check_launch(const char* what);
int device_cus();
// kernel timing hooks (no-ops unless rs_profile_enable(1))
// A profiled launch gets a slot: its "did work" flag and the two events that the
// launch itself updates with the kernel's start and stop times
// (hipExtLaunchKernelGGL), so timing adds no packets to the stream.
struct ProfSlot {
  int64_t slot = -1;        // -1: not profiled
  int* ran = nullptr;       // the launch's "did work" flag, or null
  hipEvent_t begin = nullptr, end = nullptr;
};
ProfSlot prof_begin();

// hipLaunchKernelGGL, or with start/stop events when either is given.
template <typename F, typename... Args>
inline void launch_timed(F kernel, dim3 grid, dim3 block, hipStream_t s, hipEvent_t e0,
                         hipEvent_t e1, Args... args) {
  if (e0 || e1)
    hipExtLaunchKernelGGL(kernel, grid, block, 0, s, e0, e1, 0, args...);
  else
    hipLaunchKernelGGL(kernel, grid, block, 0, s, args...);
}

// ---------------------------------------------------------------- SRHT
struct SrhtBuffers {
  uint32_t* hist;      // 4096 bins, zero between calls
  int8_t* signs;       // npad
  int32_t* kmap;       // npad: row -> sample index or -1
  void* state;         // selection record
  uint64_t* cand_key;  // candidate cap
  int64_t* cand_idx;
  uint32_t* blk_less;  // npad / 1024
  int32_t* used;       // 1024, zero between calls
  int32_t* qmap;       // 1024
  int32_t* qlist;      // 1024
  int32_t* qcount;     // 1
  void* zbuf;          // pass-1 output: n1 * Qmax rows of ldz elements
  int32_t* dest2;      // npad: SA row of each second-pass row (q n1 + r1), or -1
};
rs_status srht_select(const SrhtBuffers& B, uint64_t seed, uint32_t sid, int64_t npad, int64_t m,
                      int64_t n2, int64_t* rows, hipStream_t s);
// The learned start's column sums taken by the first pass of its probe sketch from
// the tiles it loads anyway (one read of A for both): for every 1024-row tile and
// column j, part[(tile * kProbeCols + k) * dp + j] = sum over the tile's rows of
// w_k(i) A_ij (k < 8, w_k(i) = -1 where bit k of bits[i] is set), A_ij^2 (k = 8) and
// b_i A_ij (k = 9, 0 without b).  FP32 A on the panel-major path only.
constexpr int kProbeCols = 10;
struct ProbeArgs {
  const uint8_t* bits;  // n probe sign bytes
  const float* b;       // n values or null
  double* part;         // n1 * kProbeCols * dp
  int64_t dp;           // column pitch of part (d rounded up to 32)
  // optional: the same read of A also runs the first pass of another SRHT with
  // these signs and every low index kept, into Z2 (srht_pass1_prep set them up)
  const int8_t* signs2 = nullptr;
  float* Z2 = nullptr;
  // optional: recorded on the stream right after the first pass (the sums are then
  // complete and can be finished beside the second pass)
  hipEvent_t p1_done = nullptr;
};
// Whether srht_transform takes the panel-major two-pass path (the one that can
// carry ProbeArgs) for FP32 A of padded size npad and leading dimension lda.
bool srht_panel_path(int64_t npad, int64_t lda);
// A second, smaller SRHT of the same seed and sketch_id formed by the same pass:
// the m2 smallest keys are among the m smallest, so its rows are rows of this
// transform.  kmap2: row -> its sample index or -1 (its own selection); dest2b:
// scratch of Qmax * n1 int32; SA2 (ldsa2, sa_t of the first output) scaled by
// scale2 = 1/sqrt(m2).  Values bit for bit those of its own transform.  FP32 A on
// the panel-major path only.
struct SrhtDual {
  const int32_t* kmap2;
  int32_t* dest2b;
  void* SA2;
  int64_t ldsa2;
  double scale2;
};
// Pass 1 already run with every low index kept (k_srht_p1_two, same seed and
// sketch_id): its intermediate Z (Qmax = n2, q = i2) and the identity list and count
// it was run with.  The transform then runs the selection's pass 2 only, over every
// low index (rows outside the selection are not stored).
struct SrhtPre {
  const void* Z;
  const int32_t* qlist;
  const int32_t* qcount;
};
template <typename T>
rs_status srht_transform(const SrhtBuffers& B, const T* A, int64_t n, int64_t d, int64_t lda,
                         int64_t npad, int64_t m, void* SA, rs_dtype sa_t, int64_t ldsa,
                         int64_t Qmax, hipStream_t s, double scale_override = 0.0,
                         const ProbeArgs* probe = nullptr, const SrhtDual* dual = nullptr,
                         const SrhtPre* pre = nullptr);
// Set-up of a first pass of the SRHT of (seed, sid) that keeps every low index, run
// by a probe sketch's pass (ProbeArgs::signs2 = B.signs, Z2 = B.zbuf, which must hold
// srht_zbuf_bytes with Qmax = n2): writes B.signs and an identity B.qmap / B.qlist /
// B.qcount.  FP32 A on the panel-major path.
rs_status srht_pass1_prep(const SrhtBuffers& B, int64_t npad, int64_t lda, uint64_t seed,
                          uint32_t sid, hipStream_t s);
rs_status srht_gather(const void* H, rs_dtype h_t, int64_t ldh, const int64_t* rows, int64_t m,
                      int64_t d, double scale, void* SA, rs_dtype sa_t, int64_t ldsa,
                      hipStream_t s);
size_t srht_state_bytes();
// bytes of the intermediate (zbuf) of srht_transform for this shape
size_t srht_zbuf_bytes(rs_dtype a_t, int64_t npad, int64_t d, int64_t Qmax);
int srht_cand_cap();
int srht_compact_block();

// ---------------------------------------------------------------- Gaussian
rs_status gauss_scale_rows(const void* G, rs_dtype g_t, int64_t m, int64_t d, double scale,
                           void* SA, rs_dtype sa_t, int64_t ldsa, hipStream_t s);
// part: scratch of at least gauss_split_bytes(n, d, m - k_off, a_t) bytes for the
// split over A's rows (without it the launch runs unsplit).
size_t gauss_split_bytes(int64_t n, int64_t d, int64_t rows, rs_dtype a_t);
rs_status gauss_launch(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda, int64_t m,
                       uint64_t seed, uint32_t sid, void* SA, rs_dtype sa_t, int64_t ldsa,
                       hipStream_t s, int64_t k_off = 0, double scale_override = 0.0,
                       void* part = nullptr, size_t part_bytes = 0);

// ---------------------------------------------------------------- factor
struct FactorBuffers {
  double* M;     // pad64(p)^2
  double* Linv;  // pad64(p)^2
  double* Hinv;  // pad64(d)^2
  double* Cw;    // pad64(m) x pad64(d) (Woodbury branch)
  int* info;     // 1: a pivot failed
  void* gram;    // split-K partial Grams
  size_t gram_bytes;
  size_t cw_bytes = 0;  // bytes at Cw (m >= d: scratch of the split inverse product)
  // m < d: stop at the whitened sketch Cw = L^-1 SA (applied by wapply_launch) and
  // leave Hinv unwritten
  bool cw_only = false;
};
rs_status factor_build(const FactorBuffers& F, const void* SA, rs_dtype sa_t,
                       const float* colscale, int64_t m, int64_t d, int64_t ldsa, double nu2,
                       hipStream_t s);
// Batched factors of one Gram with several shifts: members z = 0..B-1 are laid
// out at element strides sM (M), sL (Linv), sH (Hinv), sC (Cw); nu2[z] on the
// device (null: the scalar shift, B = 1).
struct FactorBatch {
  int64_t sM = 0, sL = 0, sH = 0, sC = 0;
  const double* nu2 = nullptr;
  const int* hz = nullptr;  // device: Hinv slot of member z (null: z itself)
};
int gram_partial_count(int64_t m, int64_t d);
rs_status gram_partials(const FactorBuffers& F, const void* SA, rs_dtype sa_t,
                        const float* colscale, int64_t m, int64_t d, int64_t ldsa, hipStream_t s);
rs_status factor_finish(const FactorBuffers& F, const void* SA, rs_dtype sa_t,
                        const float* colscale, int64_t m, int64_t d, int64_t ldsa, double nu2,
                        int B, FactorBatch zb, hipStream_t s);

// ---------------------------------------------------------------- FP8 storage
rs_status quantize_fp8(const float* X, int64_t m, int64_t d, int64_t ldx, uint32_t* colmax,
                       float* scale, uint8_t* Q, int64_t ldq, hipStream_t s);
size_t factor_bytes_M(int64_t m, int64_t d);
size_t factor_bytes_Hinv(int64_t d);
size_t factor_bytes_gram(int64_t m, int64_t d, rs_dtype sa_t);
size_t factor_bytes_Cw(int64_t m, int64_t d);

// ---------------------------------------------------------------- gradient
int grad_partial_blocks(int64_t n);
int grad_partial_blocks_max(int64_t n);  // partial-sum blocks of any plan (buffer size)
struct GradPlan {
  int tpr = 0, nv = 0, grid = 0, r = 0;  // r: rows per group and step
};
template <typename T>
GradPlan grad_plan(int64_t n, int64_t d, int k);
template <typename T>
rs_status gradient_set_plan(int64_t n, int64_t d, int k, const GradPlan& pl);
template <typename T>
rs_status gradient_autotune(const T* A, int64_t n, int64_t d, int64_t lda, const T* b,
                            const double* X, int k, double* G, double* partial, int grid_cap,
                            hipStream_t s, GradPlan* chosen);
template <typename T>
rs_status gradient_launch(const T* A, int64_t n, int64_t d, int64_t lda, const T* b, double nu2,
                          const double* X, int k, double* G, double* partial, int grid,
                          const int* status, hipStream_t s, const double* c = nullptr,
                          bool prof = true);  // prof: false keeps the launch out of the profiler
// Two jobs on the same FP32 A and b, k = 2 columns each (X[j], G[j], partial[j],
// status[j], nu2[j]): one pass over A whose per-job results are those of
// gradient_launch with k = 2 (same plan, same arithmetic).  Only for plans on the
// 512-thread kernel (gradient_two_fits); partial[j] as for gradient_launch.
bool gradient_two_fits(int64_t n, int64_t d, int64_t lda, int grid_cap);
rs_status gradient_two_launch(const float* A, int64_t n, int64_t d, int64_t lda, const float* b,
                              const double* nu2, const double* const* X, double* const* G,
                              double* const* partial, int grid_cap, const int* const* status,
                              hipStream_t s);

// ---------------------------------------------------------------- sparse A (CSR)
struct GrowBuf {  // grow-only device buffer released with its owner
  void* p = nullptr;
  size_t bytes = 0;
  GrowBuf() = default;
  GrowBuf(const GrowBuf&) = delete;
  GrowBuf& operator=(const GrowBuf&) = delete;
  ~GrowBuf() {
    if (p) (void)hipFree(p);
  }
  rs_status ensure(size_t want);
  template <typename T>
  T* as() const {
    return reinterpret_cast<T*>(p);
  }
};
struct SparseA {
  const int64_t* rowptr = nullptr;  // n + 1 entries
  const int32_t* col = nullptr;     // nnz column indices
  const void* val = nullptr;        // nnz values (a_t)
  rs_dtype a_t = RS_F32;
  int64_t n = 0, d = 0, nnz = 0;
};
struct SparseWork {
  GrowBuf ckey, cpos, rid, crow, cval, colptr, R, hkey, hrow, hsign, hoff, flag;
  GrowBuf cnch, ccst, cpart;  // chunks of the columns (A^T r pass)
  GrowBuf hnch, hcst, spart;  // chunks of the buckets (sketch)
  GrowBuf tmp;
  int64_t atr_chunks = 0;     // upper bound on the column chunks
};
// 0 when rowptr runs from 0 to nnz without decreasing and every column is in [0, d)
rs_status sparse_check(SparseWork& W, const SparseA& sp, hipStream_t s, int* bad_host);
rs_status sparse_to_csc(SparseWork& W, const SparseA& sp, hipStream_t s);
rs_status sparse_gradient(SparseWork& W, const SparseA& sp, const void* b, double nu2,
                          const double* X, int K, double* G, const int* status, hipStream_t s,
                          const double* sub);
rs_status count_sketch_run(SparseWork& W, const SparseA& sp, int64_t m, uint64_t seed,
                           uint32_t sid, void* SA, rs_dtype sa_t, int64_t ldsa, hipStream_t s);

// ---------------------------------------------------------------- dual (n < d)
// M = A^T (d x ldm, padding columns zeroed); c = b in FP64; x = M z.
rs_status dual_transpose(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda, void* M,
                         int64_t ldm, hipStream_t s);
rs_status dual_widen(const void* b, rs_dtype a_t, int64_t n, double* c, hipStream_t s);
rs_status dual_rowdot(const void* M, rs_dtype a_t, int64_t rows, int64_t cols, int64_t ldm,
                      const double* z, double* x, hipStream_t s);

// ---------------------------------------------------------------- apply
constexpr int kApplyRPW = 1;  // rows of H_S^-1 per wave in the apply
int apply_blocks(int64_t d);
rs_status apply_launch(const double* Hinv, int64_t ldh, int64_t d, const double* G, int k,
                       double* Y, double* rpart, const int* status, hipStream_t s);
rs_status rsum_launch(const double* rpart, int nblk, int k, double* r, hipStream_t s);
// The Woodbury form for m < d: gtilde = (G - C^T (C G)) / nu^2 with C = L^-1 SA
// (m x d at leading dimension ldc), the same rpart layout (nrp >= ceil(d / 256)
// blocks) as apply_launch; scratch: wapply_scratch_doubles(m, d) doubles.
size_t wapply_scratch_doubles(int64_t m, int64_t d);
rs_status wapply_launch(const double* C, int64_t ldc, int64_t m, int64_t d, double nu2,
                        const double* G, int k, double* GT, double* rpart, int nrp,
                        double* scratch, const int* status, hipStream_t s);

// ---------------------------------------------------------------- control
enum {
  RS_CTL_RUNNING = 0,
  RS_CTL_CONVERGED = 1,
  RS_CTL_DOUBLE = 2,
  RS_CTL_STUCK = 3,
  RS_CTL_MAXITER = 4,
  RS_CTL_NONFINITE = 5,
  RS_CTL_INDEFINITE = 6  // a decrement < 0 at m_max: the factor's H_S^-1 is not positive definite
};

// The two tests of one step of Algorithm 1, in FP64: the Polyak candidate
// (decrement r0, only when `polyak`) passes if (r0 / r1)^(1/t) <= cbar_p, else the
// gradient candidate (rg) if rg / rt <= cbar_gd; ties accept.  At m_max a double
// rejection still takes the gradient candidate if it lowers r.  Returns the chosen
// candidate (0 Polyak, 1 gradient, -1 none) and the status in *st.  H_S is positive
// definite (eq. (3)), so each decrement 1/2 g^T H_S^-1 g is >= 0; a negative one
// means the factor lost definiteness (the Woodbury subtraction of a low-precision
// Gram when nu^2 is small): it fails every test and asks for a larger sketch, and
// at m_max ends the run as INDEFINITE.  Every decision kernel and the exported
// host check (rs_step_rule) run this one copy.
// v - v is 0 exactly for finite v and NaN for NaN or an infinity (host and device alike)
__host__ __device__ inline bool finite_value(double v) { return (v - v) == 0.0; }

__host__ __device__ inline int step_rule(bool polyak, double r0, double rg, double rt, double r1,
                                         int64_t t, int at_cap, double cbar_p, double cbar_gd,
                                         int* st) {
  *st = RS_CTL_RUNNING;
  if (!finite_value(rg) || (polyak && !finite_value(r0))) {
    *st = RS_CTL_NONFINITE;
    return -1;
  }
  if (rg < 0.0 || (polyak && r0 < 0.0)) {
    *st = at_cap ? RS_CTL_INDEFINITE : RS_CTL_DOUBLE;
    return -1;
  }
  if (polyak && pow(r0 / r1, 1.0 / (double)t) <= cbar_p) return 0;
  if (rg / rt <= cbar_gd) return 1;
  if (at_cap) {
    if (rg < rt) return 1;
    *st = RS_CTL_STUCK;
    return -1;
  }
  *st = RS_CTL_DOUBLE;
  return -1;
}

// The state after a (re)factor: decrement r at the current point and the stop
// test's reference r_ref, both under the new sketch.  Negative values mean an
// indefinite H_S^-1 (see step_rule): a larger sketch, or INDEFINITE at m_max.
__host__ __device__ inline int start_rule(double r, double r_ref, double tol, int at_cap) {
  if (!finite_value(r) || !finite_value(r_ref)) return RS_CTL_NONFINITE;
  if (r < 0.0 || r_ref < 0.0) return at_cap ? RS_CTL_INDEFINITE : RS_CTL_DOUBLE;
  if (r <= tol * r_ref) return RS_CTL_CONVERGED;
  return RS_CTL_RUNNING;
}

struct DevCtl {
  double r_t, r_1, r_ref;
  double last_r[2];
  int64_t t, steps, passes, polyak, gd;
  int32_t status;
  int32_t at_cap;
};

// A copy of the control record (and the factor's pivot flag right after it, at
// kSnapFlagOff) that the kernels changing the record write into host memory the
// device can store to (pinned), so the host reads the state after the completion
// event with no copy on the stream.  ctl null: not written.
constexpr size_t kSnapFlagOff = (sizeof(DevCtl) + 15) / 16 * 16;
struct CtlSnap {
  void* host = nullptr;         // DevCtl at offset 0, int flag at kSnapFlagOff
  const int* flag = nullptr;    // the factor's pivot flag on the device
};

struct CtlParams {
  double mu_p, beta_p, mu_gd, cbar_p, cbar_gd, tol;
  int64_t max_iter;
};

rs_status candidates_launch(int K, int64_t d, const double* x, const double* x_prev,
                            const double* gt, double* X, double mu_p, double beta_p, double mu_gd,
                            const int* status, hipStream_t s);
rs_status decide_launch(int K, DevCtl* ctl, const double* rpart, int nrp, const CtlParams& p,
                        int64_t d, double* X, const double* G, const double* GT, double* x,
                        double* x_prev, double* g, double* gt, int32_t* ev_kind, int ev_cap,
                        hipStream_t s, bool next = false, CtlSnap snap = CtlSnap());
// The next step's candidates, written by the kernel that leaves the state running
// (X null: not written).
struct NextCand {
  double* X = nullptr;
  double mu_p = 0.0, beta_p = 0.0, mu_gd = 0.0;
  int K = 2;
};
rs_status init_state_launch(DevCtl* ctl, const double* rpart, int nrp, double tol,
                            int64_t max_iter, int64_t d, const double* G, const double* GT,
                            const double* x, double* x_prev, double* g, double* gt, double* gref,
                            int at_cap, hipStream_t s, NextCand nc = NextCand(),
                            CtlSnap snap = CtlSnap(), int cols = 1);
rs_status refresh_step_launch(DevCtl* ctl, const double* rpart, int nrp, int64_t d,
                              const double* GT, double* x, double* x_prev, double mu, double beta,
                              double tol, int64_t max_iter, double* rhist, int64_t rcap,
                              hipStream_t s);
rs_status post_resample_launch(DevCtl* ctl, const double* rpart, int nrp, double tol, int64_t d,
                               const double* GT, double* gt, int at_cap, hipStream_t s,
                               NextCand nc = NextCand(), const double* x = nullptr,
                               const double* x_prev = nullptr, CtlSnap snap = CtlSnap());
rs_status pack2_launch(int64_t d, const double* a, const double* b, double* out, hipStream_t s);

// ---------------------------------------------------------------- nu grid
struct DecideParams {
  double mu_p, beta_p, mu_gd, cbar_p, cbar_gd, tol;
  int64_t max_iter;
};
struct GridPtrs {
  double* x;          // slot z: x at x + z d
  double* vec;        // slot z: x_prev, g, gtilde, g_ref at vec + z 4d
  DevCtl* ctl;        // slot z: ctl[z]
  int32_t* ev;        // slot z: ev + z ev_cap
  int ev_cap;
  const double* Hinv; // slot z: Hinv + z sH, leading dimension ldh
  int64_t sH, ldh;
  double* rpart;      // slot z: rpart + z nrp 2
  int nrp;
  double* Xc;         // list entry y: Xc / Gc / GTc + y K d
  double* Gc;
  double* GTc;
  const int* zl;      // list entry y -> slot
};
int mr_splits(int64_t n, int64_t d, int64_t Kc, int64_t& rows_per_split);
template <typename T>
rs_status mr_gradient(const T* A, int64_t n, int64_t d, int64_t lda, const T* b, const double* X,
                      int64_t Kc, int kper, const double* nu2, const int* zl, T* R, int64_t ldr,
                      double* Gp, double* G, T* XT, hipStream_t s);
// Up to iters steps of every listed nu in one cooperative (persistent) launch:
// candidates, the multi-RHS gradient, the apply and the decision, separated by
// grid barriers; returns early once no listed nu is running.  Same results as
// the separate launches (grid_candidates, mr_gradient, grid_apply, grid_decide).
template <typename T>
rs_status grid_steps(const GridPtrs& P, int nl, int K, const T* A, int64_t n, int64_t d,
                     int64_t lda, const T* b, const double* nu2, T* R, int64_t ldr, double* Gp,
                     T* XT, double mu_p, double beta_p, double mu_gd, const DecideParams& dp,
                     int iters, hipStream_t s);
rs_status grid_candidates(const GridPtrs& P, int nl, int K, int64_t d, double mu_p, double beta_p,
                          double mu_gd, hipStream_t s);
rs_status grid_pack(const GridPtrs& P, int nl, int64_t d, int what, hipStream_t s);
rs_status grid_apply(const GridPtrs& P, int nl, int K, int64_t d, const double* Gsrc, int always,
                     hipStream_t s);
rs_status grid_decide(const GridPtrs& P, int nl, int K, const DecideParams& a, int64_t d,
                      hipStream_t s);
rs_status grid_init(const GridPtrs& P, int nl, double tol, int64_t max_iter, int64_t d,
                    const int* at_cap, hipStream_t s);
rs_status grid_post_resample(const GridPtrs& P, int nl, double tol, int64_t d, const int* at_cap,
                             hipStream_t s);

// ---------------------------------------------------------------- learned form
int feature_chunks(int64_t n, int64_t d, int vec);
template <typename T>
rs_status features_pass(const T* A, int64_t n, int64_t d, int64_t lda, const T* b,
                        uint64_t seed, double* part, double* U, hipStream_t s);
// U column of A^T b in the features pass's output (after the 8 probes and the
// squared column norms)
constexpr int kFeatAtbCol = 9;
// bits[i] = the 8 probe signs of row i (bit k set: w_k(i) = -1), Philox stream 7
rs_status probe_bits(uint64_t seed, int64_t n, uint8_t* bits, hipStream_t s);
// U[k * d + j] = sum over the ntiles tiles of part[(tile * kProbeCols + k) * dp + j]
// (fixed order), k < kProbeCols
rs_status probe_tiles_finish(const double* part, int64_t ntiles, int64_t d, int64_t dp, double* U,
                             hipStream_t s);
// G = -A^T b and *skip = 1 when every x_j is 0 (the gradient at the origin), else
// *skip = 0 and G untouched; one block
rs_status start_from_atb(const double* x, const double* atb, int64_t d, double* G, int* skip,
                         hipStream_t s);
rs_status probe_quads(const void* SA, rs_dtype sa_t, int64_t m, int64_t d, int64_t ldsa,
                      const double* Linv, int64_t ldl, const double* U, double nu2, double* V,
                      double* r, hipStream_t s);
rs_status features_final(const double* U, int64_t d, const double* rprobe, int64_t n, double nu2,
                         float* feat, hipStream_t s);
rs_status mlp_forward(const float* P, const float* X, int64_t B, const float* mu, const float* sd,
                      float* Y, float* cache, hipStream_t s);
rs_status mlp_backward(const float* P, const float* cache, const float* T, int64_t B, float* G,
                       float* loss, float* work, hipStream_t s);
rs_status mlp_adam(float* P, const float* G, float* M, float* V, int64_t count, int64_t step,
                   float lr, float b1, float b2, float eps, hipStream_t s);
int mlp_params();
int mlp_cache_floats();
int mlp_work_floats();

}  // namespace rs
