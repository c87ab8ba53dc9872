/*
 * rs.h -- C ABI of librs, the MI355X (gfx950) adaptive Hessian-sketch ridge solver.
 *
 * Problem (Lacotte & Pilanci, NeurIPS 2020, eq. (1)):
 *     x* = argmin_x  1/2 ||A x - b||^2 + nu^2/2 ||x||^2,   A is n x d, n >= d.
 *
 * Conventions shared by every entry point
 *   - Array arguments are DEVICE pointers owned by the caller unless a comment
 *     says "host".  The library never frees caller memory.
 *   - Matrices are row-major with an explicit leading dimension (elements).
 *     A (n x d) has lda >= d; lda must be a multiple of 16/sizeof(element) and A
 *     16-byte aligned (vector loads).  Sizes are int64_t.
 *   - Vectors of the iteration (x, g, g~) are FP64.  A k-column block of vectors
 *     ("k RHS") is stored column after column: V[c*d + i].
 *   - All work is enqueued on the given stream.  Functions that return host
 *     values synchronize that stream first; the others do not.
 *   - Every argument is validated before any launch; errors come back as
 *     rs_status and rs_last_error() returns a thread-local message.  No C++
 *     exception crosses the ABI.
 *   - Internal scratch (histograms, transform intermediates, partial sums) is
 *     owned by the library, allocated once per device and grown on demand.
 *     Every call holds a per-device lock while it queues its work, so calls
 *     from several host threads keep the library's host state consistent; the
 *     device work of two calls queued on different streams can still overlap
 *     and race on that scratch: queue them on one stream or serialize them.
 *     The batched solvers run their jobs on worker streams with scratch of
 *     their own (a per-device worker pool, locked for the whole call).
 */
#ifndef RS_H_
#define RS_H_

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  RS_OK = 0,
  RS_ERR_ARG = 1,             /* null pointer, bad enum, bad alignment/leading dimension */
  RS_ERR_SHAPE = 2,           /* n < d, m < 1, m > padded n, unsupported size */
  RS_ERR_NOT_POW2 = 3,        /* reserved: non power-of-two sizes are zero-padded */
  RS_ERR_NOT_SPD = 4,         /* a Cholesky pivot was not positive (e.g. nu^2 <= 0) */
  RS_ERR_NONFINITE = 5,       /* NaN or Inf met in the iteration */
  RS_ERR_NO_CONVERGENCE = 6,  /* tolerance not met within max_iter, or stuck at m_max */
  RS_ERR_OOM = 7,
  RS_ERR_HIP = 8,             /* a HIP runtime call failed */
  RS_ERR_UNSUPPORTED = 9      /* valid request outside what the library implements */
} rs_status;

typedef enum { RS_F64 = 0, RS_F32 = 1, RS_BF16 = 2, RS_FP8E4M3 = 3 } rs_dtype;
/* COUNT: the CountSketch, one signed nonzero per column of S (for sparse A, see
 * rs_adaptive_solve_csr). */
typedef enum { RS_SKETCH_SRHT = 0, RS_SKETCH_GAUSSIAN = 1, RS_SKETCH_COUNT = 2 } rs_sketch_kind;
/* FRESH: each doubling draws a new sketch (Algorithm 1 samples S afresh).
 * NESTED: keeps the signs and row keys; the 2m rows include the previous m. */
typedef enum { RS_RESAMPLE_FRESH = 0, RS_RESAMPLE_NESTED = 1 } rs_resample;
/* POLYAK: Algorithm 1.  GD_ONLY: its gradient-only variant (Section 4). */
typedef enum { RS_VARIANT_POLYAK = 0, RS_VARIANT_GD_ONLY = 1 } rs_variant;

/* Step sizes and target rates of Algorithm 1. */
typedef struct {
  double mu_gd, mu_p, beta_p, cbar_gd, cbar_p;
} rs_ihs_params;

/* Parameters from Definition 3.2 (SRHT: lambda, Lambda = 1 -+ sqrt(rho), rho in (0,1))
 * or Definition 3.1 (Gaussian: (1 -+ sqrt(c_eta rho))^2, c_eta = (1+3 sqrt(eta))^2,
 * rho in (0, 0.18], eta in (0, 0.01]) plugged into Theorem 1 (mu_gd, cbar_gd) and
 * Theorem 2 (mu_p, beta_p, cbar_p).  out: host.  RS_ERR_ARG outside the domains. */
rs_status rs_params(rs_sketch_kind kind, double rho, double eta, rs_ihs_params* out);

/* Outcomes of the step and start rules below. */
#define RS_RULE_ACCEPT_POLYAK 0  /* step: the Polyak candidate passes its test */
#define RS_RULE_ACCEPT_GD 1      /* step: the gradient candidate is taken */
#define RS_RULE_RUNNING 2        /* start: keep iterating */
#define RS_RULE_CONVERGED 3      /* start: r <= tol * r_ref already */
#define RS_RULE_DOUBLE 4         /* double m and resample */
#define RS_RULE_STUCK 5          /* both rejected at m_max, no decrease */
#define RS_RULE_NONFINITE 6      /* a decrement is NaN or infinite */
#define RS_RULE_INDEFINITE 7     /* a decrement < 0 at m_max */

/* The tests of one step of Algorithm 1 exactly as the decision kernels apply them
 * (one FP64 copy of the rule, compiled for host and device; host side exported so
 * the rule can be checked without a GPU).  Polyak candidate (decrement r_p, when
 * polyak != 0): accepted if (r_p / r_1)^(1/t) <= cbar_p; else the gradient
 * candidate (r_gd) if r_gd / r_t <= cbar_gd (ties accept); else at m_max
 * (at_cap != 0) the gradient candidate if r_gd < r_t, or STUCK; else DOUBLE.  The
 * decrement 1/2 g^T H_S^-1 g of Lemma 1 is >= 0 for the positive definite H_S of
 * eq. (3); a negative one (a factor that lost definiteness, e.g. the Woodbury
 * subtraction of a low-precision Gram at small nu^2) fails every test: DOUBLE, or
 * INDEFINITE at m_max (solves then return RS_ERR_NOT_SPD).  Returns RS_RULE_*. */
int32_t rs_step_rule(int32_t polyak, double r_p, double r_gd, double r_t, double r_1, int64_t t,
                     int32_t at_cap, double cbar_p, double cbar_gd);

/* The state right after a (re)factor, as the start and resample kernels judge it:
 * r = decrement at the current point, r_ref = the stop test's reference, both
 * under the new sketch.  NONFINITE, then DOUBLE / INDEFINITE (at_cap) for a
 * negative value, then CONVERGED if r <= tol * r_ref, else RUNNING. */
int32_t rs_start_rule(double r, double r_ref, double tol, int32_t at_cap);

/* ------------------------------------------------------------------ sketches */

/* SRHT embedding (Appendix C.2): SA = (1/sqrt(m)) R H diag(eps) A, with H the
 * Sylvester-ordered Walsh-Hadamard matrix of order npad = 2^ceil(log2 n)
 * (entries +-1; rows of A past n count as zero), eps Rademacher signs and R the
 * m rows with the smallest Philox4x32-10 keys, drawn without replacement
 * (Theorem 10's sampling rule).  Randomness: key (seed), counter
 * (row, 0, stream, sketch_id) with stream 4 = signs (eps_i = 1 - 2 (w0 & 1)) and
 * stream 5 = row keys (w1 * 2^32 + w0; ties broken by row index).
 *   A    : n x d, dtype a_t in {F64, F32}, leading dimension lda.
 *   m    : 1 <= m <= npad; npad <= 2^22.
 *   SA   : m x d output, dtype sa_t (F64 only with F64 A; F32; BF16; FP8E4M3),
 *          leading dimension ldsa >= d.  Row k is sampled row rows[k]; rows are
 *          in ascending order.
 *   sa_col_scale : FP8 only (d floats, else NULL): SA = fp8 value * scale[j],
 *          per column, a power of two chosen from the column's max.
 *   rows_out  : NULL or m int64 (ascending sampled rows).
 *   signs_out : NULL or npad int8 (+-1).
 * Asynchronous. */
rs_status rs_sketch_srht(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda,
                         int64_t m, uint64_t seed, uint32_t sketch_id,
                         void* SA, rs_dtype sa_t, int64_t ldsa, float* sa_col_scale,
                         int64_t* rows_out, int8_t* signs_out, hipStream_t stream);

/* Gaussian embedding (Section 1): SA = S A with S[k][j] = z_{k n + j} / sqrt(m),
 * z standard normal by Box-Muller from Philox4x32-10 counter (k n + j, stream 6,
 * sketch_id):  F64 path: u1 = ((w0>>6) 2^26 + (w1>>6) + 1/2) 2^-52, u2 likewise
 * from (w2, w3); F32 path: u1 = ((w0>>9) + 1/2) 2^-23, u2 = ((w1>>9) + 1/2) 2^-23;
 * z = sqrt(-2 ln u1) cos(2 pi u2).  S is generated tile by tile and never stored.
 *   m: 1 <= m <= n.  Other arguments as for rs_sketch_srht.  Asynchronous. */
rs_status rs_sketch_gaussian(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda,
                             int64_t m, uint64_t seed, uint32_t sketch_id,
                             void* SA, rs_dtype sa_t, int64_t ldsa, float* sa_col_scale,
                             hipStream_t stream);

/* ------------------------------------------------------------------ factor */

typedef struct rs_factor rs_factor;

/* Factor the sketched Hessian H_S = (SA)^T SA + nu^2 I (eq. (3))
 * for repeated solves.  m < d: Woodbury identity through the m x m matrix
 * nu^2 I_m + SA SA^T = L L^T (proof of Theorem 7); the handle keeps the whitened
 * sketch C = L^-1 SA (m x d, FP64) and applies H_S^-1 g = (g - C^T (C g)) / nu^2,
 * O(m d) per apply and m d doubles of memory (no d x d inverse).  m >= d: the
 * d x d matrix itself, applied through its explicit FP64 inverse.  The Gram is
 * accumulated in FP32 (FP64 for F64 SA) on the matrix cores, the Cholesky factor
 * and its triangular inverse are FP64.
 *   SA    : m x d device array, read during this call only.
 *   nu2   : > 0.
 *   out   : host pointer receiving a handle; release with rs_factor_destroy.
 * Synchronizes the stream (checks the pivots); RS_ERR_NOT_SPD on a failed pivot. */
rs_status rs_factor_woodbury(const void* SA, rs_dtype sa_t, const float* sa_col_scale,
                             int64_t m, int64_t d, int64_t ldsa, double nu2,
                             rs_factor** out, hipStream_t stream);

/* gtilde = H_S^-1 g for k right-hand sides, and r[c] = 1/2 g_c^T gtilde_c (the
 * sketched Newton decrement of Lemma 1).  g, gtilde: d x k FP64 (column after
 * column); r: k FP64 on the device.  All accumulation in FP64.  Asynchronous. */
rs_status rs_factor_apply(const rs_factor* F, const double* g, double* gtilde, double* r,
                          int64_t k, hipStream_t stream);

void rs_factor_destroy(rs_factor* F);

/* ------------------------------------------------------------------ gradient */

/* G = A^T (A X - b) + nu^2 X for k right-hand sides (from eq. (1)), in one
 * read of A.  X, G: d x k FP64; b: n entries of A's dtype.  Row residuals are
 * formed in A's precision; the A^T r sums are accumulated in FP64 (FP32 over
 * groups of at most 8 rows for FP32 A).  k in 1..4.  Asynchronous. */
rs_status rs_gradient(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda,
                      const void* b, double nu2, const double* X, int64_t k, double* G,
                      hipStream_t stream);

/* The gradients of two problems that share A and b (two nu, or two starting
 * points), each with a block of two iterates, in one read of A:
 * G_j = A^T (A X_j - b) + nu2[j] X_j for j = 0, 1.  The proof of Theorem 7 prices
 * an iteration at these products; two solves on the same data share them.  Each
 * G_j equals rs_gradient(A, F32, ..., nu2[j], X_j, k = 2) bit for bit.  FP32 A
 * only, and only where the k = 2 gradient plan of (n, d) runs on the 512-thread
 * kernel (a plan rs_gradient_autotune picks for wide rows, or one set with
 * rs_gradient_set_plan); otherwise RS_ERR_UNSUPPORTED and nothing is queued.
 *   nu2    : host, 2 values.
 *   X0, X1 : device, 2 x d FP64 each (column after column).
 *   G0, G1 : device, 2 x d FP64 out.
 * Asynchronous. */
rs_status rs_gradient_two(const float* A, int64_t n, int64_t d, int64_t lda, const float* b,
                          const double* nu2, const double* X0, const double* X1, double* G0,
                          double* G1, hipStream_t stream);

/* rs_gradient for callers that cannot allocate device memory (code under HIP
 * graph capture, serving loops, harnesses that forbid hipMalloc): the same kernels
 * and the same result as rs_gradient (bit for bit when the grid is the same), with
 * the per-block FP64 partial sums in a fixed array of 8 Mi doubles (64 MiB) that
 * the library holds on each device it runs on until the process ends; the call
 * itself allocates nothing.  The array's device address is looked up once per
 * device (first call with that device current).  Arguments, layout and limits as
 * rs_gradient; RS_ERR_SHAPE when k * d exceeds the array (it cannot for the built
 * d <= 8192, k <= 4), and the grid is capped at 8 Mi / (k d) blocks.  Every call
 * on one device shares the array: calls that overlap on a device (two host threads,
 * or two streams with no ordering between them) race on it and must be
 * serialized by the caller.  Each call overwrites every partial sum it reads, so
 * nothing needs clearing between calls.  Asynchronous. */
rs_status rs_gradient_noalloc(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda,
                              const void* b, double nu2, const double* X, int64_t k, double* G,
                              hipStream_t stream);

/* ------------------------------------------------------------------ iteration */

typedef struct {
  double* x;        /* device, d: x_t                                   */
  double* x_prev;   /* device, d: x_{t-1}                               */
  double* g;        /* device, d: grad f(x_t)                           */
  double* gtilde;   /* device, d: H_S^-1 g_t                            */
  double r_t;       /* host: 1/2 g_t^T gtilde_t                         */
  double r_1;       /* host: r at the first iterate                     */
  int64_t t;        /* host: step index, starting at 1                  */
} rs_ihs_state;

typedef struct {
  int32_t accepted; /* 0: Polyak candidate, 1: gradient candidate, -1: both rejected */
  double r_p;       /* decrement at the Polyak candidate (NaN for GD_ONLY) */
  double r_gd;      /* decrement at the gradient candidate */
} rs_step_result;

/* Autotuner of the gradient pass (the step's dominant kernel): times every built
 * partial-sum shape that covers d (threads per row x 16-byte vectors per thread)
 * at 1, 2 and 4 blocks per CU on this problem (k right-hand sides) and keeps the
 * fastest for (dtype, n rounded up to a power of two, d, k); later gradients of
 * that key, including those inside the solvers, use it.  The shapes include
 * deeper row batches per step (more loads in flight).  plan: NULL or 4 host
 * int32 (threads per row, vectors per thread, blocks, rows per group and step).
 * Synchronizes.  Without tuning the shape follows d and the grid is 2 blocks
 * per CU. */
rs_status rs_gradient_autotune(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda,
                               const void* b, int64_t k, int32_t* plan, hipStream_t stream);

/* The plan the gradient pass uses for this key (tuned or default). */
rs_status rs_gradient_plan(rs_dtype a_t, int64_t n, int64_t d, int64_t k, int32_t* plan);

/* Fix the plan of a key (dtype, n rounded up to a power of two, d, k) without
 * timing, e.g. one tuned earlier and stored by the caller.  plan: 4 host int32 as
 * returned by rs_gradient_autotune.  RS_ERR_UNSUPPORTED for a shape that is not
 * built, RS_ERR_SHAPE for one that does not cover d (or exceeds it more than 4x),
 * RS_ERR_ARG for a grid outside [1, 4 blocks per CU].  Host only. */
rs_status rs_gradient_set_plan(rs_dtype a_t, int64_t n, int64_t d, int64_t k,
                               const int32_t* plan);

/* One step of Algorithm 1 under a fixed factor: candidates
 * x_p = x_t - mu_p g~_t + beta_p (x_t - x_{t-1}) and x_gd = x_t - mu_gd g~_t, their
 * gradients in one pass over A, their decrements, then the tests
 * (r_p / r_1)^(1/t) <= cbar_p, else r_gd / r_t <= cbar_gd (ties accept).  On
 * acceptance the state moves to the accepted candidate (t += 1); when both are
 * rejected the state is left unchanged and the caller is expected to double m,
 * refactor and recompute gtilde_t and r_t.  Synchronizes the stream. */
rs_status rs_ihs_step(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda,
                      const void* b, double nu2, const rs_factor* F, const rs_ihs_params* p,
                      rs_variant variant, rs_ihs_state* st, rs_step_result* out,
                      hipStream_t stream);

/* ------------------------------------------------------------------ solver */

#define RS_MAX_EVENTS 512

typedef struct {
  rs_sketch_kind kind;       /* default SRHT */
  rs_variant variant;        /* default POLYAK */
  rs_resample resample;      /* default FRESH */
  rs_dtype sketch_dtype;     /* storage of SA: F64 (F64 A only), F32, BF16, FP8E4M3 */
  double rho;                /* default 0.1 */
  double eta;                /* default 0.01 (Gaussian only) */
  int64_t m_init;            /* default 1 */
  int64_t m_max;             /* 0: padded n (SRHT) or n (Gaussian) */
  double tol;                /* stop when r_t <= tol * r_ref; default 1e-7 */
  int64_t max_iter;          /* cap on accepted steps; default 200 */
  uint64_t seed;
  int32_t check_every;       /* steps queued between host reads of the device state; default 4 */
  int32_t flags;             /* RS_SOLVE_* bits; default 0 */
} rs_solve_opts;

/* rs_solve_opts.flags: replay each job's queued steps from HIP graphs captured on
 * the job's first use (batched solves only; the capture and instantiation are
 * paid once per solve, so this pays off when a solve takes many step rounds). */
#define RS_SOLVE_GRAPH_STEPS 1
/* rs_solve_opts.flags: take the stop test's reference from the origin,
 * r_ref = 1/2 g(0)^T H_S^-1 g(0) with g(0) = -A^T b (re-evaluated under each new
 * sketch), instead of from the starting point.  A warm-started solve then stops at
 * the relative accuracy delta(x) / delta(0) <= tol a cold one reaches (Section 4,
 * warm starts along a regularization path).  g(0) is one more column of the
 * first gradient pass.  A start at the origin is unchanged by the flag. */
#define RS_SOLVE_REF_AT_ZERO 2
/* rs_solve_opts.flags: time the solve's phases on its stream with HIP events
 * (rs_adaptive_solve and its CSR, dual and learned forms, the batch forms,
 * rs_refreshed_ihs and rs_solve_path; rs_solve_nu_grid leaves the fields 0)
 * into rs_solve_info.ms_sketch (every sketch the run
 * forms), ms_factor (every Gram and factor) and ms_iterate (the rest of the
 * run's GPU time line: gradients, applies, decisions, the learned start's
 * features, and the waits between them), in milliseconds.  Off by default (the
 * events add packets to the stream). */
#define RS_SOLVE_TIMING 4
/* rs_solve_opts.flags, rs_solve_nu_grid only: run each window of check_every
 * steps of all nu (candidates, the multi-right-hand-side gradient, the apply,
 * the decision) as one cooperative persistent launch with grid-wide barriers
 * between the phases, instead of four launches per step (batching form; the
 * results are the same bit for bit).  The host still resamples and factors
 * between windows. */
#define RS_SOLVE_PERSISTENT 8

/* Event kinds recorded in rs_solve_info. */
#define RS_EVENT_POLYAK 0
#define RS_EVENT_GD 1
#define RS_EVENT_DOUBLE 2

typedef struct {
  rs_status status;
  int32_t reserved;
  int64_t m_final, doublings, steps, grad_passes, applies;
  int64_t accepted_polyak, accepted_gd;
  double r_final, r_ref;
  int64_t n_events;                     /* min(#events, RS_MAX_EVENTS) */
  int32_t event_kind[RS_MAX_EVENTS];    /* RS_EVENT_* in order */
  int32_t event_t[RS_MAX_EVENTS];       /* step index t of each event */
  int64_t event_m[RS_MAX_EVENTS];       /* sketch size after the event */
  double ms_sketch, ms_factor, ms_iterate; /* phase times under RS_SOLVE_TIMING, else 0 */
} rs_solve_info;

/* Fill opts with the defaults listed above. */
void rs_solve_opts_default(rs_solve_opts* opts);

/* Algorithm 1 end to end (Section 3): start at m = m_init, double m and resample
 * whenever both candidates fail their tests, stop at r_t <= tol * r_ref with
 * r_ref = 1/2 g_1^T H_S^-1 g_1 under the current sketch (g(0) in place of g_1
 * under RS_SOLVE_REF_AT_ZERO).  The step control runs on the device; the host reads a small
 * state record every check_every steps and performs the resamplings.
 *   A, b   : problem (F64 or F32); nu2 > 0.
 *   x      : device, d FP64: in = initial point x_1 (= x_0), out = solution.
 *   info   : host.
 * Synchronizes the stream.  Returns RS_OK, RS_ERR_NO_CONVERGENCE (x holds the
 * last iterate) or an error. */
rs_status rs_adaptive_solve(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda,
                            const void* b, double nu2, const rs_solve_opts* opts,
                            double* x, rs_solve_info* info, hipStream_t stream);

/* One problem of a batch: A (n x d, row-major, leading dimension lda, F32 or F64,
 * 16-byte aligned), b (n, same type), nu2 > 0, x (d FP64: in = x_1, out =
 * solution).  All device pointers, owned by the caller. */
typedef struct rs_problem {
  const void* A;
  rs_dtype a_t;
  int32_t reserved;
  int64_t n, d, lda;
  const void* b;
  double nu2;
  double* x;
} rs_problem;

/* Many independent ridge problems of any sizes, each solved by Algorithm 1 with
 * the same opts (result i identical to rs_adaptive_solve on problem i, whose
 * arithmetic does not depend on how jobs are scheduled).  The library multiplexes
 * the jobs over `workers` streams of its own (default priority; 0 = 8), each with
 * private scratch; the host advances a job whenever its last queued work has
 * finished, so small solves run concurrently and fill the device.  The worker
 * streams wait for work already queued on `stream`, and `stream` waits for all of
 * them on return.  Workers past the first run on host threads that the library
 * starts on first use and keeps until the process ends.  Jobs on the same FP32 A
 * and b (the same pointers, shape and lda; e.g. several nu of one data set) run as
 * pairs when the k = 2 gradient plan of (n, d) is on the 512-thread kernel: one host
 * thread drives both on two worker streams, each step the two jobs have in common
 * takes one gradient pass for both (rs_gradient_two), a learned start forms the
 * features' pass over A once (with learned starts and the SRHT, that pass also runs
 * the first pass of the two first sketches' transform), and the two first sketches
 * come from one transform; the results are those of the jobs alone, bit for bit.
 * infos: count host records.  Synchronizes.  Returns RS_OK when
 * every job ended RS_OK or RS_ERR_NO_CONVERGENCE (see infos[i].status), else the
 * first other error; an argument error in any problem is reported before any
 * work is queued. */
rs_status rs_solve_batch(const rs_problem* probs, int64_t count, const rs_solve_opts* opts,
                         rs_solve_info* infos, int32_t workers, hipStream_t stream);

/* Algorithm 1 for count values nu2[k] (host array, each > 0) on one (A, b), with
 * one option set.  The sketch of level m = m_init 2^L (sketch_id L when fresh, 0
 * when nested: what a single solve draws at that level) and its Gram do not
 * depend on nu (Section 3), so they are formed once per level and shared; each
 * nu keeps its own shifted FP64 factor, state and doubling ladder.  The
 * gradients of all candidates of all running nu come from one multi-RHS product
 * per step (matrix cores).  X: device, count x d FP64 row-major: in = x_1 of each
 * nu, out = solutions.  infos: count host records, filled as rs_adaptive_solve
 * fills one.  Synchronizes.  Returns RS_OK when every nu ended RS_OK or
 * RS_ERR_NO_CONVERGENCE, else the first other error.  Memory: count d^2 doubles
 * of factors plus the level cache. */
rs_status rs_solve_nu_grid(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda,
                           const void* b, const double* nu2, int64_t count,
                           const rs_solve_opts* opts, double* X, rs_solve_info* infos,
                           hipStream_t stream);

/* Sparse A (the remark on sparse data matrices, which names O(nnz) embeddings
 * and leaves them open): Algorithm 1 with the CountSketch, S[h_i, i] = s_i, bucket
 * h_i = high word of (Philox word0 * m) and sign s_i from word1 (stream 8, counter
 * (i, sketch_id), key seed).  Forming SA and the gradient cost O(nnz); the step
 * sizes are the SRHT's for the same rho (the paper gives none); under NESTED
 * resampling a doubling splits every bucket in two, under FRESH it re-hashes.
 * m is capped at n (or opts->m_max).  opts->kind must be RS_SKETCH_COUNT;
 * sketch_dtype F64 (F64 values), F32 or BF16.  The library forms a column-major
 * copy of A once per call (nnz indices and values) for the A^T r pass; every sum
 * runs in a fixed order (no floating-point atomics).
 *   rowptr : device, n + 1 int64, rowptr[0] = 0, rowptr[n] = nnz, non-decreasing.
 *   col    : device, nnz int32 in [0, d), distinct within a row (a repeated
 *            column within a row gives an unspecified sketch).
 *   val    : device, nnz values of type a_t (F32 or F64).
 *   b      : device, n values of type a_t.   x: device, d FP64 in = x_1, out.
 * n >= d, n and nnz below 2^31, d <= 8192.  Synchronizes.  Returns RS_OK,
 * RS_ERR_NO_CONVERGENCE, RS_ERR_ARG for a malformed CSR (checked on the device
 * before any other work), or another error. */
rs_status rs_adaptive_solve_csr(const int64_t* rowptr, const int32_t* col, const void* val,
                                rs_dtype a_t, int64_t n, int64_t d, int64_t nnz, const void* b,
                                double nu2, const rs_solve_opts* opts, double* x,
                                rs_solve_info* info, hipStream_t stream);

/* IHS with refreshed embeddings (Section 1, other versions of the IHS), an
 * ablation of the fixed sketch: the update of eq. (2) (beta = 0 for
 * RS_VARIANT_GD) with a new sketch of fixed size m = opts->m_init (clamped to the
 * padded n, SRHT, or n, Gaussian) drawn at every step t (sketch_id t - 1) and
 * H_S re-formed; the step sizes are the fixed-embedding ones for (kind, rho, eta);
 * no acceptance tests, no doubling.  Stops at r_t <= tol * r_1, with r_t the
 * decrement under step t's sketch, or after max_iter updates.  opts->resample,
 * check_every and flags are ignored.
 *   x      : device, d FP64: in = x_1 (= x_0), out = last iterate.
 *   r_hist : host, max_iter + 1 doubles or null: r_1, r_2, ... (info->grad_passes
 *            of them are written).
 *   info   : host; steps = updates taken, grad_passes = decrements evaluated,
 *            r_ref = r_1, m_final = m, no events.
 * Synchronizes every step.  Returns RS_OK, RS_ERR_NO_CONVERGENCE, or an error. */
rs_status rs_refreshed_ihs(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda,
                           const void* b, double nu2, const rs_solve_opts* opts, double* x,
                           double* r_hist, rs_solve_info* info, hipStream_t stream);

/* The underdetermined case n <= d (appendix, the dual problem): Algorithm 1 on
 * min_z 1/2 |A^T z - b^|^2 + nu^2/2 |z|^2 with b^ = A^+ b, whose data matrix is A^T
 * (the sketch acts on its d rows, m <= padded d) and whose gradient is
 * A A^T z - b + nu^2 z (b^ is never formed); the primal solution is x = A^T z.
 * The library forms A^T once (d x n, row-major, in its own scratch: d * n elements
 * of A's type), then runs the solver of rs_adaptive_solve on it; every option of
 * rs_adaptive_solve applies (RS_SOLVE_GRAPH_STEPS has no effect), and info
 * describes the dual run (its r values are dual decrements).
 *   A, b   : problem (F64 or F32), A n x d with n <= d; nu2 > 0.
 *   z      : device, n FP64: in = initial dual point (zeros for a cold start),
 *            out = dual solution.
 *   x      : device, d FP64, out = A^T z (also after RS_ERR_NO_CONVERGENCE).
 * Synchronizes.  Returns RS_OK, RS_ERR_NO_CONVERGENCE, RS_ERR_SHAPE when n > d, or
 * another error. */
rs_status rs_adaptive_solve_dual(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda,
                                 const void* b, double nu2, const rs_solve_opts* opts, double* z,
                                 double* x, rs_solve_info* info, hipStream_t stream);

/* Regularization path (Section 4, warm starts): Algorithm 1 for count values
 * nu2[k] (host array, each > 0, non-increasing) on one (A, b), one after another.
 * Solve k starts at solution k - 1 and at its final sketch size (m_init of solve 0
 * is opts->m_init), with nested resampling (a sketch of size m is the first m rows
 * of one sketch family, so the transformed A of the SRHT, or the Gaussian rows
 * already drawn, serve the whole path) and RS_SOLVE_REF_AT_ZERO set: every solve
 * stops at the relative accuracy tol measured from the origin.  Solve k starts at
 * the sketch solve k - 1 ended with; that sketch and its Gram do not depend on nu
 * (Section 3), so only the shifted FP64 factor is formed again.  opts->resample is
 * ignored (nested) and RS_SOLVE_GRAPH_STEPS has no effect.
 *   X     : device, count x d FP64 row-major: in = row 0 holds the first start
 *           (zeros for a cold path; rows 1.. are overwritten), out = row k the
 *           solution at nu2[k].
 *   infos : count host records, each filled as rs_adaptive_solve fills one.
 * Result k equals rs_adaptive_solve at nu2[k] started at row k - 1 with
 * m_init = infos[k - 1].m_final, nested resampling and RS_SOLVE_REF_AT_ZERO.
 * Synchronizes.
 * Returns RS_OK when every solve ended RS_OK or RS_ERR_NO_CONVERGENCE (then its
 * row holds the last iterate and the path goes on from it), RS_ERR_ARG for an
 * increasing nu2, else the first other error (rows past the failing solve are
 * left as they were). */
rs_status rs_solve_path(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda,
                        const void* b, const double* nu2, int64_t count,
                        const rs_solve_opts* opts, double* X, rs_solve_info* infos,
                        hipStream_t stream);

/* ------------------------------------------------------------------ learned start */

/* Algorithm 1 holds for any initial sketch size (Theorems 5 and 6).  The learned
 * form predicts log2 of the final sketch size of a plain run from 16 features and
 * starts the doubling ladder at m_init = 2^floor(prediction); the adaptive rule
 * stays as the fallback.  The predictor is a 16 -> 128 -> 128 -> 1 MLP with exact
 * GELU, FP32, parameters in one flat array:
 *   W1 [16][128] at 0, b1 [128] at 2048, W2 [128][128] at 2176, b2 [128] at 18560,
 *   W3 [128] at 18688, b3 at 18816 (RS_MLP_PARAMS floats). */
#define RS_MLP_FEATURES 16
#define RS_MLP_PARAMS 18817
#define RS_MLP_CACHE 273   /* floats per sample kept by the forward pass */
#define RS_MLP_WORK 257    /* floats per sample used by the backward pass */

/* Features of (A, nu^2), 16 floats on the device (feat):
 *   log2 n, log2 d, log10 nu^2;
 *   ln q_k, k = 0..7, q_k = (A^T w_k)^T H_S0^-1 (A^T w_k) with w_k Rademacher
 *     (Philox stream 7, sketch_id k, counter = row) and H_S0 the sketched Hessian of
 *     a min(256, padded n)-row SRHT (seed, sketch_id 0x7fff0000): a Hutchinson
 *     estimate of the effective dimension tr(A H^-1 A^T);
 *   order statistics at round(q (d-1)), q = 0, 1/4, 1/2, 3/4, 1, of ln ||A e_j||.
 * d <= 8192.  Asynchronous. */
rs_status rs_features(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda,
                      double nu2, uint64_t seed, float* feat, hipStream_t stream);

/* y[s] = MLP((X[s] - mu) / sd) for B samples (X: B x 16, mu, sd: 16; all device
 * FP32).  cache: NULL or B * RS_MLP_CACHE floats kept for rs_mlp_backward. */
rs_status rs_mlp_forward(const float* params, const float* X, int64_t B, const float* mu,
                         const float* sd, float* y, float* cache, hipStream_t stream);

/* Gradient of the loss mean_s (y_s - t_s)^2 with respect to every parameter
 * (grad: RS_MLP_PARAMS floats), from the forward cache.  loss: NULL or one device
 * float.  work: B * RS_MLP_WORK floats of scratch.  Sums over the batch run in a
 * fixed order (deterministic).  Asynchronous. */
rs_status rs_mlp_backward(const float* params, const float* cache, const float* t, int64_t B,
                          float* grad, float* loss, float* work, hipStream_t stream);

/* One Adam step (bias-corrected; step counts from 1) on count parameters. */
rs_status rs_mlp_adam_step(float* params, const float* grad, float* m, float* v, int64_t count,
                           int64_t step, float lr, float beta1, float beta2, float eps,
                           hipStream_t stream);

/* Features -> MLP -> m_init = clamp(2^floor(y), 1, m_max) -> rs_adaptive_solve with
 * opts->m_init replaced.  m_init_used: host, may be NULL.  Synchronizes. */
/* The batched form of rs_learned_solve: each problem's features and prediction
 * run on its worker stream, then its Algorithm 1 run starts at the predicted m
 * (fallback: the doubling rule).  m_init_used: NULL or count host int64.  Same
 * scheduling, synchronization and return rules as rs_solve_batch. */
rs_status rs_learned_solve_batch(const rs_problem* probs, int64_t count, const rs_solve_opts* opts,
                                 const float* params, const float* mu, const float* sd,
                                 rs_solve_info* infos, int64_t* m_init_used, int32_t workers,
                                 hipStream_t stream);

rs_status rs_learned_solve(const void* A, rs_dtype a_t, int64_t n, int64_t d, int64_t lda,
                           const void* b, double nu2, const rs_solve_opts* opts,
                           const float* params, const float* mu, const float* sd, double* x,
                           rs_solve_info* info, int64_t* m_init_used, hipStream_t stream);

/* ------------------------------------------------------------------ timing */

/* Diagnostics for measuring the dominant kernel (not part of the method).
 * While enabled, every launch of the gradient's partial-sum kernel (the pass
 * over A) is bracketed by two HIP events recorded on the stream it is launched
 * on, and the kernel raises a device flag when it does its work (launches
 * queued behind a raised status flag return at once and are not counted).
 * rs_profile_read synchronizes the device, returns the number of launches that
 * did their work and their summed duration in milliseconds (host pointers),
 * and clears the record.  At most 65536 launches are recorded between reads.
 * Not thread-safe. */
rs_status rs_profile_enable(int on);
rs_status rs_profile_read(int64_t* launches, double* total_ms);

/* Message describing the last error on the calling thread ("" if none). */
const char* rs_last_error(void);

/* Library version string. */
const char* rs_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RS_H_ */
