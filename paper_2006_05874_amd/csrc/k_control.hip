// Step control of Algorithm 1 on the device.
//
// One step = candidates -> gradient (one pass over A for both candidates) ->
// apply -> decide.  The decision kernel applies the two ratio tests in FP64,
// moves the state to the accepted candidate, records the event, and raises a
// status flag (converged / double m / stuck / step cap / non-finite) that makes
// every later kernel of the queued steps return at once.  The host therefore
// queues several steps, reads the small control record, and only intervenes to
// resample.
#include "rs_internal.hpp"

namespace rs {

// X[0] = x - mu_p gt + beta_p (x - x_prev), X[K-1] = x - mu_gd gt (K = 2);
// K = 1 (gradient-only): X[0] = x - mu_gd gt.  One element; every kernel that
// writes candidates goes through here, so they agree bit for bit.
__device__ __forceinline__ void candidate_at(int K, int64_t d, int64_t i, double xi, double xpi,
                                             double gi, double* __restrict__ X, double mu_p,
                                             double beta_p, double mu_gd) {
  if (K == 2) {
    X[i] = xi - mu_p * gi + beta_p * (xi - xpi);
    X[d + i] = xi - mu_gd * gi;
  } else {
    X[i] = xi - mu_gd * gi;
  }
}

template <int K>
__global__ __launch_bounds__(256) void k_candidates(int64_t d, const double* __restrict__ x,
                                                    const double* __restrict__ x_prev,
                                                    const double* __restrict__ gt,
                                                    double* __restrict__ X, double mu_p,
                                                    double beta_p, double mu_gd,
                                                    const int* __restrict__ status) {
  if (status && *status != 0) return;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < d; i += (int64_t)gridDim.x * 256)
    candidate_at(K, d, i, x[i], x_prev[i], gt[i], X, mu_p, beta_p, mu_gd);
}

struct DecideArgs {
  double mu_p, beta_p, mu_gd, cbar_p, cbar_gd, tol;
  int64_t max_iter;
  int32_t polyak;  // variant has a Polyak candidate (K = 2)
};

// Thread 0, after it changed the record: the copy for the host (system-scope
// release, so it is visible once the kernel has completed).
__device__ __forceinline__ void publish(const DevCtl* ctl, const CtlSnap& sn) {
  if (!sn.host) return;
  *reinterpret_cast<DevCtl*>(sn.host) = *ctl;
  *reinterpret_cast<int*>(reinterpret_cast<char*>(sn.host) + kSnapFlagOff) =
      sn.flag ? *sn.flag : 0;
  __threadfence_system();
}

// The decision on one block of NT threads.  rpart: nrp x K partial sums of
// g^T gtilde.  With next set, an accepted step that leaves the state running also
// writes the next step's candidates into X (from the new x, the old x and the new
// gtilde).
template <int K, int NT>
__device__ __forceinline__ void decide_body(DevCtl* __restrict__ ctl,
                                            const double* __restrict__ rpart, int nrp,
                                            const DecideArgs& a, int64_t d,
                                            double* __restrict__ X, const double* __restrict__ G,
                                            const double* __restrict__ GT,
                                            double* __restrict__ x, double* __restrict__ x_prev,
                                            double* __restrict__ g, double* __restrict__ gt,
                                            int32_t* __restrict__ ev_kind, int ev_cap, bool next,
                                            const CtlSnap& sn) {
  __shared__ double r[K];
  __shared__ double sh[NT * K];
  __shared__ int chosen, run_next;
  block_sum_cols<K, NT>(rpart, nrp, sh, r);
  if (threadIdx.x < K) r[threadIdx.x] *= 0.5;
  __syncthreads();
  if (threadIdx.x == 0) {
    int st = RS_CTL_RUNNING;
    const int64_t t = ctl->t;
    ctl->passes += 1;
    const bool pk = a.polyak && K == 2;
    const int rule = step_rule(pk, r[0], r[K - 1], ctl->r_t, ctl->r_1, t, ctl->at_cap, a.cbar_p,
                               a.cbar_gd, &st);
    const int c = rule == 0 ? 0 : (rule == 1 ? K - 1 : -1);
    if (c >= 0) {
      const int kind = (a.polyak && c == 0) ? 0 : 1;
      if (t < ev_cap) ev_kind[t] = kind;
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
    run_next = next && c >= 0 && st == RS_CTL_RUNNING;
    publish(ctl, sn);
  }
  __syncthreads();
  const int c = chosen;
  if (c < 0) return;
  const bool nx = run_next != 0;
  for (int64_t i = threadIdx.x; i < d; i += NT) {
    const double xi = x[i];
    const double xn = X[(int64_t)c * d + i];
    const double gtn = GT[(int64_t)c * d + i];
    x_prev[i] = xi;
    x[i] = xn;
    g[i] = G[(int64_t)c * d + i];
    gt[i] = gtn;
    if (nx) candidate_at(K, d, i, xn, xi, gtn, X, a.mu_p, a.beta_p, a.mu_gd);
  }
}

// Single block.  With next set the decision also writes the next step's
// candidates (the step then needs no separate candidate launch).
template <int K>
__global__ __launch_bounds__(1024) void k_decide(DevCtl* __restrict__ ctl,
                                                 const double* __restrict__ rpart, int nrp,
                                                 DecideArgs a, int64_t d, double* __restrict__ X,
                                                 const double* __restrict__ G,
                                                 const double* __restrict__ GT,
                                                 double* __restrict__ x, double* __restrict__ x_prev,
                                                 double* __restrict__ g, double* __restrict__ gt,
                                                 int32_t* __restrict__ ev_kind, int ev_cap,
                                                 int next, CtlSnap sn) {
  if (ctl->status != RS_CTL_RUNNING) return;
  decide_body<K, 1024>(ctl, rpart, nrp, a, d, X, G, GT, x, x_prev, g, gt, ev_kind, ev_cap,
                       next != 0, sn);
}

// After the first gradient and apply: g <- G[0], gtilde <- GT[0], x_prev <- x,
// r_t = r_1 = r.  With C = 1 the start is its own reference (g_ref <- G[0],
// r_ref = r_1); with C = 2 column 1 holds the gradient at the origin and its
// decrement (g_ref <- G[1], r_ref from the second sum).
template <int C>
__global__ __launch_bounds__(1024) void k_init_state(DevCtl* __restrict__ ctl,
                                                     const double* __restrict__ rpart, int nrp,
                                                     double tol, int64_t max_iter, int64_t d,
                                                     const double* __restrict__ G,
                                                     const double* __restrict__ GT,
                                                     const double* __restrict__ x,
                                                     double* __restrict__ x_prev,
                                                     double* __restrict__ g,
                                                     double* __restrict__ gt,
                                                     double* __restrict__ gref, int at_cap,
                                                     NextCand nc, CtlSnap sn) {
  __shared__ double sh[C * 1024];
  __shared__ double rs1[C];
  __shared__ int run;
  block_sum_cols<C, 1024>(rpart, nrp, sh, rs1);
  if (threadIdx.x == 0) {
    const double r = 0.5 * rs1[0];
    const double rr = 0.5 * rs1[C - 1];
    ctl->r_t = r;
    ctl->r_1 = r;
    ctl->r_ref = rr;
    ctl->t = 1;
    ctl->steps = 0;
    ctl->passes = 1;
    ctl->polyak = 0;
    ctl->gd = 0;
    ctl->at_cap = at_cap;
    int st = start_rule(r, rr, tol, at_cap);
    if (st == RS_CTL_RUNNING && 1 >= max_iter) st = RS_CTL_MAXITER;
    ctl->status = st;
    run = nc.X != nullptr && st == RS_CTL_RUNNING;
    publish(ctl, sn);
  }
  __syncthreads();
  const bool nx = run != 0;
  for (int64_t i = threadIdx.x; i < d; i += 1024) {
    const double xi = x[i], gti = GT[i];
    x_prev[i] = xi;
    g[i] = G[i];
    gref[i] = G[(C - 1) * d + i];
    gt[i] = gti;
    if (nx) candidate_at(nc.K, d, i, xi, xi, gti, nc.X, nc.mu_p, nc.beta_p, nc.mu_gd);
  }
}

// After a resample: apply was run on [g_t, g_ref] -> GT; rpart holds 2 sums.
__global__ __launch_bounds__(1024) void k_post_resample(DevCtl* __restrict__ ctl,
                                                        const double* __restrict__ rpart, int nrp,
                                                        double tol, int64_t d,
                                                        const double* __restrict__ GT,
                                                        double* __restrict__ gt, int at_cap,
                                                        NextCand nc,
                                                        const double* __restrict__ x,
                                                        const double* __restrict__ x_prev,
                                                        CtlSnap sn) {
  __shared__ double sh[2048];
  __shared__ double s2[2];
  __shared__ int run;
  block_sum_cols<2, 1024>(rpart, nrp, sh, s2);
  if (threadIdx.x == 0) {
    ctl->r_t = 0.5 * s2[0];
    ctl->r_ref = 0.5 * s2[1];
    ctl->at_cap = at_cap;
    const int st = start_rule(ctl->r_t, ctl->r_ref, tol, at_cap);
    // r_1 stays from the start (Algorithm 1) unless the start's own factor was
    // indefinite: then the first valid decrement takes its place
    if (st == RS_CTL_RUNNING && !(ctl->r_1 >= 0.0)) ctl->r_1 = ctl->r_t;
    ctl->status = st;
    run = nc.X != nullptr && st == RS_CTL_RUNNING;
    publish(ctl, sn);
  }
  __syncthreads();
  const bool nx = run != 0;
  for (int64_t i = threadIdx.x; i < d; i += 1024) {
    const double gti = GT[i];
    gt[i] = gti;
    if (nx) candidate_at(nc.K, d, i, x[i], x_prev[i], gti, nc.X, nc.mu_p, nc.beta_p, nc.mu_gd);
  }
}

// IHS with refreshed embeddings, after the gradient and the apply of evaluation t
// under that step's own sketch: r_t = 1/2 g_t^T gtilde_t (r_1 kept from t = 1,
// r_t stored at rhist[t - 1]); stop at r_t <= tol r_1 (or after max_iter updates),
// else x <- x - mu gtilde + beta (x - x_prev), x_prev <- the old x, t += 1.
__global__ __launch_bounds__(1024) void k_refresh_step(DevCtl* __restrict__ ctl,
                                                       const double* __restrict__ rpart, int nrp,
                                                       int64_t d, const double* __restrict__ GT,
                                                       double* __restrict__ x,
                                                       double* __restrict__ x_prev, double mu,
                                                       double beta, double tol, int64_t max_iter,
                                                       double* __restrict__ rhist, int64_t rcap) {
  __shared__ double sh[1024];
  __shared__ double rs1[1];
  __shared__ int upd;
  block_sum_cols<1, 1024>(rpart, nrp, sh, rs1);
  if (threadIdx.x == 0) {
    const double r = 0.5 * rs1[0];
    const int64_t t = ctl->t;
    if (t == 1) ctl->r_1 = r;
    ctl->r_t = r;
    ctl->r_ref = ctl->r_1;
    if (t - 1 < rcap) rhist[t - 1] = r;
    int st = RS_CTL_RUNNING;
    if (!isfinite(r)) st = RS_CTL_NONFINITE;
    else if (r < 0.0 || !(ctl->r_1 >= 0.0)) st = RS_CTL_INDEFINITE;  // H_S^-1 lost definiteness
    else if (r <= tol * ctl->r_1) st = RS_CTL_CONVERGED;
    else if (ctl->steps >= max_iter) st = RS_CTL_MAXITER;
    ctl->status = st;
    ctl->passes += 1;
    upd = st == RS_CTL_RUNNING;
    if (upd) {
      ctl->steps += 1;
      ctl->t = t + 1;
    }
  }
  __syncthreads();
  if (!upd) return;
  for (int64_t i = threadIdx.x; i < d; i += 1024) {
    const double xi = x[i];
    const double xn = xi - mu * GT[i] + beta * (xi - x_prev[i]);
    x_prev[i] = xi;
    x[i] = xn;
  }
}

rs_status refresh_step_launch(DevCtl* ctl, const double* rpart, int nrp, int64_t d,
                              const double* GT, double* x, double* x_prev, double mu, double beta,
                              double tol, int64_t max_iter, double* rhist, int64_t rcap,
                              hipStream_t s) {
  hipLaunchKernelGGL(k_refresh_step, dim3(1), dim3(1024), 0, s, ctl, rpart, nrp, d, GT, x, x_prev,
                     mu, beta, tol, max_iter, rhist, rcap);
  return check_launch("refresh step");
}

// Copy two vectors into a 2-column block (for the post-resample apply).
__global__ __launch_bounds__(256) void k_pack2(int64_t d, const double* __restrict__ a,
                                               const double* __restrict__ b,
                                               double* __restrict__ out) {
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < d; i += (int64_t)gridDim.x * 256) {
    out[i] = a[i];
    out[d + i] = b[i];
  }
}

static unsigned vec_grid(int64_t d) { return (unsigned)std::min<int64_t>((d + 255) / 256, 1024); }

rs_status candidates_launch(int K, int64_t d, const double* x, const double* x_prev,
                            const double* gt, double* X, double mu_p, double beta_p, double mu_gd,
                            const int* status, hipStream_t s) {
  if (K == 2)
    hipLaunchKernelGGL(k_candidates<2>, dim3(vec_grid(d)), dim3(256), 0, s, d, x, x_prev, gt, X,
                       mu_p, beta_p, mu_gd, status);
  else
    hipLaunchKernelGGL(k_candidates<1>, dim3(vec_grid(d)), dim3(256), 0, s, d, x, x_prev, gt, X,
                       mu_p, beta_p, mu_gd, status);
  return check_launch("candidates");
}

rs_status decide_launch(int K, DevCtl* ctl, const double* rpart, int nrp, const CtlParams& p,
                        int64_t d, double* X, const double* G, const double* GT, double* x,
                        double* x_prev, double* g, double* gt, int32_t* ev_kind, int ev_cap,
                        hipStream_t s, bool next, CtlSnap snap) {
  DecideArgs a{p.mu_p, p.beta_p, p.mu_gd, p.cbar_p, p.cbar_gd, p.tol, p.max_iter, K == 2 ? 1 : 0};
  const int nx = next ? 1 : 0;
  if (K == 2)
    hipLaunchKernelGGL(k_decide<2>, dim3(1), dim3(1024), 0, s, ctl, rpart, nrp, a, d, X, G, GT, x,
                       x_prev, g, gt, ev_kind, ev_cap, nx, snap);
  else
    hipLaunchKernelGGL(k_decide<1>, dim3(1), dim3(1024), 0, s, ctl, rpart, nrp, a, d, X, G, GT, x,
                       x_prev, g, gt, ev_kind, ev_cap, nx, snap);
  return check_launch("decide");
}

rs_status init_state_launch(DevCtl* ctl, const double* rpart, int nrp, double tol,
                            int64_t max_iter, int64_t d, const double* G, const double* GT,
                            const double* x, double* x_prev, double* g, double* gt, double* gref,
                            int at_cap, hipStream_t s, NextCand nc, CtlSnap snap, int cols) {
  if (cols == 2)
    hipLaunchKernelGGL(k_init_state<2>, dim3(1), dim3(1024), 0, s, ctl, rpart, nrp, tol, max_iter,
                       d, G, GT, x, x_prev, g, gt, gref, at_cap, nc, snap);
  else
    hipLaunchKernelGGL(k_init_state<1>, dim3(1), dim3(1024), 0, s, ctl, rpart, nrp, tol, max_iter,
                       d, G, GT, x, x_prev, g, gt, gref, at_cap, nc, snap);
  return check_launch("init state");
}

rs_status post_resample_launch(DevCtl* ctl, const double* rpart, int nrp, double tol, int64_t d,
                               const double* GT, double* gt, int at_cap, hipStream_t s,
                               NextCand nc, const double* x, const double* x_prev,
                               CtlSnap snap) {
  if (nc.X && (!x || !x_prev)) return set_error(RS_ERR_ARG, "post resample: candidates need x");
  hipLaunchKernelGGL(k_post_resample, dim3(1), dim3(1024), 0, s, ctl, rpart, nrp, tol, d, GT, gt,
                     at_cap, nc, x, x_prev, snap);
  return check_launch("post resample");
}

rs_status pack2_launch(int64_t d, const double* a, const double* b, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_pack2, dim3(vec_grid(d)), dim3(256), 0, s, d, a, b, out);
  return check_launch("pack2");
}

}  // namespace rs
