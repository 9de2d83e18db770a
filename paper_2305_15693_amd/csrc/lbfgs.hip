// L-BFGS (Liu & Nocedal) with a cap on the step length and a backtracking line
// search (Nocedal & Wright), the optimiser the paper's main text feeds the
// configuration and gradient to, written as a device-side state machine so that one trial step -- evaluation plus optimiser update -- is
// a fixed sequence of kernels that is captured in a HIP graph and replayed
// without host synchronisation.
//
// The search direction uses the compact representation of the limited-memory
// inverse Hessian (Byrd, Nocedal & Schnabel 1994), which needs two streaming
// passes over the history instead of the 2m dependent passes of the two-loop
// recursion:
//   H g = gamma g + S u - gamma Y t,   t = R^-1 (S^T g),
//   u = R^-T ((D + gamma Y^T Y) t - gamma Y^T g),
// with S, Y the stored pairs in chronological order, R the upper triangle of
// S^T Y, D its diagonal and gamma = s.y / y.y of the newest pair.  The m x m
// products S^T Y and Y^T Y are kept in the state and updated with the new pair.
//
// Per replay, after the loss/gradient evaluation at the trial point xt, four
// kernels:
//   pass A   decision: Armijo test f(xt) <= f(x) + c1 alpha g.p -> ACCEPT or
//            REJECT (REJECT: alpha *= shrink; after max_backtracks rejections
//            the history is dropped and the search restarts along -g; a second
//            failure sets the failure flag), computed by every block from the
//            state; on ACCEPT s = alpha p, y = g(xt) - g(x) into the ring,
//            x = xt, g = g(xt), and the new dot products s_j.y, y_j.y, s_j.g,
//            y_j.g, g.g as block partials;
//   small    one block: applies the decision, reduces the partials, stores the
//            pair when y.s > 0 and solves for u, t (FP64, one wavefront);
//   pass B   p = -(gamma g + S u - gamma Y t), max |p| per block;
//   pass C   alpha = min(1, max_step / max|p|), xt = x + alpha p.
// (Cross-block steps stay at kernel boundaries: a device-scope fence per block
// writes back the L2 of its XCD and cost more than the launches it saved.)
// Vectors are in the working precision; every dot product is accumulated in FP64
// with a fixed reduction order.
#include <cmath>

#include "common.h"
#include "lbfgs.h"

namespace fresco {

enum { LB_IDLE = 0, LB_ACCEPT = 1, LB_REJECT = 2, LB_RESTART = 3, LB_INIT = 4 };

constexpr int kThreads = kLbfgsThreads;
constexpr int kWaves = kThreads / 64;

#define GRID_LOOP(i, n) \
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (long long)gridDim.x * blockDim.x)

// Reduce `cnt` per-thread values across the block (fixed order) and write them to
// part[c * nb + blockIdx.x].
template <int CNT>
__device__ __forceinline__ void block_partials(double* v, int cnt, double* part, int nb,
                                               double* sh /* [CNT][kWaves] */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < CNT; ++c) {
    if (c < cnt) {
      double x = v[c];
      for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
      if (lane == 0) sh[c * kWaves + wave] = x;
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < cnt; c += blockDim.x) {
    double t = 0.0;
    for (int w = 0; w < kWaves; ++w) t += sh[c * kWaves + w];
    part[(long long)c * nb + blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------- decide
// Decision on the evaluation just finished, as a function of the state (every
// block of pass A computes it; the small step then applies it).
__device__ __forceinline__ int lb_decided_step(const LbfgsState* S, const LbfgsOpts& o) {
  if (S->mode == LB_INIT) return LB_INIT;  // first evaluation of a call
  if (S->fail || S->iter >= S->target || S->converged) return LB_IDLE;
  const double f = S->f_trial;
  if (isfinite(f) && f <= S->f_cur + o.c1 * S->alpha * S->gtp) return LB_ACCEPT;
  if (S->nbt + 1 > o.max_backtracks) return (S->k > 0 || !S->restarted) ? LB_RESTART : LB_IDLE;
  return LB_REJECT;
}
__device__ void lb_decide(LbfgsState* S, const LbfgsOpts& o) {
  const int step = lb_decided_step(S, o);
  // an evaluation counts when it can inform a decision: replays that run after
  // the call has stopped (target reached, converged, failed) are not counted
  if (S->mode == LB_INIT || !(S->fail || S->iter >= S->target || S->converged)) S->nevals += 1;
  if (step == LB_INIT) {
    S->f_cur = S->f_trial;  // take the point as current
    S->nbt = 0;
  } else if (step == LB_ACCEPT) {
    S->f_cur = S->f_trial;
    S->iter += 1;
    S->nbt = 0;
  } else if (step == LB_RESTART) {
    S->k = 0;  // drop the history, restart along the steepest descent direction
    S->restarted = 1;
    S->resets += 1;
    S->nbt = 0;
  } else if (step == LB_REJECT) {
    S->nbt += 1;
    S->alpha *= o.shrink;
  } else if (!(S->fail || S->iter >= S->target || S->converged)) {
    S->nbt += 1;  // second line-search failure
    S->fail = 1;
  }
  S->step = step;
}

// ---------------------------------------------------------------- pass A
__device__ __forceinline__ void lb_small_update(LbfgsState* S, const LbfgsOpts& o,
                                                const double* red, int step, long long n,
                                                int* cs);
__device__ __forceinline__ void lb_small_direction(LbfgsState* S, const LbfgsOpts& o,
                                                   const int* cs);

// One block after pass A: apply the decision, reduce the partials, update the
// pair products (one thread) and solve for the direction coefficients (one
// wavefront), on an LDS copy of the state (dependent global loads would
// dominate otherwise).
__global__ void lb_small_kernel(LbfgsState* Sg, LbfgsOpts o, const double* part, int nb,
                                long long n) {
  __shared__ double red[4 * kLbfgsMaxM + 1];
  __shared__ LbfgsState sh;
  __shared__ int cs[kLbfgsMaxM];
  static_assert(sizeof(LbfgsState) % 4 == 0, "state copied as 32-bit words");
  constexpr int kWords = (int)(sizeof(LbfgsState) / 4);
  const int m = o.m;
  // value c is reduced by wave c mod (waves): lane l sums the partials l,
  // l + 64, ... (nb <= 1024: at most 16).  With at most three values per wave
  // their loads are issued before the state copy, so that both wait on one
  // memory round (they are used only when the decision accepts)
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (int)(blockDim.x >> 6);
  constexpr int kU = kLbfgsMaxBlocks / 64;
  const bool fast = 4 * m + 1 <= 3 * nw;
  double v[3][kU];
  if (fast) {
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int c = wave + r * nw;
      const double* pc = part + (long long)c * nb;
#pragma unroll
      for (int u = 0; u < kU; ++u) {
        const int b = lane + 64 * u;
        v[r][u] = (c < 4 * m + 1 && b < nb) ? pc[b] : 0.0;
      }
    }
  }
  for (int i = threadIdx.x; i < kWords; i += blockDim.x)
    reinterpret_cast<uint32_t*>(&sh)[i] = reinterpret_cast<const uint32_t*>(Sg)[i];
  if (fast) {
    // reduced whatever the decision (a rejection or restart does not read them)
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int c = wave + r * nw;
      double t = 0.0;
#pragma unroll
      for (int u = 0; u < kU; ++u) t += v[r][u];
      for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
      if (lane == 0 && c < 4 * m + 1) red[c] = t;
    }
  }
  __syncthreads();
  if (threadIdx.x == 0) lb_decide(&sh, o);
  __syncthreads();
  const int step = sh.step;
  if (step == LB_ACCEPT || step == LB_INIT) {
    if (!fast) {
      for (int c = wave; c < 4 * m + 1; c += nw) {
        const double* pc = part + (long long)c * nb;
        double w[kU];
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int b = lane + 64 * u;
          w[u] = (b < nb) ? pc[b] : 0.0;
        }
        double t = 0.0;
#pragma unroll
        for (int u = 0; u < kU; ++u) t += w[u];
        for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
        if (lane == 0) red[c] = t;
      }
    }
  }
  __syncthreads();
  const bool dir = step == LB_ACCEPT || step == LB_INIT || step == LB_RESTART;
  if (threadIdx.x == 0 && dir) lb_small_update(&sh, o, red, step, n, cs);
  __syncthreads();
  if (threadIdx.x < 64 && dir) lb_small_direction(&sh, o, cs);
  __syncthreads();
  for (int i = threadIdx.x; i < kWords; i += blockDim.x)
    reinterpret_cast<uint32_t*>(Sg)[i] = reinterpret_cast<const uint32_t*>(&sh)[i];
}

// Partial slots: [0, m) s_j.y_new, [m, 2m) y_j.y_new, [2m, 3m) s_j.g, [3m, 4m) y_j.g,
// 4m g.g (slot j indexes the ring; the new pair's own entries sit at its slot).
// MM = history length m (compile time, so the accumulators stay in registers).
// Every load of an element is issued before its stores and products (the ring
// slot of the new pair is read before it is overwritten and its value replaced
// by the new pair's); ALL: every slot holds a pair (the steady state), so no
// load waits behind a branch.
template <class R, int MM, bool ACC, bool ALL>
__device__ __forceinline__ void pass_a_loop(const LbfgsVec<R>& v, unsigned live, int ns, R alpha,
                                            double (&acc_v)[4 * MM + 1]) {
  R* Sn = v.S + (long long)ns * v.n;
  R* Yn = v.Y + (long long)ns * v.n;
  GRID_LOOP(i, v.n) {
    R sj[MM], yj[MM];
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      const bool lj = ALL || ((live >> j) & 1u);
      sj[j] = lj ? v.S[(long long)j * v.n + i] : R(0);
      yj[j] = lj ? v.Y[(long long)j * v.n + i] : R(0);
    }
    const R gn = v.gt[i];
    const R g0 = v.g[i];
    R yy = R(0);
    if (ACC) {
      const R sy = alpha * v.p[i];
      const R xt = v.xt[i];
      yy = gn - g0;
      Sn[i] = sy;
      Yn[i] = yy;
      v.x[i] = xt;
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        sj[j] = (j == ns) ? sy : sj[j];
        yj[j] = (j == ns) ? yy : yj[j];
      }
    }
    v.g[i] = gn;
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      if (ALL || ((live >> j) & 1u)) {
        if (ACC) {
          acc_v[j] += (double)sj[j] * (double)yy;
          acc_v[MM + j] += (double)yj[j] * (double)yy;
        }
        acc_v[2 * MM + j] += (double)sj[j] * (double)gn;
        acc_v[3 * MM + j] += (double)yj[j] * (double)gn;
      }
    }
    acc_v[4 * MM] += (double)gn * (double)gn;
  }
}

template <class R, int MM>
__global__ void lb_pass_a_kernel(LbfgsVec<R> v, LbfgsState* S, LbfgsOpts o) {
  __shared__ double sh[(4 * MM + 1) * kWaves];
  const int step = lb_decided_step(S, o);
  if (step == LB_ACCEPT || step == LB_INIT) {
    const bool acc = (step == LB_ACCEPT);
    const int ns = (S->head + 1) % MM;  // slot of the new pair
    const R alpha = (R)S->alpha;
    // slots holding pairs after this step (the new slot included when accepting)
    unsigned live = 0;
    {
      const int k = S->k;
      for (int t = 0; t < k; ++t) live |= 1u << ((S->head - t + MM) % MM);
      if (acc) live |= 1u << ns;
    }
    double acc_v[4 * MM + 1];
#pragma unroll
    for (int c = 0; c < 4 * MM + 1; ++c) acc_v[c] = 0.0;
    constexpr unsigned kAll = (MM >= 32) ? 0xffffffffu : ((1u << MM) - 1u);
    if (acc && live == kAll) pass_a_loop<R, MM, true, true>(v, live, ns, alpha, acc_v);
    else if (acc) pass_a_loop<R, MM, true, false>(v, live, ns, alpha, acc_v);
    else pass_a_loop<R, MM, false, false>(v, live, ns, alpha, acc_v);
    block_partials<4 * MM + 1>(acc_v, 4 * MM + 1, v.part0, v.nb, sh);
  }
}

// Serial part of the small step (one thread, state in LDS): the new pair's
// products, and the chronological slots cs[0] (oldest) .. cs[k-1] (newest).
__device__ __forceinline__ void lb_small_update(LbfgsState* S, const LbfgsOpts& o,
                                                const double* red, int step, long long n,
                                                int* cs) {
  const int m = o.m;
  if (step != LB_RESTART) {
    S->gg = red[4 * m];
    for (int j = 0; j < m; ++j) {
      S->SG[j] = red[2 * m + j];
      S->YG[j] = red[3 * m + j];
    }
  }
  S->gnorm_rms = sqrt(S->gg / (double)n);
  if (o.gtol > 0.0 && S->gnorm_rms <= o.gtol) S->converged = 1;
  if (step == LB_ACCEPT) {
    const int ns = (S->head + 1) % m;
    const double ys = red[ns], yy = red[m + ns];
    if (ys > 0.0 && yy > 0.0) {
      // dropping the oldest pair when the ring is full: its slot is ns
      for (int j = 0; j < m; ++j) {
        S->SY[j * kLbfgsMaxM + ns] = red[j];      // s_j . y_new
        S->YY[j * kLbfgsMaxM + ns] = red[m + j];  // y_j . y_new
        S->YY[ns * kLbfgsMaxM + j] = red[m + j];
      }
      S->head = ns;
      if (S->k < m) S->k += 1;
      S->gamma = ys / yy;
      S->restarted = 0;
    } else {
      S->k = 0;  // curvature condition failed: steepest descent
    }
  }
  const int k = S->k;
  for (int i = 0; i < k; ++i) cs[i] = (S->head - (k - 1) + i + m) % m;
  for (int j = 0; j < m; ++j) {
    S->coefS[j] = 0.0;
    S->coefY[j] = 0.0;
  }
}

// Direction coefficients by one wavefront: lane i < k holds the pair of
// chronological index i, with its row of R = S^T Y (upper triangle used), its
// column of R and its row of Y^T Y in registers; the triangular solves pass
// each solved unknown to the other lanes by shuffle.
__device__ __forceinline__ void lb_small_direction(LbfgsState* S, const LbfgsOpts& o,
                                                   const int* cs) {
  const int lane = threadIdx.x & 63;
  const int k = S->k;
  double gtp;
  if (k == 0) {
    if (lane == 0) S->coefG = 1.0;
    gtp = -S->gg;
  } else {
    const double gam = S->gamma;
    const bool mine = lane < k;
    const int si = mine ? cs[lane] : 0;
    double Rrow[kLbfgsMaxM], Rcol[kLbfgsMaxM], Yrow[kLbfgsMaxM];
#pragma unroll
    for (int j = 0; j < kLbfgsMaxM; ++j) {
      const bool on = mine && j < k;
      const int sj = (j < k) ? cs[j] : 0;
      Rrow[j] = on ? S->SY[si * kLbfgsMaxM + sj] : 0.0;  // s_i . y_j
      Rcol[j] = on ? S->SY[sj * kLbfgsMaxM + si] : 0.0;  // s_j . y_i
      Yrow[j] = on ? S->YY[si * kLbfgsMaxM + sj] : 0.0;  // y_i . y_j
    }
    const double a = mine ? S->SG[si] : 0.0;  // s_i . g
    const double b = mine ? S->YG[si] : 0.0;  // y_i . g
    const double D = mine ? S->SY[si * kLbfgsMaxM + si] : 1.0;
    // R t = a, from the newest pair down
    double r = a, t = 0.0;
#pragma unroll
    for (int i0 = kLbfgsMaxM - 1; i0 >= 0; --i0) {
      if (i0 < k) {
        const double ti = __shfl(r, i0, 64) / __shfl(D, i0, 64);
        if (lane == i0) t = ti;
        if (lane < i0) r -= Rrow[i0] * ti;
      }
    }
    // w = (D + gamma Y^T Y) t - gamma b
    double w = D * t - gam * b;
#pragma unroll
    for (int j = 0; j < kLbfgsMaxM; ++j)
      if (j < k) w += gam * Yrow[j] * __shfl(t, j, 64);
    // R^T u = w, from the oldest pair up
    double q = w, u = 0.0;
#pragma unroll
    for (int j0 = 0; j0 < kLbfgsMaxM; ++j0) {
      if (j0 < k) {
        const double uj = __shfl(q, j0, 64) / __shfl(D, j0, 64);
        if (lane == j0) u = uj;
        if (lane > j0) q -= Rcol[j0] * uj;
      }
    }
    if (mine) {
      S->coefS[si] = u;
      S->coefY[si] = -gam * t;
    }
    double ua = mine ? u * a : 0.0, tb = mine ? t * b : 0.0;
    for (int off = 32; off > 0; off >>= 1) {
      ua += __shfl_down(ua, off, 64);
      tb += __shfl_down(tb, off, 64);
    }
    ua = __shfl(ua, 0, 64);
    tb = __shfl(tb, 0, 64);
    if (lane == 0) S->coefG = gam;
    gtp = -(gam * S->gg + ua - gam * tb);
    if (!(gtp < 0.0) || !isfinite(gtp)) {
      // not a descent direction: drop the history, steepest descent
      if (mine) {
        S->coefS[si] = 0.0;
        S->coefY[si] = 0.0;
      }
      if (lane == 0) {
        S->k = 0;
        S->resets += 1;
        S->coefG = 1.0;
      }
      gtp = -S->gg;
    }
  }
  if (lane == 0) {
    S->gtp = gtp;
    if (!(gtp < 0.0)) {
      S->converged = 1;  // zero gradient
      S->step = LB_IDLE;
    }
  }
}

// ---------------------------------------------------------------- pass B
// p = -(cg g + sum over live slots of cS S_j + cY Y_j); returns max |p| of the
// thread's elements.  ALL: every slot holds a pair (no branch between loads).
template <class R, int MM, bool ALL>
__device__ __forceinline__ double pass_b_loop(const LbfgsVec<R>& v, unsigned live, R cg,
                                              const R (&cS)[MM], const R (&cY)[MM]) {
  double pm = 0.0;
  GRID_LOOP(j, v.n) {
    R r = cg * v.g[j];
#pragma unroll
    for (int i = 0; i < MM; ++i) {
      if (ALL || ((live >> i) & 1u)) {
        r += cS[i] * v.S[(long long)i * v.n + j];
        r += cY[i] * v.Y[(long long)i * v.n + j];
      }
    }
    v.p[j] = -r;
    pm = fmax(pm, fabs((double)r));
  }
  return pm;
}

template <class R, int MM>
__global__ void lb_pass_b_kernel(LbfgsVec<R> v, LbfgsState* S) {
  __shared__ double sh[kWaves];
  const int step = S->step;
  if (step != LB_ACCEPT && step != LB_INIT && step != LB_RESTART) return;
  const int k = S->k;
  // coefficients by slot; slots without a pair have coefficient 0 and are skipped
  R cS[MM], cY[MM];
  unsigned live = 0;
#pragma unroll
  for (int j = 0; j < MM; ++j) {
    cS[j] = (R)S->coefS[j];
    cY[j] = (R)S->coefY[j];
  }
  for (int t = 0; t < k; ++t) live |= 1u << ((S->head - t + MM) % MM);
  const R cg = (R)S->coefG;
  double pm = 0.0;
  constexpr unsigned kAll = (MM >= 32) ? 0xffffffffu : ((1u << MM) - 1u);
  if (live == kAll) {
    pm = pass_b_loop<R, MM, true>(v, live, cg, cS, cY);
  } else {
    pm = pass_b_loop<R, MM, false>(v, live, cg, cS, cY);
  }
  for (int off = 32; off > 0; off >>= 1) pm = fmax(pm, __shfl_down(pm, off, 64));
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = pm;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < kWaves; ++w) t = fmax(t, sh[w]);
    v.part1[blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------- pass C
// xt = x + alpha p from element j of the thread on (stride: the grid), four
// elements in flight at once
template <class R>
__device__ __forceinline__ void trial_point(const R* __restrict__ x, const R* __restrict__ p,
                                            R* __restrict__ xt, long long n, R alpha,
                                            long long j) {
  const long long st = (long long)gridDim.x * blockDim.x;
  for (; j + 3 * st < n; j += 4 * st) {
    R a[4], b[4];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      a[u] = x[j + u * st];
      b[u] = p[j + u * st];
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) xt[j + u * st] = a[u] + alpha * b[u];
  }
  for (; j < n; j += st) xt[j] = x[j] + alpha * p[j];
}

// step length of a new direction (every block reduces the pass B maxima), or
// the one shrunk by the decision; then the trial point
template <class R>
__global__ void lb_pass_c_kernel(LbfgsVec<R> v, LbfgsState* S, LbfgsOpts o) {
  __shared__ double sh[kWaves];
  __shared__ double alpha_s;
  const int step = S->step;
  if (step == LB_IDLE) return;
  // the thread's first four elements of x and p, loaded before the step length
  // is known (their latency overlaps the reduction of the block maxima)
  const long long st = (long long)gridDim.x * blockDim.x;
  const long long j0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  R xa[4], pa[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const long long j = j0 + u * st;
    xa[u] = (j < v.n) ? v.x[j] : R(0);
    pa[u] = (j < v.n) ? v.p[j] : R(0);
  }
  if (step == LB_REJECT) {
    if (threadIdx.x == 0) alpha_s = S->alpha;
  } else {
    // nb <= kLbfgsMaxBlocks: every maximum a thread reads is loaded at once
    constexpr int kU = (kLbfgsMaxBlocks + kThreads - 1) / kThreads;
    double q[kU];
#pragma unroll
    for (int u = 0; u < kU; ++u) {
      const int b = threadIdx.x + u * blockDim.x;
      q[u] = (b < v.nb) ? v.part1[b] : 0.0;
    }
    double pm = 0.0;
#pragma unroll
    for (int u = 0; u < kU; ++u) pm = fmax(pm, q[u]);
    for (int off = 32; off > 0; off >>= 1) pm = fmax(pm, __shfl_down(pm, off, 64));
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = pm;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < kWaves; ++w) t = fmax(t, sh[w]);
      const double a = (t > o.max_step) ? o.max_step / t : 1.0;
      alpha_s = a;
      if (blockIdx.x == 0) S->alpha = a;
    }
  }
  __syncthreads();
  const R alpha = (R)alpha_s;
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    const long long j = j0 + u * st;
    if (j < v.n) v.xt[j] = xa[u] + alpha * pa[u];
  }
  trial_point<R>(v.x, v.p, v.xt, v.n, alpha, j0 + 4 * st);
}

// set the mode read by the next decision (host-driven transitions)
__global__ void lb_set_mode_kernel(LbfgsState* S, int mode, int target) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    S->mode = mode;
    if (target >= 0) {
      S->target = target;
      S->iter = 0;
      S->nevals = 0;
      S->fail = 0;
      S->converged = 0;
    }
  }
}

template <class R>
void launch_lbfgs_update(const LbfgsVec<R>& v, LbfgsState* S, const LbfgsOpts& o,
                         hipStream_t st) {
#define LB_A(MM) lb_pass_a_kernel<R, MM><<<v.nb, kThreads, 0, st>>>(v, S, o)
#define LB_B(MM) lb_pass_b_kernel<R, MM><<<v.nb, kThreads, 0, st>>>(v, S)
#define LB_SWITCH(CALL)                                                        \
  switch (v.m) {                                                               \
    case 1: CALL(1); break;   case 2: CALL(2); break;   case 3: CALL(3); break;   \
    case 4: CALL(4); break;   case 5: CALL(5); break;   case 6: CALL(6); break;   \
    case 7: CALL(7); break;   case 8: CALL(8); break;   case 9: CALL(9); break;   \
    case 10: CALL(10); break; case 11: CALL(11); break; case 12: CALL(12); break; \
    case 13: CALL(13); break; case 14: CALL(14); break; case 15: CALL(15); break; \
    case 16: CALL(16); break;                                                  \
  }
  LB_SWITCH(LB_A)
  lb_small_kernel<<<1, 1024, 0, st>>>(S, o, v.part0, v.nb, v.n);
  LB_SWITCH(LB_B)
#undef LB_SWITCH
#undef LB_B
#undef LB_A
  lb_pass_c_kernel<R><<<v.nb, kThreads, 0, st>>>(v, S, o);
}

void launch_lbfgs_set_mode(LbfgsState* S, int mode, int target, hipStream_t st) {
  lb_set_mode_kernel<<<1, 64, 0, st>>>(S, mode, target);
}

// ------------------------------------------------------- permutations
template <class R>
__global__ void gather_rows_kernel(const R* __restrict__ src, const int* __restrict__ idx,
                                   long long n, int d, R* __restrict__ dst) {
  GRID_LOOP(j, n) {
    const long long s = (long long)idx[j] * d;
    for (int a = 0; a < d; ++a) dst[j * d + a] = src[s + a];
  }
}
template <class R>
__global__ void scatter_rows_kernel(const R* __restrict__ src, const int* __restrict__ idx,
                                    long long n, int d, R* __restrict__ dst) {
  GRID_LOOP(j, n) {
    const long long s = (long long)idx[j] * d;
    for (int a = 0; a < d; ++a) dst[s + a] = src[j * d + a];
  }
}
template <class R>
void launch_gather_rows(const R* src, const int* idx, long long n, int d, R* dst, hipStream_t st) {
  long long b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  gather_rows_kernel<R><<<(unsigned)b, 256, 0, st>>>(src, idx, n, d, dst);
}
template <class R>
void launch_scatter_rows(const R* src, const int* idx, long long n, int d, R* dst,
                         hipStream_t st) {
  long long b = (n + 255) / 256;
  if (b > 4096) b = 4096;
  scatter_rows_kernel<R><<<(unsigned)b, 256, 0, st>>>(src, idx, n, d, dst);
}

#define FRESCO_LB_INST(R)                                                                       \
  template void launch_lbfgs_update<R>(const LbfgsVec<R>&, LbfgsState*, const LbfgsOpts&,       \
                                       hipStream_t);                                            \
  template void launch_gather_rows<R>(const R*, const int*, long long, int, R*, hipStream_t);   \
  template void launch_scatter_rows<R>(const R*, const int*, long long, int, R*, hipStream_t);
FRESCO_LB_INST(float)
FRESCO_LB_INST(double)

}  // namespace fresco
