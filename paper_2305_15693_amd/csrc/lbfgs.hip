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
// Per replay, after the loss/gradient evaluation at the trial point xt, three
// kernels:
//   pass A   decision: Armijo test f(xt) <= f(x) + c1 alpha g.p -> ACCEPT or
//            REJECT (REJECT: alpha *= shrink; after max_backtracks rejections
//            the history is dropped and the search restarts along -g; a second
//            failure sets the failure flag), computed by every block from the
//            state; on ACCEPT s = alpha p, y = g(xt) - g(x) into the ring,
//            x = xt, g = g(xt), and the new dot products s_j.y, y_j.y, s_j.g,
//            y_j.g, g.g as block partials; block 0 leaves a snapshot of the
//            state with f(xt);
//   pass B   the small step, in every block on its LDS copy of the snapshot:
//            applies the decision, reduces the partials, stores the pair when
//            y.s > 0 and solves for u, t (FP64, one wavefront), block 0
//            writing the new state back; then p = -(gamma g + S u - gamma Y t),
//            max |p| per block;
//   pass C   alpha = min(1, max_step / max|p|), xt = x + alpha p (not run when
//            the next evaluation keeps the tile order of the last binning: its
//            spreading pass forms the trial point and its records).
// (Cross-block steps stay at kernel boundaries: a device-scope fence per block
// writes back the L2 of its XCD and cost more than the launches it saved.)
// Vectors are in the working precision; every dot product is accumulated in FP64
// with a fixed reduction order.
#include <cmath>
#include <cstring>

#include "common.h"
#include "lbfgs.h"

namespace fresco {


constexpr int kThreads = kLbfgsThreads;
constexpr int kWaves = kThreads / 64;

#define GRID_LOOP(i, n) \
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < (n); i += (long long)gridDim.x * blockDim.x)

// Reduce CNT per-thread values across a block of NW waves (fixed order) and
// write value c to part[row(c) * nb + blockIdx.x] (not written when row(c) < 0).
template <int CNT, int NW, class Row>
__device__ __forceinline__ void block_partials(const double* v, double* part, int nb,
                                               double* sh /* [CNT][NW] */, Row row) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int c = 0; c < CNT; ++c) {
    double x = v[c];
    for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
    if (lane == 0) sh[c * NW + wave] = x;
  }
  __syncthreads();
  for (int c = threadIdx.x; c < CNT; c += blockDim.x) {
    double t = 0.0;
    for (int w = 0; w < NW; ++w) t += sh[c * NW + w];
    const int r = row(c);
    if (r >= 0) part[(long long)r * nb + blockIdx.x] = t;
  }
}

// ---------------------------------------------------------------- decide
// Decision on the evaluation just finished, as a function of the state (every
// block of pass A computes it; the small step then applies it).
__device__ __forceinline__ int lb_decided_step(const LbfgsState* S, const LbfgsOpts& o,
                                               double f) {
  if (S->mode == LB_INIT) return LB_INIT;  // first evaluation of a call
  if (S->fail || S->iter >= S->target || S->converged) return LB_IDLE;
  if (isfinite(f) && f <= S->f_cur + o.c1 * S->alpha * S->gtp) return LB_ACCEPT;
  if (S->nbt + 1 > o.max_backtracks) return (S->k > 0 || !S->restarted) ? LB_RESTART : LB_IDLE;
  return LB_REJECT;
}
__device__ __forceinline__ void lb_decide(LbfgsState* S, const LbfgsOpts& o) {
  const int step = lb_decided_step(S, o, S->f_trial);
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

// ---------------------------------------------------------------- small step
// LDS writes of this wavefront visible to its later LDS reads by other lanes:
// the wave's LDS accesses are performed in order once issued; the fence waits
// for them and keeps the compiler from moving accesses across.
__device__ __forceinline__ void wave_lds_fence() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
  __builtin_amdgcn_wave_barrier();
}

template <int MM>
__device__ __forceinline__ void lb_small_wave(LbfgsState* S, const LbfgsOpts& o,
                                              const double* red, long long n);

// Small step, run by every block of pass B on its LDS copy of the snapshot that
// pass A left (block 0 rewrites the state itself while the other blocks may still
// be reading, so none of them reads it): reduce the pass A partials, then on one
// wavefront apply the decision, update the pair products and solve for the
// direction coefficients.  Every block computes the same values in the same
// order, so no block waits for another and no one-block launch sits between the
// two streaming passes.
template <int MM>
__device__ __forceinline__ void lb_small_step(const LbfgsState* __restrict__ snap,
                                              const LbfgsOpts& o, const double* __restrict__ part,
                                              int nb, long long n, LbfgsState& ss,
                                              double* red) {
  static_assert(sizeof(LbfgsState) % 4 == 0, "state copied as 32-bit words");
  constexpr int kWords = (int)(sizeof(LbfgsState) / 4);
  const int nv = 4 * o.m + 1;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int i = threadIdx.x; i < kWords; i += blockDim.x)
    reinterpret_cast<uint32_t*>(&ss)[i] = reinterpret_cast<const uint32_t*>(snap)[i];
  // value c is reduced by wave c mod kWaves: lane l sums the partials l, l + 64,
  // ... in index order, then the wave's shuffle tree.  Five values of a wave and
  // four of each value's loads per round: one round for the 33 values of m = 8
  // over 256 partials.  Reduced whatever the decision (a rejection or restart
  // does not read them).
  constexpr int kR = 5, kU = 4;
  for (int c0 = wave; c0 < nv; c0 += kR * kWaves) {
    double t[kR];
#pragma unroll
    for (int r = 0; r < kR; ++r) t[r] = 0.0;
    for (int u0 = 0; 64 * u0 < nb; u0 += kU) {
      double w[kR][kU];
#pragma unroll
      for (int r = 0; r < kR; ++r) {
        const int c = c0 + r * kWaves;
#pragma unroll
        for (int u = 0; u < kU; ++u) {
          const int b = lane + 64 * (u0 + u);
          w[r][u] = (c < nv && b < nb) ? part[(long long)c * nb + b] : 0.0;
        }
      }
#pragma unroll
      for (int r = 0; r < kR; ++r)
#pragma unroll
        for (int u = 0; u < kU; ++u) t[r] += w[r][u];
    }
#pragma unroll
    for (int r = 0; r < kR; ++r) {
      const int c = c0 + r * kWaves;
      double x = t[r];
      for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
      if (lane == 0 && c < nv) red[c] = x;
    }
  }
  __syncthreads();
  if (threadIdx.x < 64) lb_small_wave<MM>(&ss, o, red, n);
  __syncthreads();
}

// ------------------------------------------------------- packed access
// The vector passes move U consecutive elements per thread and step with one
// 16-byte access per array (U = 4 in FP32, 2 in FP64): fewer, wider requests
// than one element per lane.  Every array is a separate allocation and the
// history slots are v.ld elements apart (a multiple of 4), so the packs are
// aligned; the launcher falls back to single elements (vec = 0) otherwise.
template <class R, int U>
struct alignas(sizeof(R) * U) Pack {
  R e[U];
};
template <class R, int U>
__device__ __forceinline__ Pack<R, U> ldp(const R* p, long long i) {
  return *reinterpret_cast<const Pack<R, U>*>(p + i);
}
template <class R, int U>
__device__ __forceinline__ void stp(R* p, long long i, const Pack<R, U>& x) {
  *reinterpret_cast<Pack<R, U>*>(p + i) = x;
}
// elements per pack: B bytes for history length MM <= 8, half that beyond,
// whose loaded slots would not fit in the registers otherwise
template <class R, int MM, int B>
constexpr int pack_u() {
  constexpr int b = MM <= 8 ? B : B / 2;
  return b / (int)sizeof(R) > 0 ? b / (int)sizeof(R) : 1;
}
// Every pass moves 16-byte packs (half that beyond m = 8).  Pass A holds 4m + 5
// FP64 accumulators besides the loaded packs: up to m = 8 it takes up to 168
// registers (three waves per SIMD); with single elements it fitted four waves per
// SIMD in 128 registers but ran 5% slower (fewer bytes in flight per wave).
constexpr int kPackBytesA = 16;
constexpr int kPackBytesBC = 16;

// Pass A on elements [i, i + U).  The old pairs are read by age (age a sits in
// slot (head - a) mod m; pointers pS[a], pY[a]), every load issued before the
// first product; MASK: only ages below k hold pairs, the others read their
// slot's first pack (index i & im[a] = 0: one cache line for the whole grid, no
// branch between the loads) and are replaced by zeros.  acc: [0, NA) s_a.y_new, [NA, 2 NA) y_a.y_new,
// [2 NA, 3 NA) s_a.g, [3 NA, 4 NA) y_a.g, then s.y, y.y, s.g, y.g of the new pair
// and g.g.
template <class R, int U, int NA, bool ACC, bool MASK>
__device__ __forceinline__ void pass_a_elems(const LbfgsVec<R>& v, const R* const* pS,
                                             const R* const* pY, const long long* im, R* Sn,
                                             R* Yn, int k, R alpha, long long i, double* acc) {
  constexpr int NB = NA > 0 ? NA : 1;
  Pack<R, U> sa[NB], ya[NB];
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    const long long ia = MASK ? (i & im[a]) : i;
    sa[a] = ldp<R, U>(pS[a], ia);
    ya[a] = ldp<R, U>(pY[a], ia);
  }
  const Pack<R, U> gn = ldp<R, U>(v.gt, i);
  const Pack<R, U> g0 = ldp<R, U>(v.g, i);
  Pack<R, U> sy, yy;
  if (ACC) {
    const Pack<R, U> pp = ldp<R, U>(v.p, i);
    const Pack<R, U> xt = ldp<R, U>(v.xt, i);
#pragma unroll
    for (int e = 0; e < U; ++e) {
      sy.e[e] = alpha * pp.e[e];
      yy.e[e] = gn.e[e] - g0.e[e];
    }
    stp<R, U>(Sn, i, sy);
    stp<R, U>(Yn, i, yy);
    stp<R, U>(v.x, i, xt);
  }
  stp<R, U>(v.g, i, gn);
#pragma unroll
  for (int e = 0; e < U; ++e) {
    const double gd = (double)gn.e[e];
    const double yd = ACC ? (double)yy.e[e] : 0.0;
#pragma unroll
    for (int a = 0; a < NA; ++a) {
      const double sv = (MASK && a >= k) ? 0.0 : (double)sa[a].e[e];
      const double yv = (MASK && a >= k) ? 0.0 : (double)ya[a].e[e];
      if (ACC) {
        acc[a] += sv * yd;
        acc[NA + a] += yv * yd;
      }
      acc[2 * NA + a] += sv * gd;
      acc[3 * NA + a] += yv * gd;
    }
    if (ACC) {
      const double sd = (double)sy.e[e];
      acc[4 * NA] += sd * yd;
      acc[4 * NA + 1] += yd * yd;
      acc[4 * NA + 2] += sd * gd;
      acc[4 * NA + 3] += yd * gd;
    }
    acc[4 * NA + 4] += gd * gd;
  }
}

// Pass A of one decision: packs of U elements strided over the grid (vec), then
// the elements past the last whole pack one at a time; the products go out as
// block partials in slot order: [0, m) s_j.y_new, [m, 2m) y_j.y_new,
// [2m, 3m) s_j.g, [3m, 4m) y_j.g, 4m g.g (slot j indexes the ring; the new pair's
// products sit at its slot ns).  Accepting, the oldest pair is dropped when the
// ring is full: its slot ns is never read.
template <class R, int MM, int NA, bool ACC, bool MASK>
__device__ __forceinline__ void pass_a_run(const LbfgsVec<R>& v, int head, int k, int ns,
                                           R alpha, bool vec, double* sh) {
  constexpr int NB = NA > 0 ? NA : 1;
  const R* pS[NB];
  const R* pY[NB];
  long long im[NB];
#pragma unroll
  for (int a = 0; a < NA; ++a) {
    const long long slot = (head - a + MM) % MM;
    pS[a] = v.S + slot * v.ld;
    pY[a] = v.Y + slot * v.ld;
    im[a] = (a < k) ? ~0LL : 0LL;
  }
  R* Sn = v.S + (long long)ns * v.ld;
  R* Yn = v.Y + (long long)ns * v.ld;
  double acc[4 * NA + 5];
#pragma unroll
  for (int c = 0; c < 4 * NA + 5; ++c) acc[c] = 0.0;
  constexpr int U = pack_u<R, MM, kPackBytesA>();
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long gs = (long long)gridDim.x * blockDim.x;
  const long long nq = vec ? v.n / U : 0;
  for (long long q = gid; q < nq; q += gs)
    pass_a_elems<R, U, NA, ACC, MASK>(v, pS, pY, im, Sn, Yn, k, alpha, q * U, acc);
  for (long long i = nq * U + gid; i < v.n; i += gs)
    pass_a_elems<R, 1, NA, ACC, MASK>(v, pS, pY, im, Sn, Yn, k, alpha, i, acc);
  // rows of the partials: kind * m + slot for the old pairs by age, the new
  // pair's four products at slot ns (zeros when not accepting; not written when
  // an old pair's age already covers ns), g.g at 4m; every row is written once
  // (ages without a pair hold zeros)
  block_partials<4 * NA + 5, kWaves>(acc, v.part0, v.nb, sh, [&](int c) {
    if (c < 4 * NA) return (c / NA) * MM + (head - c % NA + MM) % MM;
    if (c < 4 * NA + 4) return NA == MM ? -1 : (c - 4 * NA) * MM + ns;
    return 4 * MM;
  });
}

// MM = history length m (compile time, so the accumulators stay in registers).
// loss.n >= 0: the evaluation's loss partials, summed here in the order of the
// loss finish (every block, for its decision; block 0 stores f_trial and hands
// over the flag); else f_trial holds the loss.
template <class R, int MM>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(MM <= 8 ? 3 : 2))) void lb_pass_a_kernel(LbfgsVec<R> v, LbfgsState* S, LbfgsOpts o, int vec, LossParts loss) {
  __shared__ double sh[(4 * MM + 5) * kWaves];
  double f;
  if (loss.n >= 0) {
    // summed as by the 256-thread loss finish
    __shared__ double s256[256];
    const double a = block_sum_256(loss.part, loss.n, s256);
    const double b = (loss.n2 > 0) ? block_sum_256(loss.part2, loss.n2, s256) : 0.0;
    f = (loss.n2 > 0) ? a + loss.w2 * b : a;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      *loss.flag_out = *loss.flag;
      *loss.flag = 0;
    }
  } else {
    f = S->f_trial;
  }
  if (blockIdx.x == 0) {
    // the snapshot S[1] that every block of pass B starts from, with this
    // evaluation's loss as f_trial (pass B's block 0 writes the state back)
    static_assert(sizeof(LbfgsState) % 4 == 0, "state copied as 32-bit words");
    constexpr int kWords = (int)(sizeof(LbfgsState) / 4);
    constexpr int kF = (int)(offsetof(LbfgsState, f_trial) / 4);
    const unsigned long long fb = (unsigned long long)__double_as_longlong(f);
    const uint32_t* src = reinterpret_cast<const uint32_t*>(S);
    uint32_t* dst = reinterpret_cast<uint32_t*>(S + 1);
    for (int i = threadIdx.x; i < kWords; i += blockDim.x) {
      uint32_t w = src[i];
      if (i == kF) w = (uint32_t)fb;
      if (i == kF + 1) w = (uint32_t)(fb >> 32);
      dst[i] = w;
    }
  }
  const int step = lb_decided_step(S, o, f);
  if (step != LB_ACCEPT && step != LB_INIT) return;  // uniform: before any barrier
  const int head = S->head, k = S->k;
  const int ns = (head + 1) % MM;  // slot of the new pair
  const R alpha = (R)S->alpha;
  if (step == LB_ACCEPT) {
    // the pairs kept are the k newest, at most m - 1 of them
    if (k >= MM - 1) pass_a_run<R, MM, MM - 1, true, false>(v, head, k, ns, alpha, vec, sh);
    else pass_a_run<R, MM, MM - 1, true, true>(v, head, k, ns, alpha, vec, sh);
  } else {
    if (k == MM) pass_a_run<R, MM, MM, false, false>(v, head, k, ns, alpha, vec, sh);
    else pass_a_run<R, MM, MM - 1, false, true>(v, head, k, ns, alpha, vec, sh);
  }
}

// Direction coefficients (one wavefront; lane i < k holds the pair of
// chronological index i, ring slot sl[i]).  R^-1 is kept in the state and
// extended by the new pair's column (dropping the oldest pair leaves the rest of
// it as it is), so t and u are products rather than dependent triangular solves:
//   R^-1[i][new] = -(sum over i <= j < new of R^-1[i][j] R[j][new]) / R[new][new],
//   R^-1[new][new] = 1 / R[new][new].
// Every lane loads its rows for all MM chronological indices at once (indices at
// or past k read slot 0 and are masked), so that no LDS load waits inside a
// divergent branch.
template <int MM>
__device__ __forceinline__ void lb_small_direction(LbfgsState* S, int head, int k, int m,
                                                   bool added) {
  constexpr int M = kLbfgsMaxM;
  const int lane = threadIdx.x & 63;
  double gtp;
  if (k == 0) {
    if (lane == 0) S->coefG = 1.0;
    gtp = -S->gg;
  } else {
    const double gam = S->gamma;
    const bool mine = lane < k;
    // ring slot of chronological index j: (head - (k - 1) + j) mod m
    int sl[MM];
    const int s0 = (head - (k - 1) + m) >= m ? head - (k - 1) : head - (k - 1) + m;
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      const int q = s0 + j < m ? s0 + j : s0 + j - m;
      sl[j] = j < k ? q : 0;
    }
    int si = 0;
#pragma unroll
    for (int j = 0; j < MM; ++j) si = (j == lane) ? sl[j] : si;
    if (added) {
      const int sn = head;  // the new pair, chronological index k - 1
      const double rho = S->SY[sn * M + sn];
      double x = 0.0;
#pragma unroll
      for (int j = 0; j < MM; ++j) {
        const double r = S->RI[si * M + sl[j]];
        const double c = S->SY[sl[j] * M + sn];
        x += (j >= lane && j < k - 1) ? r * c : 0.0;
      }
      if (lane < k - 1) S->RI[si * M + sn] = -x / rho;
      else if (lane == k - 1) S->RI[sn * M + sn] = 1.0 / rho;
      wave_lds_fence();
    }
    const double a = mine ? S->SG[si] : 0.0;  // s_i . g
    const double b = mine ? S->YG[si] : 0.0;  // y_i . g
    const double D = mine ? S->SY[si * M + si] : 0.0;
    // t = R^-1 a: lane i sums over i <= j < k (row i of R^-1)
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      const double r = S->RI[si * M + sl[j]], aj = S->SG[sl[j]];
      t += (mine && j >= lane && j < k) ? r * aj : 0.0;
    }
    // w = (D + gamma Y^T Y) t - gamma b
    double w = D * t - gam * b;
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      const double yij = S->YY[si * M + sl[j]];
      const double tj = __shfl(t, j, 64);
      w = (mine && j < k) ? w + gam * yij * tj : w;
    }
    // u = R^-T w: lane j sums over i <= j (column j of R^-1)
    double u = 0.0;
#pragma unroll
    for (int i = 0; i < MM; ++i) {
      const double r = S->RI[sl[i] * M + si];
      const double wi = __shfl(w, i, 64);
      u += (mine && i <= lane && i < k) ? r * wi : 0.0;
    }
    if (mine) {
      S->coefS[si] = u;
      S->coefY[si] = -gam * t;
    }
    // sums over the k <= MM lanes: a butterfly over the smallest power of two
    // holding them (every lane gets the sum; the additions are those of a
    // shuffle-down tree, the other lanes holding zeros)
    double ua = mine ? u * a : 0.0, tb = mine ? t * b : 0.0;
    constexpr int kSpan = MM <= 1 ? 1 : MM <= 2 ? 2 : MM <= 4 ? 4 : MM <= 8 ? 8 : MM <= 16 ? 16 : 64;
#pragma unroll
    for (int off = kSpan / 2; off > 0; off >>= 1) {
      ua += __shfl_xor(ua, off, 64);
      tb += __shfl_xor(tb, off, 64);
    }
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

// The small step on one wavefront, state in LDS: the decision (lane 0), the new
// pair's products (lanes by ring slot), then the direction coefficients.
template <int MM>
__device__ __forceinline__ void lb_small_wave(LbfgsState* S, const LbfgsOpts& o,
                                              const double* red, long long n) {
  constexpr int M = kLbfgsMaxM;
  const int lane = threadIdx.x & 63;
  // every lane takes the decision from the state as it stands (the same value);
  // lane 0 then applies it (of what it changes, only the history count is read
  // below, and that follows from the decision)
  const int step = lb_decided_step(S, o, S->f_trial);
  if (lane == 0) lb_decide(S, o);
  if (step != LB_ACCEPT && step != LB_INIT && step != LB_RESTART) return;  // uniform
  const int m = o.m;
  double gg = S->gg;
  if (step != LB_RESTART) {
    gg = red[4 * m];
    if (lane < m) {
      S->SG[lane] = red[2 * m + lane];
      S->YG[lane] = red[3 * m + lane];
    }
  }
  int head = S->head, k = (step == LB_RESTART) ? 0 : S->k;
  bool added = false;
  if (step == LB_ACCEPT) {
    const int ns = head + 1 == m ? 0 : head + 1;
    const double ys = red[ns], yy = red[m + ns];
    if (ys > 0.0 && yy > 0.0) {
      // dropping the oldest pair when the ring is full: its slot is ns
      if (lane < m) {
        S->SY[lane * M + ns] = red[lane];      // s_j . y_new
        S->YY[lane * M + ns] = red[m + lane];  // y_j . y_new
        S->YY[ns * M + lane] = red[m + lane];
      }
      head = ns;
      if (k < m) k += 1;
      added = true;
      if (lane == 0) {
        S->gamma = ys / yy;
        S->restarted = 0;
      }
    } else {
      k = 0;  // curvature condition failed: steepest descent
    }
  }
  if (lane == 0) {
    S->gg = gg;
    S->gnorm_rms = sqrt(gg / (double)n);
    if (o.gtol > 0.0 && S->gnorm_rms <= o.gtol) S->converged = 1;
    S->head = head;
    S->k = k;
  }
  if (lane < m) {
    S->coefS[lane] = 0.0;
    S->coefY[lane] = 0.0;
  }
  wave_lds_fence();
  lb_small_direction<MM>(S, head, k, m, added);
}

// ---------------------------------------------------------------- pass B
// p = -(cg g + sum over slots of cS_j S_j + cY_j Y_j) on elements [i, i + U), the
// slots in ring order; MASK: slots without a pair (live bit clear) read their
// first pack (one cache line, no branch between the loads) and are replaced by
// zeros.  Returns max |p| over the elements.
template <class R, int U, int MM, bool MASK>
__device__ __forceinline__ double pass_b_elems(const LbfgsVec<R>& v, unsigned live, R cg,
                                               const R (&cS)[MM], const R (&cY)[MM],
                                               long long i) {
  Pack<R, U> sj[MM], yj[MM];
#pragma unroll
  for (int j = 0; j < MM; ++j) {
    const long long ij = (MASK && !((live >> j) & 1u)) ? 0LL : i;
    sj[j] = ldp<R, U>(v.S + (long long)j * v.ld, ij);
    yj[j] = ldp<R, U>(v.Y + (long long)j * v.ld, ij);
  }
  const Pack<R, U> g = ldp<R, U>(v.g, i);
  Pack<R, U> out;
  double pm = 0.0;
#pragma unroll
  for (int e = 0; e < U; ++e) {
    R r = cg * g.e[e];
#pragma unroll
    for (int j = 0; j < MM; ++j) {
      const bool on = !MASK || ((live >> j) & 1u);
      r += cS[j] * (on ? sj[j].e[e] : R(0));
      r += cY[j] * (on ? yj[j].e[e] : R(0));
    }
    out.e[e] = -r;
    pm = fmax(pm, fabs((double)r));
  }
  stp<R, U>(v.p, i, out);
  return pm;
}

template <class R, int MM, bool MASK>
__device__ __forceinline__ double pass_b_run(const LbfgsVec<R>& v, unsigned live, R cg,
                                             const R (&cS)[MM], const R (&cY)[MM], bool vec) {
  constexpr int U = pack_u<R, MM, kPackBytesBC>();
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long gs = (long long)gridDim.x * blockDim.x;
  const long long nq = vec ? v.n / U : 0;
  double pm = 0.0;
  for (long long q = gid; q < nq; q += gs)
    pm = fmax(pm, pass_b_elems<R, U, MM, MASK>(v, live, cg, cS, cY, q * U));
  for (long long i = nq * U + gid; i < v.n; i += gs)
    pm = fmax(pm, pass_b_elems<R, 1, MM, MASK>(v, live, cg, cS, cY, i));
  return pm;
}

// The small step on the snapshot (every block), block 0 writing the new state
// back, then the direction pass with the coefficients from the block's copy.
// (Loading each thread's first packs before the small step, to overlap their
// latency with it, measured no faster: those loads delay the small step's own.)
template <class R, int MM>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(MM <= 8 ? 4 : 2))) void lb_pass_b_kernel(LbfgsVec<R> v, LbfgsState* Sg,
                                                             LbfgsOpts o, int vec) {
  __shared__ double sh[kWaves];
  __shared__ LbfgsState ss;
  __shared__ double red[4 * kLbfgsMaxM + 1];
  lb_small_step<MM>(Sg + 1, o, v.part0, v.nb, v.n, ss, red);
  if (blockIdx.x == 0) {
    constexpr int kWords = (int)(sizeof(LbfgsState) / 4);
    for (int i = threadIdx.x; i < kWords; i += blockDim.x)
      reinterpret_cast<uint32_t*>(Sg)[i] = reinterpret_cast<const uint32_t*>(&ss)[i];
  }
  const LbfgsState* S = &ss;
  const int step = S->step;
  if (step != LB_ACCEPT && step != LB_INIT && step != LB_RESTART) return;
  const int k = S->k;
  // coefficients by slot; slots without a pair have coefficient 0 (and zeros)
  R cS[MM], cY[MM];
  unsigned live = 0;
#pragma unroll
  for (int j = 0; j < MM; ++j) {
    cS[j] = (R)S->coefS[j];
    cY[j] = (R)S->coefY[j];
  }
  for (int t = 0; t < k; ++t) live |= 1u << ((S->head - t + MM) % MM);
  const R cg = (R)S->coefG;
  constexpr unsigned kAll = (MM >= 32) ? 0xffffffffu : ((1u << MM) - 1u);
  const double pm0 = (live == kAll) ? pass_b_run<R, MM, false>(v, live, cg, cS, cY, vec != 0)
                                    : pass_b_run<R, MM, true>(v, live, cg, cS, cY, vec != 0);
  double pm = pm0;
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
// step length of a new direction (every block reduces the pass B maxima), or
// the one shrunk by the decision
template <class R>
__device__ __forceinline__ R pass_c_alpha(const LbfgsVec<R>& v, LbfgsState* S,
                                          const LbfgsOpts& o, int step, double* sh,
                                          double* alpha_s) {
  if (step == LB_REJECT) {
    if (threadIdx.x == 0) *alpha_s = S->alpha;
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
      *alpha_s = a;
      if (blockIdx.x == 0) S->alpha = a;
    }
  }
  __syncthreads();
  return (R)*alpha_s;
}

// the trial point xt = x + alpha p (packs of U elements strided over the grid,
// then the elements past the last whole pack; the thread's first pack is loaded
// before the step length is known, so that its latency overlaps the reduction)
template <class R>
__global__ __launch_bounds__(kThreads) void lb_pass_c_kernel(LbfgsVec<R> v, LbfgsState* S, LbfgsOpts o, int vec) {
  __shared__ double sh[kWaves];
  __shared__ double alpha_s;
  const int step = S->step;
  if (step == LB_IDLE) return;
  constexpr int U = pack_u<R, 1, kPackBytesBC>();
  const long long gid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long gs = (long long)gridDim.x * blockDim.x;
  const long long nq = vec ? v.n / U : 0;
  Pack<R, U> xa, pa;
  if (gid < nq) {
    xa = ldp<R, U>(v.x, gid * U);
    pa = ldp<R, U>(v.p, gid * U);
  }
  const R alpha = pass_c_alpha<R>(v, S, o, step, sh, &alpha_s);
  if (gid < nq) {
    Pack<R, U> t;
#pragma unroll
    for (int e = 0; e < U; ++e) t.e[e] = xa.e[e] + alpha * pa.e[e];
    stp<R, U>(v.xt, gid * U, t);
  }
  for (long long q = gid + gs; q < nq; q += gs) {
    const Pack<R, U> x = ldp<R, U>(v.x, q * U), p = ldp<R, U>(v.p, q * U);
    Pack<R, U> t;
#pragma unroll
    for (int e = 0; e < U; ++e) t.e[e] = x.e[e] + alpha * p.e[e];
    stp<R, U>(v.xt, q * U, t);
  }
  for (long long i = nq * U + gid; i < v.n; i += gs) v.xt[i] = v.x[i] + alpha * v.p[i];
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
      S->drift = 0;
    }
  }
}

template <class R>
void launch_lbfgs_update(const LbfgsVec<R>& v, LbfgsState* S, const LbfgsOpts& o,
                         hipStream_t st, bool skip_c, const LossParts* loss) {
  LossParts lp;
  if (loss) {
    lp = *loss;
  } else {
    std::memset(&lp, 0, sizeof(lp));
    lp.n = -1;
  }
  // packed access needs every array and history slot aligned to a pack
  constexpr size_t kPackBytes = sizeof(R) * pack_u<R, 1, kPackBytesBC>();
  auto al = [&](const void* q) { return ((uintptr_t)q % kPackBytes) == 0; };
  const int vec = al(v.x) && al(v.g) && al(v.p) && al(v.xt) && al(v.gt) && al(v.S) && al(v.Y) &&
                  (v.ld % pack_u<R, 1, kPackBytesBC>()) == 0;
#define LB_A(MM) lb_pass_a_kernel<R, MM><<<v.nb, kThreads, 0, st>>>(v, S, o, vec, lp)
#define LB_B(MM) lb_pass_b_kernel<R, MM><<<v.nb, kThreads, 0, st>>>(v, S, o, vec)
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
  LB_SWITCH(LB_B)
#undef LB_SWITCH
#undef LB_B
#undef LB_A
  // skip_c: the next evaluation forms the trial point itself (kept tile order)
  if (!skip_c) lb_pass_c_kernel<R><<<v.nb, kThreads, 0, st>>>(v, S, o, vec);
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
                                       hipStream_t, bool, const LossParts*);                    \
  template void launch_gather_rows<R>(const R*, const int*, long long, int, R*, hipStream_t);   \
  template void launch_scatter_rows<R>(const R*, const int*, long long, int, R*, hipStream_t);
FRESCO_LB_INST(float)
FRESCO_LB_INST(double)

}  // namespace fresco
