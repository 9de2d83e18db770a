// Device-side L-BFGS state machine (see lbfgs.hip).
#pragma once

#include "common.h"

namespace fresco {

constexpr int kLbfgsMaxM = 16;

// decision of a trial step
enum { LB_IDLE = 0, LB_ACCEPT = 1, LB_REJECT = 2, LB_RESTART = 3, LB_INIT = 4 };
// vector passes: blocks of kLbfgsThreads; at least 16 elements per thread, but
// one block per CU of the chip (256) while a thread keeps 4 or more; at most
// kLbfgsMaxBlocks.  Every block of pass B reduces the partials of all blocks of
// pass A, with eight waves: 33 rows of 256 partials (m = 8, the 2D workload) in
// one round of loads.
constexpr int kLbfgsThreads = 512;
constexpr int kLbfgsMaxBlocks = 512;
inline int lbfgs_blocks(long long n) {
  long long nb = (n + 16LL * kLbfgsThreads - 1) / (16LL * kLbfgsThreads);
  const long long fill = (n + 4LL * kLbfgsThreads - 1) / (4LL * kLbfgsThreads);
  if (nb < fill && nb < 256) nb = fill < 256 ? fill : 256;
  if (nb > kLbfgsMaxBlocks) nb = kLbfgsMaxBlocks;
  if (nb < 1) nb = 1;
  return (int)nb;
}

inline long long lbfgs_slot_stride(long long n) { return (n + 3) / 4 * 4; }

// Lives in device memory (followed by the snapshot the direction pass reads); the
// host reads it back between batches of replays.
struct LbfgsState {
  int mode;       // 0 normal, 4 = first evaluation of a call
  int step;       // decision of the last replay (idle / accept / reject / restart / init)
  int k;          // stored pairs
  int head;       // ring slot of the newest pair
  int nbt;        // rejections in the current line search
  int iter;       // accepted iterations in this call
  int target;     // iterations requested for this call
  int nevals;     // evaluations in this call
  int fail;       // line search failed after a restart
  int converged;  // gradient RMS below gtol (or zero)
  int restarted;  // last restart not yet followed by a stored pair
  int resets;     // history resets
  int drift;      // a trial point left the slack of its cached tile order
  double f_cur;   // loss at the current point
  double f_trial; // loss at the trial point (written by the evaluation)
  double gtp;     // g . p at the current point
  double alpha;   // current step length along p
  double gamma;   // initial inverse-Hessian scaling s.y / y.y of the newest pair
  double gg;      // g . g at the current point
  double gnorm_rms;
  double coefG;   // p = -(coefG g + sum_j coefS_j s_j + coefY_j y_j)
  double coefS[kLbfgsMaxM];
  double coefY[kLbfgsMaxM];
  double SG[kLbfgsMaxM];  // s_j . g
  double YG[kLbfgsMaxM];  // y_j . g
  double SY[kLbfgsMaxM * kLbfgsMaxM];  // [i][j] = s_i . y_j (ring slots)
  double YY[kLbfgsMaxM * kLbfgsMaxM];  // [i][j] = y_i . y_j
  // [i][j] = (R^-1)_ij for pair i not newer than pair j (ring slots), R the upper
  // triangle of S^T Y in chronological order; extended by one column per stored
  // pair
  double RI[kLbfgsMaxM * kLbfgsMaxM];
};

struct LbfgsOpts {
  int m;
  int max_backtracks;
  double max_step;  // largest allowed |alpha p_j| per coordinate
  double c1;        // Armijo constant
  double shrink;    // backtracking factor
  double gtol;      // stop when the RMS gradient falls below (0: never)
};

template <class R>
struct LbfgsVec {
  R* x;   // current point (internal order)
  R* g;   // gradient at x
  R* p;   // search direction
  R* xt;  // trial point
  R* gt;  // gradient at xt
  R* S;   // m slots of s, ld elements apart
  R* Y;   // m slots of y, ld elements apart
  double* part0;  // block partials of pass A (4 m + 1 slots of nb)
  double* part1;  // block maxima of pass B (nb)
  long long n;    // vector length N d
  long long ld;   // slot stride of S and Y: n rounded up to a multiple of 4
  int m;
  int nb;         // blocks of the vector kernels
};

// Host side of an optimiser call: replays trial steps (replay(count) enqueues
// count of them) until the state reports a stop -- target iterations reached,
// convergence or line-search failure.  Replays go out in chunks of at most
// `chunk`, each followed by an asynchronous copy of the state to its own pinned
// host slot and an event; two chunks are in flight, so the host reads one
// chunk's copy while the next runs and the stream never waits on the host.
// Replays that run after the stop find the optimiser idle: they change no
// state and are not counted as evaluations (at most two chunks of them).
// host: pinned LbfgsState[2]; ev: two events.  Returns FRESCO_OK, replay's own
// status, or FRESCO_EHIP with the HIP error in *hip_err.
template <class F>
int lbfgs_replay_until_stop(hipStream_t st, LbfgsState* dev, LbfgsState* host, hipEvent_t ev[2],
                            int n_iter, int chunk, F&& replay, int* hip_err) {
#define LB_RCHK(x)                   \
  do {                               \
    hipError_t e_ = (x);             \
    if (e_ != hipSuccess) {          \
      *hip_err = (int)e_;            \
      return FRESCO_EHIP;            \
    }                                \
  } while (0)
  LB_RCHK(hipMemcpyAsync(&host[0], dev, sizeof(LbfgsState), hipMemcpyDeviceToHost, st));
  LB_RCHK(hipStreamSynchronize(st));
  LbfgsState h = host[0];
  int q_slot[2] = {0, 0}, q_cnt[2] = {0, 0};
  int q_head = 0, q_len = 0, next_slot = 0;
  long long inflight = 0;  // replays enqueued whose state copy has not been read
  while (!(h.iter >= n_iter || h.fail || h.converged)) {
    const long long need = (long long)n_iter - h.iter - inflight;
    if (need > 0 && q_len < 2) {
      const int cnt = (int)(need < chunk ? need : chunk);
      const int s = replay(cnt);
      if (s) return s;
      const int slot = next_slot;
      next_slot ^= 1;
      LB_RCHK(hipMemcpyAsync(&host[slot], dev, sizeof(LbfgsState), hipMemcpyDeviceToHost, st));
      LB_RCHK(hipEventRecord(ev[slot], st));
      const int q = (q_head + q_len) & 1;
      q_slot[q] = slot;
      q_cnt[q] = cnt;
      ++q_len;
      inflight += cnt;
      continue;
    }
    // here a chunk is in flight (with none, need = n_iter - iter > 0)
    const int slot = q_slot[q_head];
    inflight -= q_cnt[q_head];
    q_head ^= 1;
    --q_len;
    LB_RCHK(hipEventSynchronize(ev[slot]));
    h = host[slot];
  }
  LB_RCHK(hipStreamSynchronize(st));
#undef LB_RCHK
  return FRESCO_OK;
}

// replays per chunk of an optimiser call (at least; up to the max when one
// binning of the kept tile order serves that many trial steps)
constexpr int kLbfgsReplayChunk = 8;
constexpr int kLbfgsMaxReplayChunk = 16;

// S: two states in device memory, S[0] the state and S[1] the snapshot of it that
// the first pass leaves for the second (whose block 0 rewrites S[0]).
// skip_c: no trial point pass (the next evaluation keeps the tile order of the
// last binning and forms the trial point in its spreading pass, KeptSpread);
// loss: the evaluation's loss partials, summed into f_trial by the first pass
// (else f_trial holds the loss already)
template <class R>
void launch_lbfgs_update(const LbfgsVec<R>& v, LbfgsState* S, const LbfgsOpts& o,
                         hipStream_t st, bool skip_c = false, const LossParts* loss = nullptr);
void launch_lbfgs_set_mode(LbfgsState* S, int mode, int target, hipStream_t st);
template <class R>
void launch_gather_rows(const R* src, const int* idx, long long n, int d, R* dst, hipStream_t st);
template <class R>
void launch_scatter_rows(const R* src, const int* idx, long long n, int d, R* dst,
                         hipStream_t st);

}  // namespace fresco
