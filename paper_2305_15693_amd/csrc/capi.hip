// C ABI of the FReSCo loss/gradient library: context lifetime, argument
// checking, buffers and the launch sequence of one evaluation.
//
// One evaluation of L_S and its gradient (the NUwU variant of the Methods: a
// type-1 transform for S, a type-2 transform for the gradient) is, on the
// context's stream:
//   bin      wrap, split and counting-sort the points by tile        (spread.hip)
//   spread   tiles -> padded tile sums -> fold into the fine grid b  (spread.hip)
//   rows     b -> half spectrum along axis 0                         (fft.hip)
//   cols     remaining axes; the last forward axis is fused with the mode
//            stage (deconvolve, S, loss, field coefficients) and with the
//            first inverse transform                                  (fft.hip)
//   cols/rows inverse transforms back to one real field              (fft.hip)
//   interp   derivative of the field at every point = gradient        (spread.hip)
//   finish   FP64 loss partials -> loss; non-finite flag             (here)
// The asynchronous entry point replays a captured HIP graph of this sequence
// when it sees the same buffers again.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "common.h"
#include "fft.h"
#include "lbfgs.h"
#include "pair.h"
#include "plan.h"

using namespace fresco;

static int g_last_hip = 0;

#define HIPCHK(x)                       \
  do {                                  \
    hipError_t e_ = (x);                \
    if (e_ != hipSuccess) {             \
      g_last_hip = (int)e_;             \
      return FRESCO_EHIP;               \
    }                                   \
  } while (0)

namespace {

template <class R>
struct State {
  AxisFft<R> ax[3];  // [0] rows: complex length nf0/2; [1], [2]: columns along axes 1, 2
  BinPlan bp;
  BinBuffers bb;
  R* tiles = nullptr;  // padded spreading tiles
  int* fold_off[3] = {nullptr, nullptr, nullptr};
  int2* fold_ent[3] = {nullptr, nullptr, nullptr};
  int fold_nent[3] = {0, 0, 0};    // entries per axis
  bool fold_fused = false;         // fold done inside the forward row pass
  R* grid = nullptr;
  cpx<R>* A1 = nullptr;  // half spectrum after the row pass
  cpx<R>* A2 = nullptr;  // 3D: after the axis-1 pass
  cpx<R>* V2 = nullptr;  // 3D: field after the inverse axis-2 pass
  cpx<R>* V1 = nullptr;  // field before the inverse row pass
  R* v = nullptr;        // real field
  R* dec[3] = {nullptr, nullptr, nullptr};
  R* deci[3] = {nullptr, nullptr, nullptr};
  R* Wp = nullptr;
  R* S0p = nullptr;
  R* Wm = nullptr;
  R* S0m = nullptr;
  cpx<R>* rho = nullptr;
  double* loss_part = nullptr;
  double* loss_dev = nullptr;
  int* flag_out = nullptr;
  RowParams<R> rows;
  ColParams<R> col1;  // axis 1 (3D: forward / inverse; 2D: fused)
  ColParams<R> col2;  // axis 2 (3D: fused)
  // 2D columns too long for LDS: two half-length sub-transforms per column
  bool long_cols = false;
  cpx<R>* twn = nullptr;  // exp(+2 pi i q / nf1)
  cpx<R>* Yl = nullptr;   // forward sub-transforms [2][2M1+1][M0+1]
  cpx<R>* Ql = nullptr;   // pre-twiddled inverse inputs, same layout
  ColParams<R> lfw{}, linv{};
  int long_blocks = 0;
  long long nloss_part = 0;
  // L-BFGS (allocated on the first fresco_step)
  LbfgsVec<R> lv{};
  LbfgsState* lst = nullptr;
  LbfgsState* lst_host = nullptr;  // pinned copies [2] (one per chunk in flight)
  hipEvent_t lb_ev[2] = {nullptr, nullptr};
  int* perm0 = nullptr;            // internal order -> caller's index
  bool have_perm0 = false;
  int lb_m = 0;
  LbfgsOpts lb_opts{};
  bool cached_eval = false;  // the last binning kept the previous tile order
  hipGraphExec_t lb_graph = nullptr;        // one trial step
  hipGraphExec_t lb_graph_chunk = nullptr;  // one chunk of trial steps (its length
                                            // follows the options, which drop it)
  void drop_lb_graphs() {
    if (lb_graph) (void)hipGraphExecDestroy(lb_graph);
    if (lb_graph_chunk) (void)hipGraphExecDestroy(lb_graph_chunk);
    lb_graph = lb_graph_chunk = nullptr;
  }
  // point strengths (fresco_set_strengths): a copy in the caller's order, the
  // optimiser's internal order, S normalised by rho0 = sum c^2
  bool has_str = false;
  R* cdev = nullptr;
  R* cint = nullptr;
  double* cstat = nullptr;      // [3 * kStatBlocks + 3] partials, then sum c^2, max |c|, bad
  double* fsum_part = nullptr;  // [nloss_part] partials of sum_K W S (S - S0)
  double rho0 = 0.0, cmax = 1.0;
  // strengths and field-value output of the evaluation being enqueued
  const R* str_eval = nullptr;
  R* val_eval = nullptr;
  // pair-correlation loss (fresco_set_pair_correlation_target): target and
  // weights on the fine grid, the grid b = 2 W_g (g - g0), loss partials
  R* g0 = nullptr;
  R* wg = nullptr;
  R* gb = nullptr;
  double* gpart = nullptr;
  bool has_g = false;
};

constexpr int kGlossBlocks = 1024;

constexpr int kStatBlocks = 256;

struct GraphEntry {
  const void* pos;
  const void* loss;
  const void* grad;
  hipGraphExec_t exec;
};

}  // namespace

struct fresco_ctx {
  Geom g;
  int dtype;
  hipStream_t st;
  long long n_constrained;
  long long bytes = 0;
  std::vector<void*> allocs;
  std::vector<size_t> alloc_bytes;  // size of each entry of allocs
  long long mem_limit = 0;          // device bytes the context may hold (0: no limit)
  double* host_loss = nullptr;  // pinned
  int* host_flag = nullptr;     // pinned
  void* state = nullptr;
  bool use_graphs = true;
  std::vector<GraphEntry> graphs;
  // positions of the latest fresco_structure_factor whose rho and point order are
  // still held (cleared by every other evaluation)
  const void* sf_pos = nullptr;
  // soft-core pair term added to every loss evaluation (not owned)
  fresco_pair_ctx* pair = nullptr;
  double pair_w = 0.0;
  // per-stage timing (diagnostics): event pairs recorded on the stream
  uint32_t timing_mask = 0;
  int timing_reps = 1;  // launches per timed spreading / interpolation stage
  std::vector<hipEvent_t> event_pool;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> pending[FRESCO_STAGE_COUNT];
  std::vector<int> pending_reps[FRESCO_STAGE_COUNT];
  double stage_ms[FRESCO_STAGE_COUNT] = {};
  long long stage_n[FRESCO_STAGE_COUNT] = {};
};

namespace {

hipEvent_t take_event(fresco_ctx* c) {
  if (!c->event_pool.empty()) {
    hipEvent_t e = c->event_pool.back();
    c->event_pool.pop_back();
    return e;
  }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Brackets the launches of one stage with events when its timing bit is set.
// reps: how many times the bracketed launches run (the timing repetitions of
// the spreading and interpolation stages, whose kernels only read their inputs
// and write their outputs; 1 otherwise and when the stage is not timed)
struct StageTimer {
  fresco_ctx* c;
  int s;
  int reps = 1;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  StageTimer(fresco_ctx* c_, int s_) : c(c_), s(s_) {
    if (c->timing_mask & (1u << s)) {
      e0 = take_event(c);
      e1 = take_event(c);
      if (e0 && e1) (void)hipEventRecord(e0, c->st);
      if (e0 && e1 && (s == FRESCO_STAGE_SPREAD || s == FRESCO_STAGE_INTERP)) reps = c->timing_reps;
    }
  }
  ~StageTimer() {
    if (e0 && e1) {
      (void)hipEventRecord(e1, c->st);
      c->pending[s].push_back({e0, e1});
      c->pending_reps[s].push_back(reps);
    } else {
      if (e0) c->event_pool.push_back(e0);
      if (e1) c->event_pool.push_back(e1);
    }
  }
};

int dalloc(fresco_ctx* c, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 16;
  if (c->mem_limit > 0 && c->bytes + (long long)bytes > c->mem_limit) {
    g_last_hip = (int)hipErrorOutOfMemory;
    return FRESCO_ENOMEM;
  }
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    g_last_hip = (int)e;
    (void)hipGetLastError();
    return FRESCO_ENOMEM;
  }
  c->allocs.push_back(*p);
  c->alloc_bytes.push_back(bytes);
  c->bytes += (long long)bytes;
  return FRESCO_OK;
}

// Frees one buffer of the context (no-op for NULL); the caller has made sure
// the stream no longer uses it.
template <class T>
void dfree(fresco_ctx* c, T*& p) {
  if (!p) return;
  for (size_t i = 0; i < c->allocs.size(); ++i)
    if (c->allocs[i] == (void*)p) {
      (void)hipFree(c->allocs[i]);
      c->bytes -= (long long)c->alloc_bytes[i];
      c->allocs.erase(c->allocs.begin() + (long)i);
      c->alloc_bytes.erase(c->alloc_bytes.begin() + (long)i);
      break;
    }
  p = nullptr;
}

template <class T>
int dalloc_t(fresco_ctx* c, T** p, size_t count) {
  void* q = nullptr;
  int st = dalloc(c, &q, count * sizeof(T));
  *p = (T*)q;
  return st;
}

// a new device array *dst holding src in the working precision
template <class R>
int upload(fresco_ctx* c, R** dst, const std::vector<double>& src) {
  int st = dalloc_t(c, dst, src.size());
  if (st) return st;
  std::vector<R> tmp(src.size());
  for (size_t i = 0; i < src.size(); ++i) tmp[i] = (R)src[i];
  HIPCHK(hipMemcpy(*dst, tmp.data(), tmp.size() * sizeof(R), hipMemcpyHostToDevice));
  return FRESCO_OK;
}

// src into the device array *dst: a new one when *dst is NULL, else the existing
// one overwritten in place (same size; the caller has drained the stream)
template <class R>
int upload_into(fresco_ctx* c, R** dst, const std::vector<double>& src) {
  if (!*dst) return upload<R>(c, dst, src);
  std::vector<R> tmp(src.size());
  for (size_t i = 0; i < src.size(); ++i) tmp[i] = (R)src[i];
  HIPCHK(hipMemcpy(*dst, tmp.data(), tmp.size() * sizeof(R), hipMemcpyHostToDevice));
  return FRESCO_OK;
}

template <class T>
int upload_raw(fresco_ctx* c, T** dst, const std::vector<T>& src) {
  int st = dalloc_t(c, dst, src.size());
  if (st) return st;
  HIPCHK(hipMemcpy(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice));
  return FRESCO_OK;
}

template <class R>
int setup_axis(fresco_ctx* c, AxisFft<R>* ax, int n, bool rows_twn) {
  if (!plan_factors(n, &ax->F, &ax->rmin)) return FRESCO_ENOTSUP;
  std::vector<double> t = twiddles(n, n);
  R* p = nullptr;
  int st = upload<R>(c, &p, t);
  if (st) return st;
  ax->tw = (cpx<R>*)p;
  if (rows_twn) {
    std::vector<double> t2 = twiddles(2 * n, n);
    st = upload<R>(c, &p, t2);
    if (st) return st;
    ax->twN = (cpx<R>*)p;
  }
  return FRESCO_OK;
}

constexpr size_t kLdsLimit = 160 * 1024;

// launch shape of a row pass: lines per block, block size, twiddles in LDS
bool shape_rows(int H, int rmin, long long nrows, size_t cs, int* lpb, int* threads, bool* twl) {
  int l = 1;
  while (l * 2 <= 16 && (size_t)(l * 2) * (H + 1) * cs <= 32768 && nrows / (l * 2) >= 1024) l *= 2;
  int t = 256;
  for (;;) {
    int JT = t / l;
    int need = (H + rmin * JT - 1) / (rmin * JT);
    if (need <= 8) break;
    if (t < 1024) t *= 2;
    else if (l > 1) l /= 2;
    else return false;
  }
  // twiddles go to LDS when they fit beside the lines, else they are read from L2
  const size_t lines = (size_t)l * (H + 1) * cs;
  if (lines > kLdsLimit) return false;
  *twl = lines + (size_t)H * cs <= kLdsLimit;
  *lpb = l;
  *threads = t;
  return true;
}

// launch shape of a column pass: columns per block, block size, twiddles in LDS
bool shape_cols(int n, int rmin, long long ncols, size_t cs, int* bc, int* threads, bool* twl) {
  int b = 1;
  while (b * 2 <= 16 && (size_t)(b * 2) * n * cs <= 49152 && ncols / (b * 2) >= 512) b *= 2;
  // one column per workgroup (few, long columns: the 2D mode pass, 301 columns
  // of 1250): 512 threads to start with, fewer butterflies per thread in every
  // stage (22.5 -> 20.2 us); several columns: 256 (the 3D passes measured
  // slower with 512)
  int t = (b == 1) ? 512 : 256;
  for (;;) {
    int JT = t / b;
    int need = (n + rmin * JT - 1) / (rmin * JT);
    if (need <= 8) break;
    if (t < 1024) t *= 2;
    else if (b > 1) b /= 2;
    else return false;
  }
  // data + mode factors (at most half a line per column); twiddles as for rows
  const size_t data = (size_t)b * ((size_t)n + n / 2 + 1) * cs;
  if (data > kLdsLimit) return false;
  *twl = data + (size_t)n * cs <= kLdsLimit;
  *bc = b;
  *threads = t;
  return true;
}

// loss = sum of the block partials (fixed order), plus w2 times the sum of a
// second set (an attached pair term); hand the non-finite flag to the
// host-visible slot and clear it for the next evaluation
__global__ void finish_kernel(const double* __restrict__ part, long long n,
                              const double* __restrict__ part2, long long n2, double w2,
                              double* __restrict__ out, int* __restrict__ flag,
                              int* __restrict__ flag_out) {
  __shared__ double s[256];
  const double a = block_sum_256(part, n, s);
  const double b = (n2 > 0) ? block_sum_256(part2, n2, s) : 0.0;
  if (threadIdx.x == 0) {
    if (out) out[0] = (n2 > 0) ? a + w2 * b : a;
    flag_out[0] = flag[0];
    flag[0] = 0;
  }
}

// per-axis CSR of the padded tiles covering each grid coordinate
int build_fold_tables(fresco_ctx* c, int a, int** off_d, int2** ent_d, int* nent) {
  const Geom& g = c->g;
  const int nf = g.nf[a], T = g.T[a], E = g.E[a], nt = g.nt[a];
  std::vector<std::vector<int2>> lists(nf);
  for (int t = 0; t < nt; ++t)
    for (int l = 0; l < E; ++l) {
      // the padded tile starts g.slack cells before the tile
      const int y = (int)((((long long)t * T - g.slack + l) % nf + nf) % nf);
      lists[y].push_back(make_int2(t, l));
    }
  std::vector<int> off(nf + 1, 0);
  std::vector<int2> ent;
  for (int y = 0; y < nf; ++y) {
    off[y] = (int)ent.size();
    for (auto& e : lists[y]) ent.push_back(e);
  }
  off[nf] = (int)ent.size();
  *nent = (int)ent.size();
  int st;
  if ((st = upload_raw(c, off_d, off))) return st;
  if ((st = upload_raw(c, ent_d, ent))) return st;
  return FRESCO_OK;
}

template <class R>
int create_state(fresco_ctx* c) {
  State<R>* S = new (std::nothrow) State<R>();
  if (!S) return FRESCO_ENOMEM;
  c->state = S;
  Geom& g = c->g;
  const int d = g.d;
  const size_t cs = sizeof(cpx<R>);
  int st;
  // FFT plans
  if ((st = setup_axis<R>(c, &S->ax[0], g.nf[0] / 2, true))) return st;
  if ((st = setup_axis<R>(c, &S->ax[1], g.nf[1], false))) return st;
  if (d == 3 && (st = setup_axis<R>(c, &S->ax[2], g.nf[2], false))) return st;
  // binning
  const long long N = g.N;
  BinPlan& bp = S->bp;
  bp.mode = BIN_ATOMIC;
  bp.G = 1;
  bp.nkeys = g.nbins;
  bp.shift = 16;
  bp.nblk = 0;
  bp.chunk = 0;
  bp.levels = 1;
  std::memset(&bp.coarse, 0, sizeof(bp.coarse));
  // histogram passes: chunks that are a multiple of 256 points (the scatter
  // pass finds its chunk from the block index) whose ranks fit in 32 - shift
  // bits; returns false when more than `max_blocks` chunks would be needed
  auto plan_level = [&](long long nkeys, long long G, bool tiles, long long max_blocks,
                        BinLevel* out) {
    int shift = 0;
    while ((1ll << shift) < nkeys) ++shift;
    if (tiles) shift = 16;
    const long long cmax = ((1ll << (32 - shift)) - 1) / 256 * 256;
    // tiles: chunks of 4096 points, at most 256 of them (longer runs per tile
    // for the scatter, a smaller count table; 3D 1e7 points: bin 422 -> 353 us
    // against 1024 chunks)
    long long nblk = tiles ? N / 4096 : N / 65536;
    if (nblk < 1) nblk = 1;
    if (nblk > (tiles ? 256 : 2048)) nblk = (tiles ? 256 : 2048);
    long long chunk = ((N + nblk - 1) / nblk + 255) / 256 * 256;
    if (chunk > cmax) chunk = cmax;
    nblk = (N + chunk - 1) / chunk;
    out->nblk = (int)nblk;
    out->chunk = chunk;
    out->nkeys = nkeys;
    out->G = G;
    out->kdiv = make_fastdiv((uint32_t)G);
    out->shift = shift;
    return nblk <= max_blocks;
  };
  {
    // keys: the tiles themselves, or ranges of G consecutive tiles (at most
    // 8192 ranges of at most 4096 tiles, so both LDS tables stay small)
    long long G = 1, nkeys = g.nbins;
    int mode = BIN_TILES;
    // FRESCO_BIN_RANGES=K sorts in two levels with at most K ranges whatever
    // the tile count (checks of the large-grid path at small sizes)
    const char* er = std::getenv("FRESCO_BIN_RANGES");
    long long kmax = er ? std::atoll(er) : 0;
    if (kmax < 1 || kmax > 8192) kmax = 0;
    if (kmax || g.nbins > 16384) {
      if (!kmax) kmax = 8192;
      G = (g.nbins + kmax - 1) / kmax;
      nkeys = (g.nbins + G - 1) / G;
      mode = BIN_RANGES;
    }
    BinLevel lv;
    if (plan_level(nkeys, G, mode == BIN_TILES, mode == BIN_TILES ? 4096 : 8192, &lv) &&
        G <= 4096) {
      bp.mode = mode;
      bp.G = (int)G;
      bp.nkeys = nkeys;
      bp.shift = lv.shift;
      bp.nblk = lv.nblk;
      bp.chunk = lv.chunk;
    }
    // FRESCO_BIN_LEVELS=2: a coarse pass over about sqrt(ranges) groups of
    // consecutive ranges first, so that each chunk of the range pass meets few
    // ranges.  Off by default: with one store per point the range pass runs as
    // fast from the caller's order (N = 1e9: 118 ms per evaluation either way)
    // and the coarse pass holds another 12 bytes per point.
    if (bp.mode == BIN_RANGES) {
      const char* el = std::getenv("FRESCO_BIN_LEVELS");
      const bool two = el && el[0] == '2' && bp.nkeys > 1;
      if (two) {
        long long k0 = 1;
        while (k0 * k0 < bp.nkeys) ++k0;
        const long long q = (bp.nkeys + k0 - 1) / k0;  // ranges per coarse key
        const long long G0 = (long long)bp.G * q;
        if (plan_level((g.nbins + G0 - 1) / G0, G0, false, 8192, &bp.coarse)) bp.levels = 2;
      }
    }
    // FRESCO_BIN_ATOMIC=1: the global-atomic fallback (grids or point counts
    // beyond both sorts) at any size, for checks
    const char* ea = std::getenv("FRESCO_BIN_ATOMIC");
    if (ea && ea[0] == '1') {
      bp.mode = BIN_ATOMIC;
      bp.G = 1;
      bp.nkeys = g.nbins;
      bp.levels = 1;
    }
  }
  bp.kdiv = make_fastdiv((uint32_t)bp.G);
  BinBuffers& bb = S->bb;
  if ((st = dalloc_t(c, &bb.kr, N))) return st;
  if (bp.mode != BIN_ATOMIC) {
    if ((st = dalloc_t(c, &bb.H, (size_t)bp.nkeys * bp.nblk))) return st;
  } else {
    if ((st = dalloc_t(c, &bb.key, N))) return st;
  }
  if (bp.mode == BIN_RANGES) {
    if ((st = dalloc_t(c, &bb.kstart, bp.nkeys + 1))) return st;
    R* tpos = nullptr;
    if ((st = dalloc_t(c, &tpos, (size_t)N * d))) return st;
    bb.tpos = tpos;
    if ((st = dalloc_t(c, &bb.tidx, N))) return st;
    if (bp.levels == 2) {
      const BinLevel& cl = bp.coarse;
      if ((st = dalloc_t(c, &bb.kr0, N))) return st;
      if ((st = dalloc_t(c, &bb.H0, (size_t)cl.nkeys * cl.nblk))) return st;
      if ((st = dalloc_t(c, &bb.count0, cl.nkeys))) return st;
      if ((st = dalloc_t(c, &bb.kstart0, cl.nkeys + 1))) return st;
      R* tpos0 = nullptr;
      if ((st = dalloc_t(c, &tpos0, (size_t)N * d))) return st;
      bb.tpos0 = tpos0;
      if ((st = dalloc_t(c, &bb.tidx0, N))) return st;
    }
  }
  if ((st = dalloc_t(c, &bb.count, bp.nkeys))) return st;
  if ((st = dalloc_t(c, &bb.start, g.nbins + 1))) return st;
  Rec<R>* rec = nullptr;
  if ((st = dalloc_t(c, &rec, N))) return st;
  bb.rec = rec;
  if ((st = dalloc_t(c, &bb.perm, N))) return st;
  if ((st = dalloc_t(c, &bb.flag, 1))) return st;
  if ((st = dalloc_t(c, &S->flag_out, 1))) return st;
  HIPCHK(hipMemset(bb.flag, 0, sizeof(int)));
  HIPCHK(hipMemset(S->flag_out, 0, sizeof(int)));
  // spreading tiles and fold tables
  const long long tcells = (long long)g.E[0] * g.E[1] * (d == 3 ? g.E[2] : 1);
  if ((st = dalloc_t(c, &S->tiles, (size_t)(g.nbins * tcells)))) return st;
  for (int a = 0; a < d; ++a)
    if ((st = build_fold_tables(c, a, &S->fold_off[a], &S->fold_ent[a], &S->fold_nent[a])))
      return st;
  // grids
  const long long H0 = g.M[0] + 1;
  const long long P1 = 2 * g.M[1] + 1;
  const long long nf1 = g.nf[1], nf2 = (d == 3) ? g.nf[2] : 1;
  if ((st = dalloc_t(c, &S->grid, g.ngrid))) return st;
  if ((st = dalloc_t(c, &S->A1, nf2 * nf1 * H0))) return st;
  if (d == 3 && (st = dalloc_t(c, &S->A2, nf2 * P1 * H0))) return st;
  if (d == 3 && (st = dalloc_t(c, &S->V2, nf2 * P1 * H0))) return st;
  if ((st = dalloc_t(c, &S->V1, nf2 * nf1 * H0))) return st;
  if ((st = dalloc_t(c, &S->v, g.ngrid))) return st;
  // deconvolution factors h_a / psihat_a(n) for both kernels
  for (int a = 0; a < d; ++a) {
    const double h = 2.0 * M_PI / g.nf[a];
    std::vector<double> ph = kernel_fourier(g.M[a], g.w, g.beta, g.nf[a], false);
    for (auto& x : ph) x = h / x;
    if ((st = upload<R>(c, &S->dec[a], ph))) return st;
    std::vector<double> pi = kernel_fourier(g.M[a], g.wi, g.beta_i, g.nf[a], true);
    for (auto& x : pi) x = h / x;
    if ((st = upload<R>(c, &S->deci[a], pi))) return st;
  }
  if ((st = dalloc_t(c, &S->rho, g.nhalf))) return st;
  if ((st = dalloc_t(c, &S->loss_dev, 1))) return st;

  // launch shapes
  RowParams<R>& rp = S->rows;
  std::memset(&rp, 0, sizeof(rp));
  rp.nrows = nf1 * nf2;
  rp.M0 = g.M[0];
  rp.rstride = g.M[0] + 1;
  rp.kstride = 1;
  if (!shape_rows(g.nf[0] / 2, S->ax[0].rmin, rp.nrows, cs, &rp.lines_per_block, &rp.threads,
                  &rp.tw_lds))
    return FRESCO_ENOTSUP;
  {
    // fold inside the forward row pass when the first axis's cover lists fit
    // in LDS beside the lines (FRESCO_FOLD=0 keeps the stand-alone fold kernel)
    RowFold<R>& f = rp.fold;
    f.tiles = S->tiles;
    for (int a = 0; a < 3; ++a) {
      f.off[a] = S->fold_off[a];
      f.ent[a] = S->fold_ent[a];
    }
    f.nent0 = S->fold_nent[0];
    f.d = d;
    f.nf0 = g.nf[0];
    f.nf1 = g.nf[1];
    f.E0 = g.E[0];
    f.E1 = g.E[1];
    f.nt0 = g.nt[0];
    f.nt1 = g.nt[1];
    f.ncell = (long long)g.E[0] * g.E[1] * (d == 3 ? g.E[2] : 1);
    bool fuse = true;
    const char* ef = std::getenv("FRESCO_FOLD");
    if (ef && ef[0] == '0') fuse = false;
    if (fuse && rows_lds_bytes<R>(rp, S->ax[0]) > kLdsLimit) fuse = false;
    if (!fuse) std::memset(&f, 0, sizeof(f));
    S->fold_fused = fuse;
  }
  auto fill_modes = [&](ColParams<R>& cp) {
    cp.d = d;
    cp.M0 = g.M[0];
    cp.M1 = g.M[1];
    cp.M2 = (d == 3) ? g.M[2] : 0;
    cp.P1 = 2 * g.M[1] + 1;
    cp.P2 = (d == 3) ? 2 * g.M[2] + 1 : 1;
    cp.h0div = make_fastdiv((uint32_t)H0);
    for (int a = 0; a < 3; ++a) {
      cp.dec[a] = (a < d) ? S->dec[a] : nullptr;
      cp.deci[a] = (a < d) ? S->deci[a] : nullptr;
    }
    cp.invN = (R)(1.0 / (double)g.N);
    cp.g_scale = (R)(1.0 / (double)g.N);
    cp.mcol = true;  // the long-column path (rows of modes) clears it
  };
  ColParams<R>& c1 = S->col1;
  std::memset(&c1, 0, sizeof(c1));
  fill_modes(c1);
  if (d == 2) {
    // fused pass along axis 1 over the H0 columns of A1[l1][n0]
    c1.ncols = H0;
    c1.M = g.M[1];
    c1.cdiv = make_fastdiv((uint32_t)H0);
    c1.in_line = H0;
    c1.out_line = H0;
    const char* el = std::getenv("FRESCO_LONG_COLS");
    const bool force_long = el && el[0] == '1' && (2 * g.M[1] + 1) * 2 <= g.nf[1];
    if (!force_long &&
        shape_cols(g.nf[1], S->ax[1].rmin, c1.ncols, cs, &c1.bc, &c1.threads, &c1.tw_lds)) {
      S->nloss_part = (c1.ncols + c1.bc - 1) / c1.bc;
      // half spectrum column-major (each column contiguous for the column
      // pass; the row passes, which have one workgroup per row, take the
      // strided accesses, with 16 consecutive rows per XCD).
      // FRESCO_ROW_MAJOR=1 keeps the row-major layout.
      const char* erm = std::getenv("FRESCO_ROW_MAJOR");
      if (rp.lines_per_block == 1 && !(erm && erm[0] == '1')) {
        rp.rstride = 1;
        rp.kstride = nf1;
        rp.xcd16 = 1;
        c1.cdiv = make_fastdiv(1u);
        c1.in_outer = nf1;
        c1.out_outer = nf1;
        c1.in_line = 1;
        c1.out_line = 1;
      }
      HIPCHK(prepare_cols<R>(COL_FUSED, c1, S->ax[1]));
      HIPCHK(prepare_cols<R>(COL_SF, c1, S->ax[1]));
      HIPCHK(prepare_cols<R>(COL_BWD, c1, S->ax[1]));
      HIPCHK(prepare_cols<R>(COL_GFIELD, c1, S->ax[1]));
      HIPCHK(prepare_cols<R>(COL_GBACK, c1, S->ax[1]));
    } else {
      // columns too long for LDS: two half-length sub-transforms per column
      // (decimation by 2; nf1 is even and 2M + 1 <= nf1 / 2)
      S->long_cols = true;
      c1.mcol = false;
      const int n = g.nf[1], m = n / 2;
      const long long P = 2LL * g.M[1] + 1;
      if ((st = setup_axis<R>(c, &S->ax[1], m, false))) return st;
      {
        std::vector<double> t = twiddles(n, n);
        R* q = nullptr;
        if ((st = upload<R>(c, &q, t))) return st;
        S->twn = (cpx<R>*)q;
      }
      if ((st = dalloc_t(c, &S->Yl, (size_t)(2 * P * H0)))) return st;
      if ((st = dalloc_t(c, &S->Ql, (size_t)(2 * P * H0)))) return st;
      // forward: column (r, n0) holds the entries 2 i + r of column n0
      ColParams<R>& f = S->lfw;
      f = c1;
      f.ncols = 2 * H0;
      f.in_outer = H0;
      f.in_line = 2 * H0;
      f.out_outer = P * H0;
      f.out_line = H0;
      if (!shape_cols(m, S->ax[1].rmin, f.ncols, cs, &f.bc, &f.threads, &f.tw_lds))
        return FRESCO_ENOTSUP;
      HIPCHK(prepare_cols<R>(COL_FWD, f, S->ax[1]));
      // inverse: component r writes the entries 2 j + r of every column
      ColParams<R>& v = S->linv;
      v = c1;
      v.ncols = H0;
      v.in_outer = 0;
      v.in_line = H0;
      v.out_outer = 0;
      v.out_line = 2 * H0;
      if (!shape_cols(m, S->ax[1].rmin, v.ncols, cs, &v.bc, &v.threads, &v.tw_lds))
        return FRESCO_ENOTSUP;
      HIPCHK(prepare_cols<R>(COL_INV, v, S->ax[1]));
      long long blocks = (P * H0 + 255) / 256;
      if (blocks > 4096) blocks = 4096;
      S->long_blocks = (int)blocks;
      S->nloss_part = blocks;
    }
  } else {
    // axis 1, columns (l2, n0): A1[l2][l1][n0] <-> A2[l2][m1][n0]
    c1.ncols = nf2 * H0;
    c1.M = g.M[1];
    c1.cdiv = make_fastdiv((uint32_t)H0);
    if (!shape_cols(g.nf[1], S->ax[1].rmin, c1.ncols, cs, &c1.bc, &c1.threads, &c1.tw_lds))
      return FRESCO_ENOTSUP;
    HIPCHK(prepare_cols<R>(COL_FWD, c1, S->ax[1]));
    HIPCHK(prepare_cols<R>(COL_INV, c1, S->ax[1]));
    ColParams<R>& c2 = S->col2;
    std::memset(&c2, 0, sizeof(c2));
    fill_modes(c2);
    c2.ncols = P1 * H0;
    c2.M = g.M[2];
    c2.cdiv = make_fastdiv((uint32_t)c2.ncols);
    c2.in_line = P1 * H0;
    c2.out_line = P1 * H0;
    if (!shape_cols(g.nf[2], S->ax[2].rmin, c2.ncols, cs, &c2.bc, &c2.threads, &c2.tw_lds))
      return FRESCO_ENOTSUP;
    S->nloss_part = (c2.ncols + c2.bc - 1) / c2.bc;
    HIPCHK(prepare_cols<R>(COL_FUSED, c2, S->ax[2]));
    HIPCHK(prepare_cols<R>(COL_SF, c2, S->ax[2]));
    HIPCHK(prepare_cols<R>(COL_BWD, c2, S->ax[2]));
    HIPCHK(prepare_cols<R>(COL_GFIELD, c2, S->ax[2]));
    HIPCHK(prepare_cols<R>(COL_GBACK, c2, S->ax[2]));
  }
  HIPCHK(prepare_rows<R>(rp, S->ax[0]));
  HIPCHK(spread_prepare<R>(g));
  HIPCHK(hipGetLastError());
  if ((st = dalloc_t(c, &S->loss_part, S->nloss_part))) return st;
  return FRESCO_OK;
}

// half-spectrum weights from the caller's cubes
template <class R>
int upload_weights(fresco_ctx* c, const std::vector<double>& Wc, const std::vector<double>& S0c) {
  State<R>* S = (State<R>*)c->state;
  const Geom& g = c->g;
  const int d = g.d;
  const long long H0 = g.M[0] + 1, P1 = 2 * g.M[1] + 1, P2 = (d == 3) ? 2 * g.M[2] + 1 : 1;
  const long long nlast = (d == 2) ? P1 : P2;
  const long long ncols = (d == 2) ? H0 : P1 * H0;
  const bool long_cols = S->long_cols;
  std::vector<double> wp(g.nhalf), sp(g.nhalf), wm(g.nhalf), sm(g.nhalf);
  auto cube_index = [&](int n0, int n1, int n2) -> long long {
    if (d == 2) return (long long)(n0 + g.M[0]) * P1 + (n1 + g.M[1]);
    return ((long long)(n0 + g.M[0]) * P1 + (n1 + g.M[1])) * P2 + (n2 + g.M[2]);
  };
  for (long long m = 0; m < nlast; ++m) {
    for (long long cidx = 0; cidx < ncols; ++cidx) {
      int n0, n1, n2 = 0;
      if (d == 2) {
        n0 = (int)cidx;
        n1 = (int)m - g.M[1];
      } else {
        n0 = (int)(cidx % H0);
        n1 = (int)(cidx / H0) - g.M[1];
        n2 = (int)m - g.M[2];
      }
      // column-major [c][m] for the column pass (each column reads its modes
      // contiguously); [m][c] for the long-column recombination, which walks
      // rows of modes
      const long long h = long_cols ? cidx + ncols * m : cidx * nlast + m;
      const long long ip = cube_index(n0, n1, n2), im = cube_index(-n0, -n1, -n2);
      wp[h] = Wc[ip];
      sp[h] = S0c[ip];
      wm[h] = Wc[im];
      sm[h] = S0c[im];
    }
  }
  int st;
  if ((st = upload_into<R>(c, &S->Wp, wp))) return st;
  if ((st = upload_into<R>(c, &S->S0p, sp))) return st;
  if ((st = upload_into<R>(c, &S->Wm, wm))) return st;
  if ((st = upload_into<R>(c, &S->S0m, sm))) return st;
  return FRESCO_OK;
}

// Targets and weights on the full mode cube from the caller's arrays (Methods,
// "Analytical gradients": W = w / S0^2 where S0 != 0 for the relative loss);
// w NULL: weight 1 on 0 < |n| <= k_cut.  Returns 1 for a negative or
// non-finite weight or a non-finite target.
int build_weights(const Geom& g, const double* s0, const double* w, double k_cut,
                  int weight_mode, std::vector<double>& Wc, std::vector<double>& S0c,
                  long long* ncons) {
  const int d = g.d;
  Wc.assign(g.ncube, 0.0);
  S0c.assign(g.ncube, 0.0);
  if (s0)
    for (long long i = 0; i < g.ncube; ++i) S0c[i] = s0[i];
  *ncons = 0;
  int bad = 0;
  for (long long i = 0; i < g.ncube; ++i) {
    long long r = i;
    long long n2 = 0;
    bool zero = true;
    for (int a = d - 1; a >= 0; --a) {
      long long P = 2LL * g.M[a] + 1;
      long long na = r % P - g.M[a];
      r /= P;
      n2 += na * na;
      if (na != 0) zero = false;
    }
    double wv;
    if (w) wv = w[i];
    else wv = (n2 > 0 && (double)n2 <= k_cut * k_cut) ? 1.0 : 0.0;
    if (!(wv >= 0.0) || !std::isfinite(wv) || !std::isfinite(S0c[i])) bad = 1;
    if (zero) wv = 0.0;  // k = 0 is never constrained
    double W = wv;
    if (weight_mode == FRESCO_WEIGHT_RELATIVE && S0c[i] != 0.0) W = wv / (S0c[i] * S0c[i]);
    Wc[i] = W;
    if (W != 0.0) ++*ncons;
  }
  return bad;
}

// ---------------------------------------------------------------- stages
// cached: the order of the last binning is kept (optimiser trial steps that stay
// within the slack of the binned positions): no binning pass, the spreading pass
// forms the trial point and the records
template <class R>
int run_bin_spread_rows(fresco_ctx* c, const R* pos, bool cached = false) {
  State<R>* S = (State<R>*)c->state;
  const Geom& g = c->g;
  hipStream_t st = c->st;
  S->cached_eval = cached;
  if (!cached) {
    StageTimer t(c, FRESCO_STAGE_BIN);
    launch_bin(g, S->bp, pos, sizeof(R) == 8, S->bb, st);
  }
  {
    StageTimer t(c, FRESCO_STAGE_SPREAD);
    Strengths<R> cs;
    cs.c = S->str_eval;
    cs.perm = S->bb.perm;
    cs.cmax = S->cmax;
    KeptSpread<R> ks;
    if (cached) {
      const LbfgsVec<R>& v = S->lv;
      ks.x = v.x;
      ks.p = v.p;
      ks.xt = v.xt;
      ks.perm = S->bb.perm;
      ks.rec = (Rec<R>*)S->bb.rec;
      ks.part1 = v.part1;
      ks.nb = v.nb;
      ks.max_step = S->lb_opts.max_step;
      ks.step = &S->lst->step;
      ks.alpha = &S->lst->alpha;
      ks.flag = S->bb.flag;
      ks.drift = &S->lst->drift;
    }
    for (int r = 0; r < t.reps; ++r)
      launch_spread<R>(g, (const Rec<R>*)S->bb.rec, S->bb.start, S->tiles, cs, st,
                       cached ? &ks : nullptr);
  }
  if (!S->fold_fused) {
    StageTimer t(c, FRESCO_STAGE_FOLD);
    FoldTables ft;
    for (int a = 0; a < 3; ++a) {
      ft.off[a] = S->fold_off[a];
      ft.ent[a] = S->fold_ent[a];
    }
    launch_fold<R>(g, S->tiles, S->grid, ft, st);
  }
  RowParams<R> rp = S->rows;
  rp.rin = S->grid;
  rp.cout = S->A1;
  {
    StageTimer t(c, FRESCO_STAGE_FFT_ROWS_FWD);
    HIPCHK(launch_rows<R>(false, rp, S->ax[0], 1, st));
  }
  if (g.d == 3) {
    const long long H0 = g.M[0] + 1, P1 = 2 * g.M[1] + 1;
    ColParams<R> fw = S->col1;
    fw.in_outer = (long long)g.nf[1] * H0;
    fw.in_line = H0;
    fw.out_outer = P1 * H0;
    fw.out_line = H0;
    fw.in[0] = S->A1;
    fw.out[0] = S->A2;
    StageTimer t(c, FRESCO_STAGE_FFT_COLS_FWD);
    HIPCHK(launch_cols<R>(COL_FWD, fw, S->ax[1], 1, st));
  }
  return FRESCO_OK;
}

// 2D last axis with columns too long for LDS: forward half-length sub-transforms
// (not for the backward, which starts from the saved rho), recombination and
// mode stage, inverse half-length sub-transforms (not for S alone) into V1.
template <class R>
int run_long_cols(fresco_ctx* c, int mode, const ColParams<R>& last) {
  State<R>* S = (State<R>*)c->state;
  const Geom& g = c->g;
  const long long H0 = g.M[0] + 1, P = 2LL * g.M[1] + 1;
  if (mode != COL_BWD) {
    ColParams<R> f = S->lfw;
    f.in[0] = S->A1;
    f.out[0] = S->Yl;
    HIPCHK(launch_cols<R>(COL_FWD, f, S->ax[1], 1, c->st));
  }
  HIPCHK(launch_long_modes<R>(mode, last, S->Yl, S->Ql, S->twn, g.nf[1], S->long_blocks, c->st));
  if (mode != COL_SF) {
    ColParams<R> v = S->linv;
    v.in[0] = S->Ql;
    v.in[1] = S->Ql + P * H0;
    v.out[0] = S->V1;
    v.out[1] = S->V1 + H0;
    HIPCHK(launch_cols<R>(COL_INV, v, S->ax[1], 2, c->st));
  }
  return FRESCO_OK;
}

// mode stage + inverse transforms + interpolation; mode = COL_FUSED or COL_BWD
template <class R>
int run_modes_to_grad(fresco_ctx* c, int mode, const R* pos, R* S_cube, const R* g_cube, R* grad,
                      double* loss_dev, LossParts* defer = nullptr) {
  State<R>* S = (State<R>*)c->state;
  const Geom& g = c->g;
  const int d = g.d;
  hipStream_t st = c->st;
  const long long H0 = g.M[0] + 1, P1 = 2 * g.M[1] + 1;
  const long long nf1 = g.nf[1];
  ColParams<R> last = (d == 2) ? S->col1 : S->col2;
  last.in[0] = (d == 2) ? S->A1 : S->A2;
  last.out[0] = (d == 2) ? S->V1 : S->V2;
  last.Wp = S->Wp;
  last.S0p = S->S0p;
  last.Wm = S->Wm;
  last.S0m = S->S0m;
  last.loss_part = S->loss_part;
  last.fsum_part = (mode == COL_FUSED && S->val_eval) ? S->fsum_part : nullptr;
  last.S_cube = S_cube;
  // the backward reads rho saved by the structure-factor pass; a loss
  // evaluation keeps none (it also invalidates the reuse of that pass)
  last.rho_save = (mode == COL_BWD || mode == COL_GFIELD || mode == COL_GBACK) ? S->rho : nullptr;
  last.g_cube = g_cube;
  {
    StageTimer t(c, FRESCO_STAGE_MODES);
    if (d == 2 && S->long_cols) {
      int ls = run_long_cols<R>(c, mode, last);
      if (ls) return ls;
    } else {
      HIPCHK(launch_cols<R>(mode, last, S->ax[d - 1], 1, st));
    }
  }
  if (d == 3) {
    ColParams<R> inv = S->col1;
    inv.in_outer = P1 * H0;
    inv.in_line = H0;
    inv.out_outer = nf1 * H0;
    inv.out_line = H0;
    inv.in[0] = S->V2;
    inv.out[0] = S->V1;
    StageTimer t(c, FRESCO_STAGE_FFT_COLS_INV);
    HIPCHK(launch_cols<R>(COL_INV, inv, S->ax[1], 1, st));
  }
  RowParams<R> rp = S->rows;
  rp.fold.tiles = nullptr;  // forward only
  rp.cin[0] = S->V1;
  rp.rout[0] = S->v;
  {
    StageTimer t(c, FRESCO_STAGE_FFT_ROWS_INV);
    HIPCHK(launch_rows<R>(true, rp, S->ax[0], 1, st));
  }
  if (mode == COL_GFIELD) return FRESCO_OK;  // the pair correlation function is in v
  {
    StageTimer t(c, FRESCO_STAGE_INTERP);
    Strengths<R> cs;
    cs.c = S->str_eval;
    cs.perm = S->bb.perm;
    cs.cmax = S->cmax;
    cs.val = (mode == COL_FUSED) ? S->val_eval : nullptr;
    const Geom gi = interp_geom(g, S->cached_eval);
    for (int r = 0; r < t.reps; ++r) launch_interp<R>(gi, S->bp, S->bb, S->v, grad, cs, st);
  }
  // the pair-correlation backward has no loss partials here, and the point
  // flag was handed over by the structure-factor pass before it
  if (mode == COL_GBACK) return FRESCO_OK;
  // attached soft-core pair term: its gradient is added to grad, its energy to
  // the loss
  const bool pair = (mode == COL_FUSED && c->pair);
  if (pair) {
    int ps = pair_enqueue(c->pair, pos, grad, true, c->pair_w, st);
    if (ps) return ps;
  }
  LossParts lp;
  lp.part = S->loss_part;
  lp.n = mode == COL_FUSED ? S->nloss_part : 0;
  lp.part2 = pair ? c->pair->part : nullptr;
  lp.n2 = pair ? c->pair->nblocks : 0;
  lp.w2 = c->pair_w;
  lp.flag = S->bb.flag;
  lp.flag_out = S->flag_out;
  // defer: the caller's next kernel sums the partials (the optimiser update)
  if (defer) {
    *defer = lp;
    return FRESCO_OK;
  }
  finish_kernel<<<1, 256, 0, st>>>(lp.part, lp.n, lp.part2, lp.n2, lp.w2,
                                   mode == COL_FUSED ? loss_dev : nullptr, lp.flag, lp.flag_out);
  HIPCHK(hipGetLastError());
  return FRESCO_OK;
}

template <class R>
int loss_grad_eager(fresco_ctx* c, const void* pos, double* loss_dev, void* grad) {
  State<R>* S = (State<R>*)c->state;
  S->str_eval = S->has_str ? S->cdev : nullptr;
  S->val_eval = nullptr;
  int st;
  if ((st = run_bin_spread_rows<R>(c, (const R*)pos))) return st;
  return run_modes_to_grad<R>(c, COL_FUSED, (const R*)pos, nullptr, nullptr, (R*)grad, loss_dev);
}

template <class R>
int loss_grad_impl(fresco_ctx* c, const void* pos, double* loss_dev, void* grad) {
  c->sf_pos = nullptr;
  // the legacy default stream cannot be captured; timed stages run eagerly; so
  // do calls made while the caller captures the stream into a graph of its own
  // (the launches then become nodes of that graph)
  if (!c->use_graphs || c->timing_mask || c->st == nullptr)
    return loss_grad_eager<R>(c, pos, loss_dev, grad);
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  HIPCHK(hipStreamIsCapturing(c->st, &cap));
  if (cap != hipStreamCaptureStatusNone) return loss_grad_eager<R>(c, pos, loss_dev, grad);
  for (auto& e : c->graphs)
    if (e.pos == pos && e.loss == loss_dev && e.grad == grad) {
      HIPCHK(hipGraphLaunch(e.exec, c->st));
      return FRESCO_OK;
    }
  hipGraph_t graph = nullptr;
  HIPCHK(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
  int st = loss_grad_eager<R>(c, pos, loss_dev, grad);
  hipError_t e = hipStreamEndCapture(c->st, &graph);
  if (st) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  HIPCHK(e);
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  HIPCHK(e);
  if (c->graphs.size() >= 8) {
    (void)hipGraphExecDestroy(c->graphs.front().exec);
    c->graphs.erase(c->graphs.begin());
  }
  c->graphs.push_back({pos, loss_dev, grad, exec});
  HIPCHK(hipGraphLaunch(exec, c->st));
  return FRESCO_OK;
}

// ------------------------------------------------------------- L-BFGS
// Frees the optimiser's device buffers (any that exist); the stream must have
// drained.
template <class R>
void lbfgs_free(fresco_ctx* c) {
  State<R>* S = (State<R>*)c->state;
  LbfgsVec<R>& v = S->lv;
  dfree(c, v.x);
  dfree(c, v.g);
  dfree(c, v.p);
  dfree(c, v.xt);
  dfree(c, v.gt);
  dfree(c, v.S);
  dfree(c, v.Y);
  dfree(c, v.part0);
  dfree(c, v.part1);
  dfree(c, S->lst);
  dfree(c, S->perm0);
  S->lb_m = 0;
}

template <class R>
int lbfgs_alloc(fresco_ctx* c, int m) {
  State<R>* S = (State<R>*)c->state;
  const long long n = c->g.N * c->g.d;
  LbfgsVec<R>& v = S->lv;
  int st;
  if ((st = dalloc_t(c, &v.x, n))) return st;
  if ((st = dalloc_t(c, &v.g, n))) return st;
  if ((st = dalloc_t(c, &v.p, n))) return st;
  if ((st = dalloc_t(c, &v.xt, n))) return st;
  if ((st = dalloc_t(c, &v.gt, n))) return st;
  const long long ld = lbfgs_slot_stride(n);
  if ((st = dalloc_t(c, &v.S, (size_t)ld * m))) return st;
  if ((st = dalloc_t(c, &v.Y, (size_t)ld * m))) return st;
  const int nb = lbfgs_blocks(n);
  v.nb = nb;
  v.n = n;
  v.ld = ld;
  v.m = m;
  if ((st = dalloc_t(c, &v.part0, (4 * (size_t)kLbfgsMaxM + 1) * nb))) return st;
  if ((st = dalloc_t(c, &v.part1, (size_t)nb))) return st;
  if ((st = dalloc_t(c, &S->lst, 2))) return st;  // the state and pass A's snapshot
  if ((st = dalloc_t(c, &S->perm0, c->g.N))) return st;
  if (!S->lst_host) HIPCHK(hipHostMalloc((void**)&S->lst_host, 2 * sizeof(LbfgsState)));
  for (int i = 0; i < 2; ++i)
    if (!S->lb_ev[i]) HIPCHK(hipEventCreateWithFlags(&S->lb_ev[i], hipEventDisableTiming));
  S->lb_m = m;
  return FRESCO_OK;
}

// Buffers of the optimiser for history length m, allocated on the first call
// and again when m changes: the buffers of the earlier length are freed first
// (after the stream has drained), so that changing m does not accumulate them,
// and so are the ones of an allocation that failed part way.
template <class R>
int lbfgs_setup(fresco_ctx* c, int m) {
  State<R>* S = (State<R>*)c->state;
  if (S->lst && S->lb_m == m) return FRESCO_OK;
  S->drop_lb_graphs();
  S->have_perm0 = false;
  HIPCHK(hipStreamSynchronize(c->st));
  lbfgs_free<R>(c);
  const int st = lbfgs_alloc<R>(c, m);
  if (st) lbfgs_free<R>(c);
  return st;
}

template <class R>
int lbfgs_reset_state(fresco_ctx* c) {
  State<R>* S = (State<R>*)c->state;
  LbfgsState h;
  std::memset(&h, 0, sizeof(h));
  h.head = S->lb_m - 1;
  h.gamma = 1.0;
  HIPCHK(hipMemcpy(S->lst, &h, sizeof(h), hipMemcpyHostToDevice));
  return FRESCO_OK;
}

// one trial step: evaluation at xt, then the optimiser update; cached: this
// evaluation keeps the tile order of the last binning (its spreading pass forms
// the trial point the previous update left out); keep_next: so does the next one,
// and this update leaves out the trial point pass
template <class R>
int lbfgs_trial(fresco_ctx* c, bool cached = false, bool keep_next = false) {
  State<R>* S = (State<R>*)c->state;
  int st;
  // the optimiser's positions are in its internal order, and so are the strengths
  S->str_eval = S->has_str ? S->cint : nullptr;
  S->val_eval = nullptr;
  if ((st = run_bin_spread_rows<R>(c, S->lv.xt, cached))) return st;
  // the update's first pass sums the loss partials into f_trial itself
  LossParts lp;
  if ((st = run_modes_to_grad<R>(c, COL_FUSED, S->lv.xt, nullptr, nullptr, S->lv.gt,
                                 &S->lst->f_trial, &lp)))
    return st;
  launch_lbfgs_update<R>(S->lv, S->lst, S->lb_opts, c->st, keep_next, &lp);
  HIPCHK(hipGetLastError());
  return FRESCO_OK;
}

template <class R>
int lbfgs_read(fresco_ctx* c) {
  State<R>* S = (State<R>*)c->state;
  HIPCHK(hipMemcpyAsync(S->lst_host, S->lst, sizeof(LbfgsState), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  return FRESCO_OK;
}

template <class R>
int step_impl(fresco_ctx* c, void* pos, const fresco_lbfgs_opts* o, int n_iter, double* loss_out,
              int32_t* n_eval_out) {
  State<R>* S = (State<R>*)c->state;
  const Geom& g = c->g;
  int st;
  c->sf_pos = nullptr;
  if ((st = lbfgs_setup<R>(c, o->m))) return st;
  LbfgsOpts lo;
  lo.m = o->m;
  lo.max_backtracks = o->max_backtracks;
  lo.max_step = o->max_step;
  lo.c1 = o->c1;
  lo.shrink = o->shrink;
  lo.gtol = o->gtol;
  if (std::memcmp(&lo, &S->lb_opts, sizeof(lo)) != 0) S->drop_lb_graphs();
  S->lb_opts = lo;
  const long long N = g.N;
  if (!S->have_perm0) {
    // internal order = tile order of the starting positions (stable: ties in
    // the caller's order, so that the order and every dot product over it are
    // the same from run to run); it stays fixed so that the history vectors
    // never need permuting, and later binning passes see nearly sorted points
    launch_bin(g, S->bp, pos, sizeof(R) == 8, S->bb, c->st);
    if (!launch_stable_index(g, S->bp, S->bb, pos, sizeof(R) == 8, S->perm0, c->st))
      launch_sorted_index(g, S->bp, S->bb, S->perm0, c->st);
    if ((st = lbfgs_reset_state<R>(c))) return st;
    S->have_perm0 = true;
  }
  launch_gather_rows<R>((const R*)pos, S->perm0, N, g.d, S->lv.x, c->st);
  if (S->has_str) launch_gather_rows<R>(S->cdev, S->perm0, N, 1, S->cint, c->st);
  HIPCHK(hipMemcpyAsync(S->lv.xt, S->lv.x, sizeof(R) * N * g.d, hipMemcpyDeviceToDevice, c->st));
  launch_lbfgs_set_mode(S->lst, 4, n_iter, c->st);  // first evaluation of the call
  if ((st = lbfgs_trial<R>(c))) return st;
  launch_lbfgs_set_mode(S->lst, 0, -1, c->st);
  const bool graphs = c->use_graphs && !c->timing_mask && c->st != nullptr;
  // Cached tile order inside a chunk: every trial point lies within max_step
  // (per coordinate) of the current point, which moves by at most max_step per
  // accepted step, so trial r after a binned trial 0 is within (r + 2) max_step
  // of it; while that is at most the slack (less a margin for rounding) in grid
  // cells, its footprint starts stay inside the padded tiles of that binning.
  int bin_every = 1;  // trials per binning in a chunk
  if (g.slack > 0 && S->bp.mode == BIN_TILES && lo.max_step > 0.0) {
    double cells = 0.0;  // grid cells per max_step, largest over the axes
    for (int a = 0; a < g.d; ++a) cells = std::max(cells, lo.max_step * g.ufac[a]);
    const double r = std::floor((g.slack - 0.25) / cells) - 2.0;  // last cached trial
    if (r >= 1.0) bin_every = (int)std::min<double>(r + 1.0, kLbfgsMaxReplayChunk);
  }
  // trial steps per chunk: kLbfgsReplayChunk, or one binning's worth when that
  // is more (fewer binnings and graph launches per trial step)
  const int chunk_len = std::max(kLbfgsReplayChunk, bin_every);
  // two graphs: one trial step, and a full chunk of them (one launch per chunk,
  // so that consecutive steps are not separated by a graph launch)
  auto capture = [&](int steps, hipGraphExec_t* out) -> int {
    hipGraph_t graph = nullptr;
    HIPCHK(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
    int s2 = FRESCO_OK;
    for (int r = 0; r < steps && !s2; ++r)
      s2 = lbfgs_trial<R>(c, r % bin_every != 0, r + 1 < steps && (r + 1) % bin_every != 0);
    hipError_t e = hipStreamEndCapture(c->st, &graph);
    if (s2) {
      if (graph) (void)hipGraphDestroy(graph);
      return s2;
    }
    HIPCHK(e);
    e = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    HIPCHK(e);
    return FRESCO_OK;
  };
  if (graphs && !S->lb_graph_chunk) {
    S->drop_lb_graphs();
    if ((st = capture(1, &S->lb_graph)) || (st = capture(chunk_len, &S->lb_graph_chunk))) {
      S->drop_lb_graphs();
      return st;
    }
  }
  auto replay = [&](int count) -> int {
    if (graphs && count == chunk_len) {
      HIPCHK(hipGraphLaunch(S->lb_graph_chunk, c->st));
      return FRESCO_OK;
    }
    for (int r = 0; r < count; ++r) {
      if (graphs) {
        HIPCHK(hipGraphLaunch(S->lb_graph, c->st));
      } else {
        // eager launches follow the graphs' binning pattern (same arithmetic)
        const bool chunk = count == chunk_len;
        const int s2 = lbfgs_trial<R>(c, chunk && r % bin_every != 0,
                                      chunk && r + 1 < count && (r + 1) % bin_every != 0);
        if (s2) return s2;
      }
    }
    return FRESCO_OK;
  };
  if ((st = lbfgs_replay_until_stop(c->st, S->lst, S->lst_host, S->lb_ev, n_iter, chunk_len,
                                    replay, &g_last_hip)))
    return st;
  launch_scatter_rows<R>(S->lv.x, S->perm0, N, g.d, (R*)pos, c->st);
  if ((st = lbfgs_read<R>(c))) return st;
  const LbfgsState& h = *S->lst_host;
  if (loss_out) *loss_out = h.f_cur;
  if (n_eval_out) *n_eval_out = h.nevals;
  // a trial point beyond the slack of its binning (excluded by the step cap)
  if (h.drift) return FRESCO_ENOTSUP;
  if (h.fail) return FRESCO_ELINESEARCH;
  return FRESCO_OK;
}

// S on the mode cube (Sout may be NULL: only rho and the point order are kept)
template <class R>
int structure_factor_impl(fresco_ctx* c, const void* pos, void* Sout) {
  State<R>* S = (State<R>*)c->state;
  const Geom& g = c->g;
  int st;
  c->sf_pos = nullptr;
  S->str_eval = S->has_str ? S->cdev : nullptr;
  S->val_eval = nullptr;
  if ((st = run_bin_spread_rows<R>(c, (const R*)pos))) return st;
  ColParams<R> last = (g.d == 2) ? S->col1 : S->col2;
  last.in[0] = (g.d == 2) ? S->A1 : S->A2;
  last.S_cube = (R*)Sout;
  last.rho_save = S->rho;
  {
    StageTimer t(c, FRESCO_STAGE_MODES);
    if (g.d == 2 && S->long_cols) {
      if ((st = run_long_cols<R>(c, COL_SF, last))) return st;
    } else {
      HIPCHK(launch_cols<R>(COL_SF, last, S->ax[g.d - 1], 1, c->st));
    }
  }
  finish_kernel<<<1, 256, 0, c->st>>>(S->loss_part, 0, nullptr, 0, 0.0, nullptr, S->bb.flag,
                                      S->flag_out);
  HIPCHK(hipGetLastError());
  c->sf_pos = pos;
  return FRESCO_OK;
}

// Backward of S: grad = sum_k gS(k) dS(k)/dr (derivative of S in the Methods'
// gradient derivation), the same type-2 field-derivative pass as the loss
// gradient with dL/dS replaced by the caller's gS.
template <class R>
int sf_backward_impl(fresco_ctx* c, const void* pos, const void* gS, void* grad, int reuse) {
  State<R>* S = (State<R>*)c->state;
  int st;
  if (reuse && c->sf_pos != pos) return FRESCO_EINVAL;
  if (!reuse && (st = structure_factor_impl<R>(c, pos, nullptr))) return st;
  S->str_eval = S->has_str ? S->cdev : nullptr;
  S->val_eval = nullptr;
  return run_modes_to_grad<R>(c, COL_BWD, (const R*)pos, nullptr, (const R*)gS, (R*)grad, nullptr);
}

// ------------------------------------------------- pair correlation loss
// L_g partials over the fine grid (fixed grid-stride order, kGlossBlocks blocks
// of 256): sum W_g (g - g0)^2; b = 2 W_g (g - g0) for the backward; g copied out
// when asked.
template <class R>
__global__ void gloss_kernel(const R* __restrict__ g, const R* __restrict__ g0,
                             const R* __restrict__ wg, long long n, R* __restrict__ b,
                             R* __restrict__ gout, double* __restrict__ part) {
  __shared__ double sh[256];
  double acc = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const R gi = g[i];
    const R r = gi - g0[i];
    const R w = wg[i];
    acc += (double)w * (double)r * (double)r;
    b[i] = R(2) * w * r;
    if (gout) gout[i] = gi;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}
__global__ void sum_parts_kernel(const double* __restrict__ part, int np, double* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double t = 0.0;
  for (int i = 0; i < np; ++i) t += part[i];
  out[0] = t;
}

// L_g and its gradient (Methods, pair correlation function optimisation):
// S and rho (type-1 pass), g on the fine grid from (S - 1)/N (inverse passes),
// L_g and b on the grid, then the forward transform of b whose real part is
// dL_g/dS, fed to the backward of S (inverse passes and interpolation).
template <class R>
int gloss_impl(fresco_ctx* c, const void* pos, double* loss_dev, void* grad, void* g_out) {
  State<R>* S = (State<R>*)c->state;
  const Geom& g = c->g;
  int st;
  if ((st = structure_factor_impl<R>(c, pos, nullptr))) return st;
  c->sf_pos = nullptr;
  S->str_eval = nullptr;
  S->val_eval = nullptr;
  if ((st = run_modes_to_grad<R>(c, COL_GFIELD, (const R*)pos, nullptr, nullptr, nullptr, nullptr)))
    return st;
  gloss_kernel<R><<<kGlossBlocks, 256, 0, c->st>>>(S->v, S->g0, S->wg, g.ngrid, S->gb, (R*)g_out,
                                                  S->gpart);
  sum_parts_kernel<<<1, 64, 0, c->st>>>(S->gpart, kGlossBlocks, loss_dev);
  HIPCHK(hipGetLastError());
  // forward transforms of b (rows from the grid, no fold; 3D: axis 1)
  RowParams<R> rp = S->rows;
  rp.fold.tiles = nullptr;
  rp.rin = S->gb;
  rp.cout = S->A1;
  HIPCHK(launch_rows<R>(false, rp, S->ax[0], 1, c->st));
  if (g.d == 3) {
    const long long H0 = g.M[0] + 1, P1 = 2 * g.M[1] + 1;
    ColParams<R> fw = S->col1;
    fw.in_outer = (long long)g.nf[1] * H0;
    fw.in_line = H0;
    fw.out_outer = P1 * H0;
    fw.out_line = H0;
    fw.in[0] = S->A1;
    fw.out[0] = S->A2;
    HIPCHK(launch_cols<R>(COL_FWD, fw, S->ax[1], 1, c->st));
  }
  return run_modes_to_grad<R>(c, COL_GBACK, (const R*)pos, nullptr, nullptr, (R*)grad, nullptr);
}

template <class R>
int set_gtarget_impl(fresco_ctx* c, const double* g0, const double* wg) {
  State<R>* S = (State<R>*)c->state;
  HIPCHK(hipStreamSynchronize(c->st));
  if (!wg) {
    S->has_g = false;
    return FRESCO_OK;
  }
  const long long n = c->g.ngrid;
  std::vector<double> a(n), b(n);
  for (long long i = 0; i < n; ++i) {
    a[i] = g0 ? g0[i] : 0.0;
    b[i] = wg[i];
    if (!std::isfinite(a[i]) || !(b[i] >= 0.0) || !std::isfinite(b[i])) return FRESCO_EINVAL;
  }
  int st;
  if ((st = upload_into<R>(c, &S->g0, a))) return st;
  if ((st = upload_into<R>(c, &S->wg, b))) return st;
  if (!S->gb) {
    if ((st = dalloc_t(c, &S->gb, n))) return st;
    if ((st = dalloc_t(c, &S->gpart, kGlossBlocks))) return st;
  }
  S->has_g = true;
  return FRESCO_OK;
}

// ------------------------------------------------------------ strengths
// Block partials of sum c^2 (FP64), max |c| and a count of non-finite values,
// in a fixed order (kStatBlocks blocks of 256 threads, grid-stride).
template <class R>
__global__ void strength_stats_kernel(const R* __restrict__ c, long long n,
                                      double* __restrict__ part) {
  __shared__ double s2[256], sm[256], sb[256];
  double a = 0.0, m = 0.0, bad = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double v = (double)c[i];
    if (!isfinite(v)) {
      bad += 1.0;
      continue;
    }
    a += v * v;
    m = fmax(m, fabs(v));
  }
  s2[threadIdx.x] = a;
  sm[threadIdx.x] = m;
  sb[threadIdx.x] = bad;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      s2[threadIdx.x] += s2[threadIdx.x + off];
      sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + off]);
      sb[threadIdx.x] += sb[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x] = s2[0];
    part[gridDim.x + blockIdx.x] = sm[0];
    part[2 * gridDim.x + blockIdx.x] = sb[0];
  }
}
__global__ void strength_stats_final_kernel(double* part, int nb) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double a = 0.0, m = 0.0, bad = 0.0;
  for (int b = 0; b < nb; ++b) {
    a += part[b];
    m = fmax(m, part[nb + b]);
    bad += part[2 * nb + b];
  }
  part[3 * nb] = a;
  part[3 * nb + 1] = m;
  part[3 * nb + 2] = bad;
}

// dL/dc_j = F(r_j) - (4 c_j / rho0) sum_K W S (S - S0) (Methods, Eq.
// lossweightgradient), in place over the field values F(r_j); every block sums
// the mode-stage partials in the same order.
template <class R>
__global__ void strength_grad_kernel(R* __restrict__ gc, const R* __restrict__ c, long long n,
                                     const double* __restrict__ fpart, long long np,
                                     double four_over_rho0) {
  __shared__ double fs;
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (long long i = 0; i < np; ++i) t += fpart[i];
    fs = t * four_over_rho0;
  }
  __syncthreads();
  const R f = (R)fs;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    gc[i] = gc[i] - f * c[i];
}

template <class R>
void set_inv_norm(fresco_ctx* c, double norm) {
  State<R>* S = (State<R>*)c->state;
  const R inv = (R)(1.0 / norm);
  S->col1.invN = inv;
  S->col2.invN = inv;
  S->lfw.invN = inv;
  S->linv.invN = inv;
}

// drop every captured graph (their launch parameters changed)
template <class R>
void drop_graphs(fresco_ctx* c) {
  State<R>* S = (State<R>*)c->state;
  for (auto& e : c->graphs) (void)hipGraphExecDestroy(e.exec);
  c->graphs.clear();
  S->drop_lb_graphs();
}

template <class R>
int set_strengths_impl(fresco_ctx* c, const void* cin) {
  State<R>* S = (State<R>*)c->state;
  const long long N = c->g.N;
  HIPCHK(hipStreamSynchronize(c->st));
  drop_graphs<R>(c);
  c->sf_pos = nullptr;
  if (!cin) {
    S->has_str = false;
    S->rho0 = 0.0;
    S->cmax = 1.0;
    set_inv_norm<R>(c, (double)N);
    return FRESCO_OK;
  }
  int st;
  if (!S->cdev) {
    if ((st = dalloc_t(c, &S->cdev, N))) return st;
    if ((st = dalloc_t(c, &S->cint, N))) return st;
    if ((st = dalloc_t(c, &S->cstat, 3 * kStatBlocks + 3))) return st;
    if ((st = dalloc_t(c, &S->fsum_part, S->nloss_part))) return st;
  }
  HIPCHK(hipMemcpyAsync(S->cdev, cin, sizeof(R) * N, hipMemcpyDeviceToDevice, c->st));
  strength_stats_kernel<R><<<kStatBlocks, 256, 0, c->st>>>(S->cdev, N, S->cstat);
  strength_stats_final_kernel<<<1, 64, 0, c->st>>>(S->cstat, kStatBlocks);
  HIPCHK(hipGetLastError());
  double h[3];
  HIPCHK(hipMemcpyAsync(h, S->cstat + 3 * kStatBlocks, sizeof(h), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  if (h[2] != 0.0 || !(h[0] > 0.0) || !std::isfinite(h[0])) {
    S->has_str = false;
    set_inv_norm<R>(c, (double)N);
    return FRESCO_EINVAL;
  }
  S->has_str = true;
  S->rho0 = h[0];
  S->cmax = h[1];
  set_inv_norm<R>(c, h[0]);
  return FRESCO_OK;
}

// loss, position gradient and strength gradient with the context's strengths
// (eager: the strength gradient is an occasional request)
template <class R>
int loss_grad_strengths_impl(fresco_ctx* c, const void* pos, double* loss, void* grad,
                             void* grad_c) {
  State<R>* S = (State<R>*)c->state;
  if (!S->has_str) return FRESCO_EINVAL;
  c->sf_pos = nullptr;
  S->str_eval = S->cdev;
  S->val_eval = (R*)grad_c;
  int st = run_bin_spread_rows<R>(c, (const R*)pos);
  if (!st) st = run_modes_to_grad<R>(c, COL_FUSED, (const R*)pos, nullptr, nullptr, (R*)grad,
                                     S->loss_dev);
  S->val_eval = nullptr;
  if (st) return st;
  long long blocks = (c->g.N + 255) / 256;
  if (blocks > 4096) blocks = 4096;
  strength_grad_kernel<R><<<(unsigned)blocks, 256, 0, c->st>>>(
      (R*)grad_c, S->cdev, c->g.N, S->fsum_part, S->nloss_part, 4.0 / S->rho0);
  HIPCHK(hipGetLastError());
  HIPCHK(hipMemcpyAsync(c->host_loss, S->loss_dev, sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipMemcpyAsync(c->host_flag, S->flag_out, sizeof(int), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  *loss = *c->host_loss;
  if (*c->host_flag) return FRESCO_ENONFINITE;
  return FRESCO_OK;
}

}  // namespace

// ================================================================== C ABI
extern "C" {

const char* fresco_error_string(int code) {
  switch (code) {
    case FRESCO_OK: return "ok";
    case FRESCO_EINVAL: return "invalid argument";
    case FRESCO_ENOMEM: return "out of memory";
    case FRESCO_EHIP: return "HIP runtime error";
    case FRESCO_ENOTSUP: return "not supported by this library";
    case FRESCO_ENONFINITE: return "non-finite position";
    case FRESCO_ELINESEARCH: return "line search failed";
    default: return "unknown status";
  }
}

int fresco_last_hip_error(void) { return g_last_hip; }

int fresco_destroy(fresco_ctx* c) {
  if (!c) return FRESCO_OK;
  (void)hipStreamSynchronize(c->st);
  for (auto& e : c->graphs) (void)hipGraphExecDestroy(e.exec);
  for (void* p : c->allocs) (void)hipFree(p);
  if (c->host_loss) (void)hipHostFree(c->host_loss);
  if (c->host_flag) (void)hipHostFree(c->host_flag);
  for (int s = 0; s < FRESCO_STAGE_COUNT; ++s)
    for (auto& pr : c->pending[s]) {
      (void)hipEventDestroy(pr.first);
      (void)hipEventDestroy(pr.second);
    }
  for (hipEvent_t e : c->event_pool) (void)hipEventDestroy(e);
  if (c->state) {
    if (c->dtype == FRESCO_F32) {
      State<float>* S = (State<float>*)c->state;
      S->drop_lb_graphs();
      if (S->lst_host) (void)hipHostFree(S->lst_host);
      for (hipEvent_t e : S->lb_ev)
        if (e) (void)hipEventDestroy(e);
      delete S;
    } else {
      State<double>* S = (State<double>*)c->state;
      S->drop_lb_graphs();
      if (S->lst_host) (void)hipHostFree(S->lst_host);
      for (hipEvent_t e : S->lb_ev)
        if (e) (void)hipEventDestroy(e);
      delete S;
    }
  }
  delete c;
  return FRESCO_OK;
}

int fresco_create(fresco_ctx** out, const fresco_problem* p, void* stream) {
  if (!out) return FRESCO_EINVAL;
  *out = nullptr;
  if (!p) return FRESCO_EINVAL;
  const int d = p->dim;
  if (d != 2 && d != 3) return FRESCO_EINVAL;
  if (p->dtype != FRESCO_F32 && p->dtype != FRESCO_F64) return FRESCO_EINVAL;
  if (p->n < 1) return FRESCO_EINVAL;
  if (p->n > 2147483647LL) return FRESCO_ENOTSUP;
  if (!(p->tol > 0.0 && p->tol <= 0.1)) return FRESCO_EINVAL;
  if (p->upsampfac != 2.0) return FRESCO_EINVAL;
  if (p->weight_mode != FRESCO_WEIGHT_ABS && p->weight_mode != FRESCO_WEIGHT_RELATIVE)
    return FRESCO_EINVAL;
  for (int a = 0; a < d; ++a) {
    if (!(p->box[a] > 0.0) || !std::isfinite(p->box[a])) return FRESCO_EINVAL;
    if (p->kmax[a] < 0) return FRESCO_EINVAL;
  }
  if (!p->w && !(p->k_cut >= 0.0)) return FRESCO_EINVAL;

  fresco_ctx* c = new (std::nothrow) fresco_ctx();
  if (!c) return FRESCO_ENOMEM;
  c->dtype = p->dtype;
  c->st = (hipStream_t)stream;
  const char* eg = std::getenv("FRESCO_GRAPHS");
  c->use_graphs = !(eg && eg[0] == '0');
  // optional cap on the device memory of the context (bytes), for callers that
  // share the GPU; allocations beyond it fail with FRESCO_ENOMEM
  const char* ml = std::getenv("FRESCO_DEVICE_MEMORY_LIMIT");
  c->mem_limit = ml ? std::atoll(ml) : 0;
  Geom& g = c->g;
  std::memset(&g, 0, sizeof(g));
  g.d = d;
  g.N = p->n;
  g.w = kernel_width(p->tol);
  g.beta = kernel_beta(g.w);
  g.wi = g.w + 1;
  g.beta_i = kernel_beta(g.wi);
  g.icb = 1.0 / std::cosh(g.beta_i);
  g.nbins = 1;
  g.ngrid = 1;
  g.nhalf = 1;
  g.ncube = 1;
  // spreading tile edge: measured over 32..64 in 2D (40: 1024 tiles on the 1250^2
  // grid, the fastest spread, fold and evaluation) and 12..20 in 3D (FP32)
  int tdef = (d == 2) ? 40 : (p->dtype == FRESCO_F32 ? 16 : 8);
  // FRESCO_TILE overrides the tile edge (4 to 64; checks and tuning)
  if (const char* et = std::getenv("FRESCO_TILE")) tdef = std::max(4, std::min(64, std::atoi(et)));
  for (int a = 0; a < 3; ++a) {
    if (a < d) {
      g.L[a] = p->box[a];
      g.M[a] = p->kmax[a];
      long long need = 2LL * (2LL * g.M[a] + 1);
      if (need < 2LL * g.wi) need = 2LL * g.wi;
      if (need > (1LL << 26)) {
        delete c;
        return FRESCO_ENOTSUP;
      }
      g.nf[a] = next_smooth_even(need);
      g.ufac[a] = (double)g.nf[a] / g.L[a];
      g.gsc[a] = -(double)g.nf[a] / g.L[a] * 2.0 / g.wi;
      g.T[a] = tdef < g.nf[a] ? tdef : g.nf[a];
      g.tdiv[a] = make_fastdiv((uint32_t)g.T[a]);
      g.nt[a] = (g.nf[a] + g.T[a] - 1) / g.T[a];
      g.nbins *= g.nt[a];
      g.ngrid *= g.nf[a];
      g.ncube *= 2LL * g.M[a] + 1;
      g.nhalf *= (a == 0) ? (g.M[a] + 1) : (2LL * g.M[a] + 1);
    } else {
      g.L[a] = 1.0;
      g.M[a] = 0;
      g.nf[a] = 1;
      g.T[a] = 1;
      g.ufac[a] = 1.0;
      g.tdiv[a] = make_fastdiv(1u);
      g.nt[a] = 1;
      g.E[a] = 1;
      g.Ei[a] = 1;
    }
  }
  // Slack of the padded spreading tiles: footprint starts may lie this many
  // cells outside their tile, so that the optimiser's trial steps can keep the
  // tile order of an earlier binning (2D: 2 cells, +18% padded cells at the
  // 40-cell tiles; the interpolation's field tiles cover the slack only in those
  // cached evaluations; 3D: none).  FRESCO_SLACK overrides it
  // in 2D (0 to 8).  Only where the padded tiles stay well inside one grid
  // period and the points are sorted by tile in one level.
  {
    int slack = (d == 2) ? 2 : 0;
    if (const char* es = std::getenv("FRESCO_SLACK"))
      if (d == 2) slack = std::max(0, std::min(8, std::atoi(es)));
    for (int a = 0; a < d; ++a)
      if (g.nf[a] < g.T[a] + 2 * slack + g.wi + 1 || g.nt[a] > 1024) slack = 0;
    // the kept order needs the one-level tile sort (at most 16384 tiles)
    if (g.nbins > 16384 || std::getenv("FRESCO_BIN_RANGES") || std::getenv("FRESCO_BIN_ATOMIC"))
      slack = 0;
    g.slack = slack;
    g.islack = 0;
    for (int a = 0; a < d; ++a) {
      g.E[a] = g.T[a] + 2 * slack + g.w - 1;
      g.Ei[a] = g.T[a] + g.wi;
    }
  }
  // 32-bit index ranges of the passes
  if (g.ngrid > (1LL << 33) || g.nhalf > (1LL << 31) || g.nbins > (1LL << 31)) {
    delete c;
    return FRESCO_ENOTSUP;
  }

  // weights and targets on the full cube (FP64, host)
  std::vector<double> Wc, S0c;
  long long ncons = 0;
  if (build_weights(g, p->s0, p->w, p->k_cut, p->weight_mode, Wc, S0c, &ncons)) {
    delete c;
    return FRESCO_EINVAL;
  }
  c->n_constrained = ncons;

  int st;
  if (p->dtype == FRESCO_F32) {
    st = create_state<float>(c);
    if (!st) st = upload_weights<float>(c, Wc, S0c);
  } else {
    st = create_state<double>(c);
    if (!st) st = upload_weights<double>(c, Wc, S0c);
  }
  if (!st) {
    hipError_t e = hipHostMalloc((void**)&c->host_loss, sizeof(double));
    if (e == hipSuccess) e = hipHostMalloc((void**)&c->host_flag, sizeof(int));
    if (e != hipSuccess) {
      g_last_hip = (int)e;
      st = FRESCO_ENOMEM;
    }
  }
  if (st) {
    fresco_destroy(c);
    return st;
  }
  *out = c;
  return FRESCO_OK;
}

int fresco_plan_info_get(const fresco_ctx* c, fresco_plan_info* o) {
  if (!c || !o) return FRESCO_EINVAL;
  std::memset(o, 0, sizeof(*o));
  o->dim = c->g.d;
  o->dtype = c->dtype;
  o->n = c->g.N;
  for (int a = 0; a < 3; ++a) {
    o->nf[a] = a < c->g.d ? c->g.nf[a] : 0;
    o->kmax[a] = a < c->g.d ? c->g.M[a] : 0;
    o->tile[a] = a < c->g.d ? c->g.T[a] : 0;
  }
  o->width = c->g.w;
  o->beta = c->g.beta;
  o->nbins = c->g.nbins;
  o->n_constrained = c->n_constrained;
  o->device_bytes = c->bytes;
  o->col_split = 1;
  if (c->dtype == FRESCO_F32 && ((const State<float>*)c->state)->long_cols) o->col_split = 2;
  if (c->dtype == FRESCO_F64 && ((const State<double>*)c->state)->long_cols) o->col_split = 2;
  const BinPlan& bp = (c->dtype == FRESCO_F32) ? ((const State<float>*)c->state)->bp
                                               : ((const State<double>*)c->state)->bp;
  o->bin_ranges = bp.mode == BIN_RANGES ? (int32_t)bp.nkeys : bp.mode == BIN_TILES ? 0 : -1;
  o->bin_levels = bp.mode == BIN_RANGES ? bp.levels : 1;
  o->slack = c->g.slack;
  return FRESCO_OK;
}

int fresco_set_timing(fresco_ctx* c, uint32_t mask) {
  if (!c) return FRESCO_EINVAL;
  c->timing_mask = mask & ((1u << FRESCO_STAGE_COUNT) - 1);
  return FRESCO_OK;
}

int fresco_set_timing_reps(fresco_ctx* c, int32_t reps) {
  if (!c || reps < 1 || reps > 1000) return FRESCO_EINVAL;
  c->timing_reps = reps;
  return FRESCO_OK;
}

int fresco_read_timing(fresco_ctx* c, double* ms_total, int64_t* launches, int reset) {
  if (!c) return FRESCO_EINVAL;
  HIPCHK(hipStreamSynchronize(c->st));
  for (int s = 0; s < FRESCO_STAGE_COUNT; ++s) {
    for (size_t i = 0; i < c->pending[s].size(); ++i) {
      auto& pr = c->pending[s][i];
      float ms = 0.f;
      HIPCHK(hipEventElapsedTime(&ms, pr.first, pr.second));
      c->stage_ms[s] += ms;
      c->stage_n[s] += c->pending_reps[s][i];
      c->event_pool.push_back(pr.first);
      c->event_pool.push_back(pr.second);
    }
    c->pending[s].clear();
    c->pending_reps[s].clear();
    if (ms_total) ms_total[s] = c->stage_ms[s];
    if (launches) launches[s] = c->stage_n[s];
    if (reset) {
      c->stage_ms[s] = 0.0;
      c->stage_n[s] = 0;
    }
  }
  return FRESCO_OK;
}

int fresco_structure_factor(fresco_ctx* c, const void* pos, void* S) {
  if (!c || !pos || !S) return FRESCO_EINVAL;
  if (c->dtype == FRESCO_F32) return structure_factor_impl<float>(c, pos, S);
  return structure_factor_impl<double>(c, pos, S);
}

int fresco_structure_factor_backward(fresco_ctx* c, const void* pos, const void* gS,
                                     void* grad, int32_t reuse) {
  if (!c || !pos || !gS || !grad) return FRESCO_EINVAL;
  if (c->dtype == FRESCO_F32) return sf_backward_impl<float>(c, pos, gS, grad, reuse);
  return sf_backward_impl<double>(c, pos, gS, grad, reuse);
}

int fresco_loss_grad_async(fresco_ctx* c, const void* pos, double* loss_dev, void* grad) {
  if (!c || !pos || !loss_dev || !grad) return FRESCO_EINVAL;
  if (c->dtype == FRESCO_F32) return loss_grad_impl<float>(c, pos, loss_dev, grad);
  return loss_grad_impl<double>(c, pos, loss_dev, grad);
}

int fresco_step(fresco_ctx* c, void* pos, const fresco_lbfgs_opts* o, int32_t n_iter,
                double* loss_out, int32_t* n_eval_out) {
  if (!c || !pos || !o || n_iter < 0) return FRESCO_EINVAL;
  if (o->m < 1 || o->m > kLbfgsMaxM || o->max_backtracks < 0) return FRESCO_EINVAL;
  if (!(o->max_step > 0.0) || !(o->c1 > 0.0 && o->c1 < 1.0) ||
      !(o->shrink > 0.0 && o->shrink < 1.0) || !(o->gtol >= 0.0))
    return FRESCO_EINVAL;
  if (c->dtype == FRESCO_F32) return step_impl<float>(c, pos, o, n_iter, loss_out, n_eval_out);
  return step_impl<double>(c, pos, o, n_iter, loss_out, n_eval_out);
}

int fresco_attach_pair(fresco_ctx* c, fresco_pair_ctx* pc, double weight) {
  if (!c) return FRESCO_EINVAL;
  if (pc) {
    if (pc->d != c->g.d || pc->dtype != c->dtype || pc->n != c->g.N) return FRESCO_EINVAL;
    for (int a = 0; a < c->g.d; ++a)
      if (pc->L[a] != c->g.L[a]) return FRESCO_EINVAL;
    if (!(weight > 0.0) || !std::isfinite(weight)) return FRESCO_EINVAL;
  }
  HIPCHK(hipStreamSynchronize(c->st));
  // captured graphs hold the previous launch sequence
  for (auto& e : c->graphs) (void)hipGraphExecDestroy(e.exec);
  c->graphs.clear();
  if (c->dtype == FRESCO_F32) {
    ((State<float>*)c->state)->drop_lb_graphs();
  } else {
    ((State<double>*)c->state)->drop_lb_graphs();
  }
  c->pair = pc;
  c->pair_w = pc ? weight : 0.0;
  return FRESCO_OK;
}

int fresco_set_pair_correlation_target(fresco_ctx* c, const double* g0, const double* wg) {
  if (!c) return FRESCO_EINVAL;
  if (c->dtype == FRESCO_F32) return set_gtarget_impl<float>(c, g0, wg);
  return set_gtarget_impl<double>(c, g0, wg);
}

int fresco_pair_correlation_loss_grad(fresco_ctx* c, const void* pos, double* loss, void* grad,
                                      void* g_out) {
  if (!c || !pos || !loss || !grad) return FRESCO_EINVAL;
  double* ldev;
  int* fout;
  int st;
  if (c->dtype == FRESCO_F32) {
    State<float>* S = (State<float>*)c->state;
    if (!S->has_g) return FRESCO_EINVAL;
    if (S->has_str || S->long_cols) return FRESCO_ENOTSUP;
    ldev = S->loss_dev;
    fout = S->flag_out;
    st = gloss_impl<float>(c, pos, ldev, grad, g_out);
  } else {
    State<double>* S = (State<double>*)c->state;
    if (!S->has_g) return FRESCO_EINVAL;
    if (S->has_str || S->long_cols) return FRESCO_ENOTSUP;
    ldev = S->loss_dev;
    fout = S->flag_out;
    st = gloss_impl<double>(c, pos, ldev, grad, g_out);
  }
  if (st) return st;
  HIPCHK(hipMemcpyAsync(c->host_loss, ldev, sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipMemcpyAsync(c->host_flag, fout, sizeof(int), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  *loss = *c->host_loss;
  if (*c->host_flag) return FRESCO_ENONFINITE;
  return FRESCO_OK;
}

int fresco_set_strengths(fresco_ctx* c, const void* cs) {
  if (!c) return FRESCO_EINVAL;
  // the signed spreading words take 8 bytes per cell of the padded tile
  if (c->dtype == FRESCO_F32) {
    State<float>* S = (State<float>*)c->state;
    if (cs && (S->bp.mode == BIN_RANGES || S->long_cols ||
               spread_lds_bytes<float>(c->g, true) > (size_t)kMaxSpreadLds))
      return FRESCO_ENOTSUP;
    return set_strengths_impl<float>(c, cs);
  }
  State<double>* S = (State<double>*)c->state;
  if (cs && (S->bp.mode == BIN_RANGES || S->long_cols ||
             spread_lds_bytes<double>(c->g, true) > (size_t)kMaxSpreadLds))
    return FRESCO_ENOTSUP;
  return set_strengths_impl<double>(c, cs);
}

int fresco_loss_grad_strengths(fresco_ctx* c, const void* pos, double* loss, void* grad,
                               void* grad_c) {
  if (!c || !pos || !loss || !grad || !grad_c) return FRESCO_EINVAL;
  if (c->dtype == FRESCO_F32) return loss_grad_strengths_impl<float>(c, pos, loss, grad, grad_c);
  return loss_grad_strengths_impl<double>(c, pos, loss, grad, grad_c);
}

int fresco_reset_history(fresco_ctx* c) {
  if (!c) return FRESCO_EINVAL;
  if (c->dtype == FRESCO_F32) ((State<float>*)c->state)->have_perm0 = false;
  else ((State<double>*)c->state)->have_perm0 = false;
  return FRESCO_OK;
}

int fresco_set_target(fresco_ctx* c, const double* s0, const double* w, double k_cut,
                      int32_t weight_mode) {
  if (!c) return FRESCO_EINVAL;
  if (weight_mode != FRESCO_WEIGHT_ABS && weight_mode != FRESCO_WEIGHT_RELATIVE)
    return FRESCO_EINVAL;
  if (!w && !(k_cut >= 0.0)) return FRESCO_EINVAL;
  std::vector<double> Wc, S0c;
  long long ncons = 0;
  if (build_weights(c->g, s0, w, k_cut, weight_mode, Wc, S0c, &ncons)) return FRESCO_EINVAL;
  // the arrays are overwritten in place, so captured graphs stay valid
  HIPCHK(hipStreamSynchronize(c->st));
  int st = (c->dtype == FRESCO_F32) ? upload_weights<float>(c, Wc, S0c)
                                    : upload_weights<double>(c, Wc, S0c);
  if (st) return st;
  c->n_constrained = ncons;
  c->sf_pos = nullptr;
  return fresco_reset_history(c);
}

int fresco_step_sequence(fresco_ctx* c, void* pos, int32_t n_targets, const double* const* s0s,
                         const double* const* ws, double k_cut, int32_t weight_mode,
                         const fresco_lbfgs_opts* o, int32_t n_iter, double* losses,
                         int32_t* n_evals, void* frames) {
  if (!c || !pos || n_targets < 0 || !o) return FRESCO_EINVAL;
  const size_t fbytes = (size_t)c->g.N * c->g.d * (c->dtype == FRESCO_F32 ? 4 : 8);
  for (int t = 0; t < n_targets; ++t) {
    int st = fresco_set_target(c, s0s ? s0s[t] : nullptr, ws ? ws[t] : nullptr, k_cut,
                               weight_mode);
    if (st) return st;
    double loss = 0.0;
    int32_t nev = 0;
    // a frame whose line search fails keeps its last accepted point; the next
    // frame starts from there
    st = fresco_step(c, pos, o, n_iter, &loss, &nev);
    if (st && st != FRESCO_ELINESEARCH) return st;
    if (losses) losses[t] = loss;
    if (n_evals) n_evals[t] = nev;
    if (frames)
      HIPCHK(hipMemcpyAsync((char*)frames + fbytes * (size_t)t, pos, fbytes,
                            hipMemcpyDeviceToDevice, c->st));
  }
  HIPCHK(hipStreamSynchronize(c->st));
  return FRESCO_OK;
}

int fresco_overlap_cycles(fresco_ctx* c, fresco_pair_ctx* pc, void* pos,
                          const fresco_lbfgs_opts* o, int32_t n_iter, int32_t max_cycles,
                          double threshold, const void* fresh, int64_t n_fresh, double* loss_out,
                          int32_t* cycles_out, int64_t* replaced_out) {
  if (!c || !pc || !pos || !o || max_cycles < 0 || (n_fresh > 0 && !fresh) || n_fresh < 0)
    return FRESCO_EINVAL;
  if (pc->n != c->g.N || pc->d != c->g.d || pc->dtype != c->dtype) return FRESCO_EINVAL;
  const size_t rowb = (size_t)c->g.d * (c->dtype == FRESCO_F32 ? 4 : 8);
  int64_t used = 0;
  double loss = 0.0;
  int cyc = 0;
  for (; cyc < max_cycles; ++cyc) {
    int32_t nev = 0;
    int st = fresco_step(c, pos, o, n_iter, &loss, &nev);
    if (st && st != FRESCO_ELINESEARCH) return st;
    // the pair context runs on its own stream: order it after this one
    HIPCHK(hipStreamSynchronize(c->st));
    int64_t rep = 0;
    st = fresco_pair_replace_overlaps(pc, pos, threshold,
                                      fresh ? (const char*)fresh + rowb * (size_t)used : nullptr,
                                      n_fresh - used, &rep);
    if (st) return st;
    used += rep;
    if (rep == 0) {
      ++cyc;
      break;
    }
    fresco_reset_history(c);  // replaced points invalidate the curvature pairs
  }
  if (loss_out) *loss_out = loss;
  if (cycles_out) *cycles_out = cyc;
  if (replaced_out) *replaced_out = used;
  return FRESCO_OK;
}

int fresco_loss_grad(fresco_ctx* c, const void* pos, double* loss, void* grad) {
  if (!c || !pos || !loss || !grad) return FRESCO_EINVAL;
  double* ldev;
  int* fout;
  int st;
  if (c->dtype == FRESCO_F32) {
    State<float>* S = (State<float>*)c->state;
    ldev = S->loss_dev;
    fout = S->flag_out;
    st = loss_grad_impl<float>(c, pos, ldev, grad);
  } else {
    State<double>* S = (State<double>*)c->state;
    ldev = S->loss_dev;
    fout = S->flag_out;
    st = loss_grad_impl<double>(c, pos, ldev, grad);
  }
  if (st) return st;
  HIPCHK(hipMemcpyAsync(c->host_loss, ldev, sizeof(double), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipMemcpyAsync(c->host_flag, fout, sizeof(int), hipMemcpyDeviceToHost, c->st));
  HIPCHK(hipStreamSynchronize(c->st));
  *loss = *c->host_loss;
  if (*c->host_flag) return FRESCO_ENONFINITE;
  return FRESCO_OK;
}

}  // extern "C"
