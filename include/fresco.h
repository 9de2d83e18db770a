/*
 * fresco.h -- C ABI of an MI355X (gfx950) implementation of the FReSCo
 * structure-factor loss and its position gradient.
 *
 * Problem (main text, "Algorithm"; Methods, "Analytical gradients"):
 *   N points r_j in a periodic box [0, L_0) x ... x [0, L_{d-1}), d = 2 or 3,
 *   unit weights c_j = 1;  k = 2 pi n / L for integer mode vectors n;
 *   rho(k)  = sum_j exp(+i k.r_j)                     (Methods, Eq. ft)
 *   S(k)    = |rho(k)|^2 / N                          (Eq. structure_factor)
 *   L_S     = sum_{k in K} W(k) (S(k) - S0(k))^2      (Eqs. SF_loss, loss with W)
 *   dL_S/dr_j = Re sum_k C(k) exp(-i k.r_j),
 *   C(k)    = -4 i k W(k) (S(k) - S0(k)) rho(k) / N   (Eq. gradient)
 * evaluated with nonuniform FFTs (the "NUwU" variant of the Methods), all on
 * the GPU: one type-1 transform gives rho; the d components of the gradient
 * are the derivatives of one type-2 field (coefficients 2 G(k) rho(k) / N with
 * G = dL/dS), interpolated with the derivative of the kernel, which equals the
 * d type-2 transforms of the Methods up to the transform accuracy.
 *
 * Conventions shared by every call:
 *   - Mode cube: the constrained region, targets and weights live on the dense
 *     cube of integer modes |n_a| <= M_a ("kmax"), stored in C order over
 *     (n_0, ..., n_{d-1}), index of n = (n_0 + M_0, ..., n_{d-1} + M_{d-1}).
 *     The region K is the set of modes with nonzero weight; n = 0 is never in K.
 *     The sum over K runs over the full set (both n and -n), as in Eq. SF_loss.
 *   - Positions and gradients: device arrays [n][d] (row-major) of the problem's
 *     dtype (float or double).  Positions may take any finite value; they are
 *     wrapped into the box (exp(i k.r) is L-periodic), which is not an error.
 *   - Streams: a context is bound to one HIP stream (passed as void*, NULL for the
 *     default stream).  Calls enqueue work on that stream and return; the ones
 *     taking a host pointer for the loss synchronise the stream before returning.
 *     A context must not be used from two threads at once.
 *   - Ownership: the context owns all scratch memory; the caller owns every
 *     pointer it passes and keeps device buffers alive until the stream has
 *     consumed them.
 *   - Errors: every call returns 0 (FRESCO_OK) or a negative FRESCO_E* code; no
 *     exception crosses the ABI.  fresco_error_string() describes a code and
 *     fresco_last_hip_error() returns the last hipError_t seen by the library.
 */
#ifndef FRESCO_H
#define FRESCO_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum fresco_dtype { FRESCO_F32 = 0, FRESCO_F64 = 1 };

/* How the caller's weights w become the W of the loss (Methods, "Analytical
 * gradients"): ABS uses W = w; RELATIVE uses W = w / S0^2 where S0 != 0 and
 * W = w where S0 == 0, which is the relative loss of Eq. loss. */
enum fresco_weight_mode { FRESCO_WEIGHT_ABS = 0, FRESCO_WEIGHT_RELATIVE = 1 };

enum fresco_status {
  FRESCO_OK = 0,
  FRESCO_EINVAL = -1,      /* invalid argument (null pointer, bad size or option) */
  FRESCO_ENOMEM = -2,      /* device or host allocation failed */
  FRESCO_EHIP = -3,        /* a HIP runtime call failed (see fresco_last_hip_error) */
  FRESCO_ENOTSUP = -4,     /* valid request outside what the library supports */
  FRESCO_ENONFINITE = -5,  /* a position was NaN or infinite (synchronous calls only) */
  FRESCO_ELINESEARCH = -6  /* line search failed repeatedly (optimizer) */
};

typedef struct fresco_problem {
  int32_t dim;          /* d = 2 or 3 */
  int32_t dtype;        /* FRESCO_F32 or FRESCO_F64: positions, gradient, S, arithmetic */
  int64_t n;            /* number of points N >= 1 */
  double box[3];        /* box sides L_a > 0 (entries beyond dim ignored) */
  int32_t kmax[3];      /* mode cube half-widths M_a >= 0 */
  double k_cut;         /* used only when w == NULL: weight 1 on 0 < |n| <= k_cut */
  const double* s0;     /* host, mode cube of targets S0(n); NULL means S0 = 0 */
  const double* w;      /* host, mode cube of weights w(n) >= 0; NULL: see k_cut */
  int32_t weight_mode;  /* fresco_weight_mode */
  double tol;           /* requested relative accuracy of the nonuniform FFTs, e.g. 1e-6 */
  double upsampfac;     /* fine-grid upsampling factor; 2.0 is the only value supported */
} fresco_problem;

typedef struct fresco_ctx fresco_ctx;

/* Plan geometry chosen by fresco_create (for reporting and tests). */
typedef struct fresco_plan_info {
  int32_t dim;
  int32_t dtype;
  int64_t n;
  int32_t nf[3];        /* fine grid size per dimension (even, 5-smooth) */
  int32_t kmax[3];
  int32_t width;        /* kernel width w (grid cells) */
  double beta;          /* exponential-of-semicircle shape parameter */
  int32_t tile[3];      /* spreading tile per dimension */
  int64_t nbins;        /* number of tiles */
  int64_t n_constrained;/* number of modes with nonzero weight (full set) */
  int64_t device_bytes; /* scratch memory held by the context */
  int32_t col_split;    /* 2D last-axis columns transformed as this many sub-columns
                           (1; 2 when a column is too long for one LDS pass) */
  int32_t bin_ranges;   /* points sorted by tile in one level (0), or in two levels
                           through this many ranges of consecutive tiles (grids with
                           more than 16384 tiles), or -1: global atomic counts */
  int32_t bin_levels;   /* two-level sorts: 2 when a coarse pass over groups of
                           ranges runs first (very many ranges), else 1 */
  int32_t slack;        /* cells by which the padded tiles extend past their tile on
                           each side (2 in 2D, 0 in 3D; FRESCO_SLACK overrides):
                           fresco_step keeps the tile order of a binned trial step
                           for the next ones while the step cap keeps their points
                           within it (0: every trial step is binned) */
} fresco_plan_info;

/* Create a context for one problem.  Chooses the fine grid, kernel width and
 * tiles, allocates every scratch buffer and copies targets and weights (host
 * cubes of (2M_0+1)...(2M_{d-1}+1) doubles) to the device.
 * Errors: EINVAL (null out/p, dim not 2 or 3, n < 1, L <= 0, M < 0, tol not in
 * (0, 0.1], upsampfac != 2, a weight < 0 or non-finite, dtype unknown),
 * ENOTSUP (more than 2^31 - 1 points, or a grid beyond the 32-bit index
 * ranges of the passes), ENOMEM, EHIP.  On error *out is set to NULL.
 * The environment variable FRESCO_DEVICE_MEMORY_LIMIT (bytes), read here, caps
 * the device memory the context may ever hold (scratch, and the optimiser's
 * buffers allocated by fresco_step); an allocation beyond it fails with ENOMEM
 * as if the device were full, and what the failing call had allocated is
 * released. */
int fresco_create(fresco_ctx** out, const fresco_problem* p, void* stream);

/* Release a context (synchronises its stream first).  NULL is accepted. */
int fresco_destroy(fresco_ctx* ctx);

/* Geometry of a context.  EINVAL on null arguments. */
int fresco_plan_info_get(const fresco_ctx* ctx, fresco_plan_info* out);

/* Structure factor S(n) on the whole mode cube (Eq. structure_factor), written to
 * the device array S of (2M_0+1)...(2M_{d-1}+1) elements of the dtype, C order;
 * S(0) = N is included.  pos: device [n][d].  Stream-ordered; returns after
 * enqueueing.  Errors: EINVAL (null pointers), EHIP. */
int fresco_structure_factor(fresco_ctx* ctx, const void* pos, void* S);

/* Backward of fresco_structure_factor, for automatic differentiation of any
 * function F of S (derivative of S with respect to a position, Methods,
 * "Analytical gradients"):
 *   grad_ja = sum_{n in cube} gS(n) dS(n)/dr_ja,
 *   dS(k)/dr_j = (2/N) Re[conj(rho(k)) i k exp(i k.r_j)].
 * gS: device mode cube (same layout and dtype as S) holding dF/dS; since S is
 * even in k only (gS(n) + gS(-n)) / 2 matters, and gS(0) is ignored (S(0) = N).
 * grad: device [n][d], overwritten.  pos: the positions S was computed at.
 * reuse != 0: take rho and the point order left by the latest call on this
 * context, which must have been fresco_structure_factor with this same pos
 * pointer (EINVAL otherwise), and the values at pos must not have changed since
 * (not checkable here: the caller vouches for it).  reuse == 0: recompute them
 * from pos first (one more forward pass).  Stream-ordered; returns after
 * enqueueing.  Errors: EINVAL (null pointers, reuse without a matching forward),
 * EHIP. */
int fresco_structure_factor_backward(fresco_ctx* ctx, const void* pos, const void* gS,
                                     void* grad, int32_t reuse);

/* Loss L_S and gradient dL_S/dr_j (Eq. gradient).  pos: device [n][d];
 * grad: device [n][d], overwritten.  loss: HOST pointer to one double; the call
 * synchronises the stream and then also reports non-finite positions
 * (ENONFINITE; the outputs are then meaningless).  Errors: EINVAL, EHIP,
 * ENONFINITE. */
int fresco_loss_grad(fresco_ctx* ctx, const void* pos, double* loss, void* grad);

/* As fresco_loss_grad, but loss_dev is a DEVICE pointer to one double and the
 * call only enqueues work (no synchronisation, no non-finite report), so it can
 * be captured in a HIP graph.  Outside a capture the library captures the
 * evaluation itself on first use and replays that graph when it sees the same
 * pos, loss_dev and grad pointers again; while the caller is capturing the
 * context's stream, the launches are enqueued as they are and become nodes of
 * the caller's graph.  Errors: EINVAL, EHIP. */
int fresco_loss_grad_async(fresco_ctx* ctx, const void* pos, double* loss_dev, void* grad);

/* Point strengths (Methods, "Analytical gradients": the density field
 * sum_j c_j delta(r - r_j); Results: polydisperse packings weigh each particle
 * by its volume over the mean volume, c_j = V_j / <V>).  With real strengths c_j
 * of any sign:
 *   rho(k) = sum_j c_j exp(+i k.r_j),   rho0 = sum_j c_j^2,   S(k) = |rho(k)|^2 / rho0,
 *   dL/dr_j = c_j Re sum_k C(k) exp(-i k.r_j),  C = -4 i k W (S - S0) rho / rho0,
 *   dL/dc_j = Re sum_k Cc(k) exp(-i k.r_j) - (4 c_j / rho0) sum_K W S (S - S0),
 *             Cc = 4 W (S - S0) rho / rho0                (Eq. lossweightgradient).
 * (The paper's position gradient divides by N; with strengths rho0 is the
 * normalisation of S, and the two agree for unit strengths.)
 * fresco_set_strengths copies c (device [n] of the dtype, the caller's point
 * order) into the context; every later evaluation of the context -- S, the
 * loss and gradient, the backward of S, fresco_step (positions optimised at
 * fixed strengths) -- uses them, and S(0) = (sum c)^2 / rho0.  c = NULL returns
 * to unit strengths.  Synchronises the stream and drops the captured graphs.
 * Errors: EINVAL (null ctx, a non-finite strength, rho0 = 0), ENOTSUP (grids
 * sorted in two levels, more than 16384 tiles, or 2D columns too long for one
 * LDS pass), ENOMEM, EHIP. */
int fresco_set_strengths(fresco_ctx* ctx, const void* c);

/* Loss, position gradient (device [n][d]) and strength gradient grad_c
 * (device [n]) with the context's strengths (fresco_set_strengths first;
 * EINVAL without).  loss: HOST pointer; synchronises and reports non-finite
 * positions (ENONFINITE).  Errors: EINVAL, EHIP, ENONFINITE. */
int fresco_loss_grad_strengths(fresco_ctx* ctx, const void* pos, double* loss, void* grad,
                               void* grad_c);

/* Pair-correlation loss (Methods, pair correlation function optimisation).  In
 * the periodic box the pair correlation function is the truncated Fourier sum
 *   g(x) = (1/N) sum_{n in cube} (S(n) - 1) exp(-i k.x)      (n = 0 included),
 * evaluated here on the fine grid x_l = (l_a L_a / nf_a) (nf from
 * fresco_plan_info_get), and
 *   L_g = sum_x W_g(x) (g(x) - g0(x))^2,
 *   dL_g/dr_j = sum_n gS(n) dS(n)/dr_j,  gS(n) = (1/N) sum_x 2 W_g (g - g0) cos(k.x),
 * i.e. the backward of S with dF/dS = gS; both sums over x are transforms on the
 * fine grid.  g0, wg: HOST arrays of prod nf doubles in the fine grid's layout
 * (C order over (l_{d-1}, ..., l_0): axis 0 fastest); g0 NULL means 0; wg >= 0,
 * NULL disables the term.  The context keeps copies.  Synchronises.
 * Errors: EINVAL (null ctx, a negative or non-finite weight, a non-finite
 * target), ENOMEM, EHIP. */
int fresco_set_pair_correlation_target(fresco_ctx* ctx, const double* g0, const double* wg);

/* L_g and dL_g/dr at pos (device [n][d]); grad (device [n][d]) is overwritten;
 * g_out (device, prod nf values of the dtype, fine-grid layout; may be NULL)
 * receives g.  loss: HOST pointer; synchronises and reports non-finite
 * positions (ENONFINITE).  Unit strengths only.  Errors: EINVAL (null pointers,
 * no target set), ENOTSUP (strengths set, or 2D columns too long for one LDS
 * pass), EHIP, ENONFINITE. */
int fresco_pair_correlation_loss_grad(fresco_ctx* ctx, const void* pos, double* loss, void* grad,
                                      void* g_out);

/* Options of the L-BFGS minimiser (main text, "Algorithm": L-BFGS with a cap on
 * the step and a backtracking line search; the constants are this library's).  Defaults used by the Python layer: m = 8,
 * max_backtracks = 20, max_step = 0.1 L / N^(1/d), c1 = 1e-4, shrink = 0.5,
 * gtol = 0. */
typedef struct fresco_lbfgs_opts {
  int32_t m;              /* history pairs, 1..16 */
  int32_t max_backtracks; /* rejections before the history is dropped (>= 0) */
  double max_step;        /* largest displacement of one coordinate in one step (> 0) */
  double c1;              /* Armijo sufficient-decrease constant, in (0, 1) */
  double shrink;          /* backtracking factor, in (0, 1) */
  double gtol;            /* stop when the RMS gradient falls to or below (0: never) */
} fresco_lbfgs_opts;

/* Minimise L_S over the positions with L-BFGS for n_iter accepted iterations
 * (fewer if the RMS gradient reaches gtol).  pos: device [n][d], updated IN
 * PLACE (the only mutated argument).  The history of (s, y) pairs and the
 * internal point order persist in the context across calls, so a run can be
 * continued by calling again with the returned positions; fresco_reset_history
 * starts afresh.  The trial steps run as replays of captured HIP graphs (on a
 * non-default stream: one graph of a chunk of trial steps, one of a single
 * step for the rest), enqueued in chunks with two chunks in flight: the host
 * reads the optimiser's state after each chunk while the next one runs, so
 * after a stop (n_iter reached, gtol reached, line-search failure) at most two
 * chunks of replays run idle -- they change nothing and are not counted.
 * Within a chunk, a trial step may keep the tile order of the previous binned
 * one (only its per-point records are recomputed) while r + 2 step caps, r the
 * steps since that binning, stay below the plan's slack (fresco_plan_info.slack,
 * in grid cells): every trial point is within max_step per coordinate of the
 * current point, which moves by at most max_step per accepted step, so its
 * footprint stays inside the padded tiles of that binning.  A chunk holds 8
 * trial steps, or as many as one binning can serve when that is more (at most
 * 16).
 * loss_out (host, may be NULL): loss at the final positions; n_eval_out (host,
 * may be NULL): loss/gradient evaluations the optimiser used (the first one at
 * the starting point included).  Synchronises the stream.  The first call, and
 * a call with another m, allocates the optimiser's buffers ((5 + 2m) N d values;
 * those of another m are freed).
 * Errors: EINVAL (null ctx/pos/opts, n_iter < 0, options out of range), EHIP,
 * ENOMEM, ELINESEARCH (no decrease even along the steepest descent direction;
 * pos holds the last accepted point), ENOTSUP (a trial point left the slack of
 * its kept tile order, which the step cap excludes; the result is not to be
 * used). */
int fresco_step(fresco_ctx* ctx, void* pos, const fresco_lbfgs_opts* opts, int32_t n_iter,
                double* loss_out, int32_t* n_eval_out);

/* Drop the L-BFGS history and internal point order kept by the context. */
int fresco_reset_history(fresco_ctx* ctx);

/* Replace the target and weights of a context without planning it again (same
 * meaning and layout as s0, w, k_cut and weight_mode of fresco_problem; the
 * geometry, kmax and tolerance stay).  For sequences of targets minimised one
 * after the other from the previous result (SI, a movie encoded frame by frame
 * into successive structure factors).  Synchronises the stream; resets the
 * L-BFGS history; captured graphs stay valid (the arrays are overwritten in
 * place).  Errors: EINVAL (as for fresco_create's weights), EHIP. */
int fresco_set_target(fresco_ctx* ctx, const double* s0, const double* w, double k_cut,
                      int32_t weight_mode);

/* Warm-started sequence (SI, movie encoding): for t = 0 .. n_targets-1, set the
 * target s0s[t] and weights ws[t] (host mode cubes as in fresco_set_target; a
 * NULL array, or a NULL entry, means S0 = 0, or the k_cut rule, for those
 * frames; one weight_mode for all) and run fresco_step from the current
 * positions for n_iter iterations.  pos (device [n][d]) is updated in place and ends at the
 * last frame; losses[t], n_evals[t] (host, may be NULL) receive each frame's
 * final loss and evaluations; frames (device [n_targets][n][d] of the dtype,
 * may be NULL) receives each frame's positions.  A frame whose line search fails
 * keeps its last accepted point and the sequence goes on.  Synchronises.
 * Errors: EINVAL, ENOMEM, EHIP. */
int fresco_step_sequence(fresco_ctx* ctx, void* pos, int32_t n_targets, const double* const* s0s,
                         const double* const* ws, double k_cut, int32_t weight_mode,
                         const fresco_lbfgs_opts* opts, int32_t n_iter, double* losses,
                         int32_t* n_evals, void* frames);

/* ---------------------------------------------------------------------------
 * Soft-core pair repulsion (Results, stealthy hyperuniform packings: a short-
 * range repulsion combined with the spectral loss keeps particles apart):
 *   U(r) = (eps / alpha) (1 - r / sigma)^alpha for r < sigma, else 0,
 *   E = sum over pairs i < j of U(|r_i - r_j|), minimum image convention,
 *   dE/dr_i = -(eps / sigma) sum_j (1 - r_ij / sigma)^(alpha - 1) (r_i - r_j) / r_ij.
 * alpha = 2 is the harmonic soft core, alpha = 2.5 the Hertzian one.  Evaluated
 * on a cell list in O(N); the energy is accumulated in FP64 and the result does
 * not depend on the order of the points' arrival (deterministic). */
typedef struct fresco_pair_problem {
  int32_t dim;     /* 2 or 3 */
  int32_t dtype;   /* FRESCO_F32 or FRESCO_F64 (positions and gradient) */
  int64_t n;       /* number of points >= 1 */
  double box[3];   /* box sides; sigma < L_a / 2 is required */
  double sigma;    /* contact diameter > 0 */
  double eps;      /* energy scale > 0 */
  double alpha;    /* exponent >= 1 */
} fresco_pair_problem;

typedef struct fresco_pair_ctx fresco_pair_ctx;

/* Create a pair context (cell list of side >= sigma, at most 2^24 cells; larger
 * boxes get larger cells).  Errors: EINVAL (null pointers, dim, n < 1, sigma,
 * eps or alpha out of range, a side <= 2 sigma), ENOTSUP (n >= 2^31), ENOMEM. */
int fresco_pair_create(fresco_pair_ctx** out, const fresco_pair_problem* p, void* stream);

/* Release a pair context (synchronises its stream).  NULL is accepted.  A pair
 * context attached to a loss context must outlive the attachment. */
int fresco_pair_destroy(fresco_pair_ctx* pair);

/* E and dE/dr at pos (device [n][d]); grad (device [n][d]) is overwritten.
 * energy: HOST pointer; the call synchronises and reports non-finite positions
 * (ENONFINITE).  Errors: EINVAL, EHIP, ENONFINITE. */
int fresco_pair_energy_grad(fresco_pair_ctx* pair, const void* pos, double* energy, void* grad);

/* As fresco_pair_energy_grad with a DEVICE energy pointer; only enqueues. */
int fresco_pair_energy_grad_async(fresco_pair_ctx* pair, const void* pos, double* energy_dev,
                                  void* grad);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * evaluation as fresco_pair_energy_grad_async for the problem p, without a pair
 * context.  The cell list lives in a fixed 32 MiB device array inside the
 * library (one per GPU, held until the process ends); the call allocates
 * nothing and only enqueues work on stream (NULL: the legacy default stream),
 * which must belong to the current device.  pos, grad: device [n][d] of p's
 * dtype (grad overwritten); energy_dev: DEVICE pointer to one double.  Size
 * limit: the cell list needs about n (8 + 16) + 8 ncell bytes in FP32 and
 * n (8 + 32) + 8 ncell in FP64 (ncell = cells of side >= sigma), which must fit
 * in 32 MiB -- for example 3e5 points at unit density in 3D with sigma = 0.5;
 * larger problems fail with ENOTSUP before any work is enqueued (use a pair
 * context).  Every call on one GPU uses that GPU's array and overwrites what the
 * previous call left there, so calls whose work overlaps on one GPU (other
 * streams, other threads) race; calls in one stream are ordered.  No non-finite
 * report.  Errors: EINVAL (null pointers, problem as for fresco_pair_create, a
 * stream of another device), ENOTSUP (beyond the size limit), EHIP. */
int fresco_pair_energy_grad_noalloc(const fresco_pair_problem* p, const void* pos,
                                    double* energy_dev, void* grad, void* stream);

/* Overlap removal (main text, quasicrystalline structures: between minimisation
 * cycles, points that sit on top of others are removed and redrawn uniformly in
 * the box, keeping N).  A point is an overlap when a point of LOWER index lies
 * closer than threshold to it (minimum image); every overlapping point is
 * replaced, in increasing index order, by the next row of fresh (device
 * [n_fresh][d] of the dtype, positions the caller drew, e.g. uniform in the
 * box).  threshold in (0, sigma] of the pair context (its cell list finds the
 * candidates).  pos (device [n][d]) is updated in place; *n_replaced receives
 * the number of overlapping points.  Runs on the pair context's stream and
 * synchronises it.  Errors: EINVAL (null pointers, threshold out of range, more
 * overlaps than fresh rows: then pos is untouched and *n_replaced holds the
 * number needed), EHIP. */
int fresco_pair_replace_overlaps(fresco_pair_ctx* pair, void* pos, double threshold,
                                 const void* fresh, int64_t n_fresh, int64_t* n_replaced);

/* Cycles of minimisation and overlap removal (main text, quasicrystalline
 * structures): up to max_cycles times, fresco_step(ctx, pos, opts, n_iter)
 * followed by fresco_pair_replace_overlaps(pair, pos, threshold, ...) with the
 * unused rows of fresh; stops after the first cycle that finds no overlap.  The
 * pair context (matching ctx in n, dim and dtype) only supplies the cell list
 * here; it need not be attached.  loss_out: loss at the end of the last
 * minimisation; cycles_out: cycles run; replaced_out: points replaced in total
 * (all may be NULL).  The L-BFGS history is reset after every replacement.
 * Errors: as fresco_step (a failed line search ends that cycle's minimisation
 * only) and fresco_pair_replace_overlaps. */
int fresco_overlap_cycles(fresco_ctx* ctx, fresco_pair_ctx* pair, void* pos,
                          const fresco_lbfgs_opts* opts, int32_t n_iter, int32_t max_cycles,
                          double threshold, const void* fresh, int64_t n_fresh, double* loss_out,
                          int32_t* cycles_out, int64_t* replaced_out);

/* Add weight * E to every loss evaluation of ctx (fresco_loss_grad,
 * fresco_loss_grad_async and fresco_step then minimise L_S + weight E); the pair
 * work runs on ctx's stream.  pair = NULL detaches.  The pair context must match
 * ctx in dim, dtype, n and box.  Synchronises ctx's stream and drops its captured
 * graphs.  Errors: EINVAL (mismatch, weight <= 0 or non-finite), EHIP. */
int fresco_attach_pair(fresco_ctx* ctx, fresco_pair_ctx* pair, double weight);

/* ---------------------------------------------------------------------------
 * Ragged batches: many independent problems of the kind above (each with its
 * own n, box, targets and weights; all with the same dim, dtype, kmax and tol)
 * evaluated together, every configuration's whole fine grid held in LDS.  One
 * evaluation of the batch is three launches, captured with the optimiser
 * kernels in one HIP graph: spreading over work items of at most `chunk` points
 * (into per-item partial grids), one workgroup per configuration for the sum of
 * its partial grids, the FFT, the modes and the inverse FFT (all in LDS), and
 * interpolation over the work items.  (A single launch with one workgroup per
 * configuration measured 8.8 times slower on 256 configurations of 1e3 to 1e5
 * points: the largest configurations ran on one CU each.)  The grid must fit: roughly
 * (16 or 24 bytes) x prod nf_a <= 156 KiB, e.g. kmax <= 19 in 2D for FP32 and
 * FP64.  Positions and gradients are the configurations' [n_b][d] rows
 * concatenated in order (row offsets from fresco_batch_offsets). */
typedef struct fresco_batch_ctx fresco_batch_ctx;

/* Create a batch of nb >= 1 problems ps[0..nb).  Errors: EINVAL (as for
 * fresco_create, or problems that differ in dim, dtype, kmax, tol or
 * upsampfac), ENOTSUP (grid does not fit in LDS, more than 2^31 - 1 points in
 * total), ENOMEM, EHIP. */
int fresco_batch_create(fresco_batch_ctx** out, int32_t nb, const fresco_problem* ps,
                        void* stream);

/* Release a batch context (synchronises its stream).  NULL is accepted. */
int fresco_batch_destroy(fresco_batch_ctx* batch);

/* offsets[0..nb]: first row of every configuration; offsets[nb] = total rows. */
int fresco_batch_offsets(const fresco_batch_ctx* batch, int64_t* offsets);

/* Loss of every configuration and the concatenated gradient.  losses: HOST array
 * of nb doubles (may be NULL); synchronises, reports non-finite positions
 * (ENONFINITE).  grad: device, overwritten. */
int fresco_batch_loss_grad(fresco_batch_ctx* batch, const void* pos, double* losses, void* grad);

/* As fresco_batch_loss_grad with a DEVICE losses array (may be NULL); only
 * enqueues (graph-capturable). */
int fresco_batch_loss_grad_async(fresco_batch_ctx* batch, const void* pos, double* losses_dev,
                                 void* grad);

/* L-BFGS on the sum of the configurations' losses (the configurations are
 * independent, so its gradient is the concatenation of theirs) for n_iter
 * accepted iterations; one trial step = the batch evaluation's three launches
 * plus the optimiser kernels, replayed from one captured HIP graph.  pos is updated in place; the
 * history persists across calls (fresco_batch_reset_history clears it).
 * loss_out: total loss at the final positions.  Errors as fresco_step. */
int fresco_batch_step(fresco_batch_ctx* batch, void* pos, const fresco_lbfgs_opts* opts,
                      int32_t n_iter, double* loss_out, int32_t* n_eval_out);

/* Drop the batch's L-BFGS history. */
int fresco_batch_reset_history(fresco_batch_ctx* batch);

/* Autotuner: time `reps` evaluations at pos (grad: scratch [rows][d]) for every
 * pair of work-item size (points per spreading / interpolation item; the
 * spreading tile of a batch is the configuration's whole grid, so the item is
 * the shape left to choose) and workgroup size (256, 512, 1024 threads), and
 * keep the fastest pair for all later calls; *threads_out (may be NULL)
 * receives the workgroup size.  Synchronises.  Errors: EINVAL, EHIP. */
int fresco_batch_autotune(fresco_batch_ctx* batch, const void* pos, void* grad, int32_t reps,
                          int32_t* threads_out);

/* Last hipError_t seen by the batch functions (0 if none). */
int fresco_batch_last_hip_error(void);

/* ---------------------------------------------------------------------------
 * Structure factor at arbitrary wave vectors, free boundary conditions (the
 * NUwNU variant of the Methods: constraints at any continuous q, such as Bragg
 * peaks of rotational symmetries no lattice has; the Ewald construction of the
 * main text):
 *   rho(q_k) = sum_j c_j exp(+i q_k . r_j)   (positions as given, not wrapped),
 *   S_k = |rho(q_k)|^2 / rho0,  rho0 = sum_j c_j^2 (N for unit strengths),
 *   L = sum_k W_k (S_k - S0_k)^2,
 *   dL/dr_j = c_j sum_k (4 W_k (S_k - S0_k) / rho0) q_k Re[i conj(rho_k) exp(i q_k . r_j)].
 * Evaluated by direct sums on the GPU, O(N K) (exact; suited to constraint sets
 * of tens to thousands of wave vectors), phases in FP64, sums in FP64. */
typedef struct fresco_q_ctx fresco_q_ctx;

/* Context for n points in dim (2, 3) dimensions of the dtype and at most max_q
 * wave vectors at a time, bound to a stream.  Errors: EINVAL, ENOTSUP (n >= 2^31,
 * max_q > 2^26), ENOMEM. */
int fresco_q_create(fresco_q_ctx** out, int32_t dim, int32_t dtype, int64_t n, int64_t max_q,
                    void* stream);
int fresco_q_destroy(fresco_q_ctx* ctx);

/* The wave vectors q (HOST [K][dim] doubles, K <= max_q), weights W (NULL: 1)
 * and targets S0 (NULL: 0) of the loss.  Synchronises.  Errors: EINVAL (K out of
 * range, non-finite values, a negative weight), EHIP. */
int fresco_q_set(fresco_q_ctx* ctx, int64_t K, const double* q, const double* W, const double* S0);

/* S at the wave vectors set (DEVICE S [K] doubles) and optionally rho (DEVICE
 * [K][2] doubles, may be NULL).  pos: device [n][dim]; c: device [n] strengths
 * of the dtype or NULL (unit).  Enqueues only.  Errors: EINVAL, EHIP. */
int fresco_q_structure_factor(fresco_q_ctx* ctx, const void* pos, const void* c, double* S,
                              double* rho);

/* Loss over the wave vectors set and its position gradient (grad: device
 * [n][dim], overwritten).  loss: HOST pointer; synchronises.  Errors: EINVAL,
 * EHIP. */
int fresco_q_loss_grad(fresco_q_ctx* ctx, const void* pos, const void* c, double* loss,
                       void* grad);

/* Loss over the wave vectors set and its gradient with respect to the strengths
 * c (device [n] of the dtype, required), for optimising the weights of fixed
 * points -- e.g. the pixels of a uniform grid constrained at non-uniform k, the
 * UwNU variant of the Methods (Eq. lossweightgradient):
 *   dL/dc_j = Re sum_k Cc_k exp(-i q_k . r_j) - (4 c_j / rho0) sum_k W_k S_k (S_k - S0_k),
 *   Cc_k = 4 W_k (S_k - S0_k) rho_k / rho0.
 * grad_c: device [n], overwritten.  loss: HOST pointer; synchronises.
 * Errors: EINVAL, EHIP. */
int fresco_q_loss_grad_strengths(fresco_q_ctx* ctx, const void* pos, const void* c, double* loss,
                                 void* grad_c);

/* Forward-scattered transmission of the Ewald construction (main text, Eq.
 * ewald; SI, single scattering): for each incident wave vector k_i e_j (k: HOST
 * [n_k] magnitudes > 0; dirs: HOST [n_dir][dim] unit directions),
 *   T = sum_{forward s} S(k (e_s - e_j)) / sum_{all s} S(k (e_s - e_j)),
 * over the scattered directions e_s of a quadrature: in 2D the ns - 1 directions
 * at angles 2 pi m / ns from e_j, m = 1 .. ns - 1 (the incident direction, where
 * S(0) = N, left out); in 3D the ns-point Fibonacci lattice z_m = 1 - (2m+1)/ns,
 * phi_m = m pi (3 - sqrt 5) in the frame whose z axis is e_j (x axis: a x e_j
 * normalised, a = e_z, or e_x when |e_j . e_z| > 0.9).  Forward: e_s . e_j > 0
 * strictly, decided on integers (2D: 4m < ns or 4m > 3ns; 3D: 2m + 1 < ns).
 * The paper cuts the pattern to a disk (ball) first, which is the caller's
 * choice of points.  T: HOST [n_k][n_dir].  Uses the context's wave-vector
 * buffer (ns - 1 or ns <= max_q), dropping the set of fresco_q_set.
 * Synchronises.  Errors: EINVAL, ENOTSUP (quadrature larger than max_q), ENOMEM,
 * EHIP. */
int fresco_ewald_transmission(fresco_q_ctx* ctx, const void* pos, const void* c, int32_t n_k,
                              const double* k, int32_t n_dir, const double* dirs, int32_t ns,
                              double* T);

/* Last hipError_t seen by a wave-vector context (0 if none). */
int fresco_q_last_hip_error(const fresco_q_ctx* ctx);

/* Stages of one evaluation, for fresco_set_timing / fresco_read_timing. */
enum fresco_stage {
  FRESCO_STAGE_BIN = 0,          /* wrap, split, counting sort by tile (4 kernels) */
  FRESCO_STAGE_SPREAD = 1,       /* points -> padded tile sums (type-1 spreading) */
  FRESCO_STAGE_FOLD = 2,         /* padded tiles -> periodic fine grid */
  FRESCO_STAGE_FFT_ROWS_FWD = 3, /* real rows -> half spectrum along axis 0 */
  FRESCO_STAGE_FFT_COLS_FWD = 4, /* forward columns before the last axis (3D) */
  FRESCO_STAGE_MODES = 5,        /* last forward axis + S, loss, coefficients + first inverse */
  FRESCO_STAGE_FFT_COLS_INV = 6, /* inverse columns after the first (3D) */
  FRESCO_STAGE_FFT_ROWS_INV = 7, /* half spectrum -> real field along axis 0 */
  FRESCO_STAGE_INTERP = 8,       /* field -> gradient at the points (type-2 interpolation) */
  FRESCO_STAGE_COUNT = 9
};

/* Diagnostics: bracket the launches of the stages whose bit (1 << stage) is set
 * in stage_mask with HIP events on the context's stream (0 turns timing off).
 * Errors: EINVAL. */
int fresco_set_timing(fresco_ctx* ctx, uint32_t stage_mask);

/* Diagnostics: with timing on, the spreading and interpolation stages launch
 * their kernels `reps` times back to back between their events (those kernels
 * read only their inputs and write all of their outputs, so the results are
 * unchanged), which brings the timed duration per launch close to the kernel's
 * own by spreading the launch overhead of the brackets.  Default 1.
 * Errors: EINVAL (reps outside 1..1000). */
int fresco_set_timing_reps(fresco_ctx* ctx, int32_t reps);

/* Synchronise the stream, add the durations of all bracketed launches since the
 * last read to the running totals and return them: ms_total[s] is the summed
 * duration in milliseconds and launches[s] the number of timed launches of
 * stage s (evaluations times the stage's repetitions; arrays of
 * FRESCO_STAGE_COUNT entries; either may be NULL).  reset != 0 clears the
 * totals after copying.  Errors: EINVAL, EHIP. */
int fresco_read_timing(fresco_ctx* ctx, double* ms_total, int64_t* launches, int reset);

/* Describe a status code (static string). */
const char* fresco_error_string(int code);

/* Last hipError_t value the library observed (0 if none). */
int fresco_last_hip_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FRESCO_H */
