// Internal declarations shared by the HIP translation units of the FReSCo
// library: complex arithmetic, fast integer division, the plan geometry, the
// per-point record produced by binning, and the launchers each unit exports.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "fresco.h"

namespace fresco {

// ---------------------------------------------------------------- complex
template <class R>
struct cpx {
  R x, y;
};
template <class R>
__host__ __device__ __forceinline__ cpx<R> cadd(cpx<R> a, cpx<R> b) { return {a.x + b.x, a.y + b.y}; }
template <class R>
__host__ __device__ __forceinline__ cpx<R> csub(cpx<R> a, cpx<R> b) { return {a.x - b.x, a.y - b.y}; }
template <class R>
__host__ __device__ __forceinline__ cpx<R> cmul(cpx<R> a, cpx<R> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
template <class R>
__host__ __device__ __forceinline__ cpx<R> cmulc(cpx<R> a, cpx<R> b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
template <class R>
__host__ __device__ __forceinline__ cpx<R> cconj(cpx<R> a) { return {a.x, -a.y}; }
template <class R>
__host__ __device__ __forceinline__ cpx<R> cscale(cpx<R> a, R s) { return {a.x * s, a.y * s}; }
// multiply by +i or -i
template <class R>
__host__ __device__ __forceinline__ cpx<R> cmul_i(cpx<R> a) { return {-a.y, a.x}; }
template <class R>
__host__ __device__ __forceinline__ cpx<R> cmul_mi(cpx<R> a) { return {a.y, -a.x}; }

// ------------------------------------------------------- fast 32-bit divide
// q = n / d for 0 <= n < 2^31 by multiply-high (Granlund & Montgomery 1994).
struct FastDiv {
  uint32_t d, m, s;
};
inline FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  uint32_t s = 0;
  while ((1ull << s) < d) ++s;
  f.s = s;
  f.m = (uint32_t)(((1ull << 32) * ((1ull << s) - d)) / d + 1);
  return f;
}
__device__ __forceinline__ uint32_t fdiv(uint32_t n, const FastDiv& f) {
  return (__umulhi(n, f.m) + n) >> f.s;
}

// ------------------------------------------------------------ FFT factors
constexpr int kMaxFactors = 20;
struct FftFactors {
  int n;                      // transform length
  int nfac;                   // number of radix stages
  int radix[kMaxFactors];     // radix of each stage (2, 3, 4 or 5)
  FastDiv ns[kMaxFactors];    // Ns before each stage (product of earlier radices)
  uint32_t twstep[kMaxFactors];  // n / (Ns * radix)
};

// ------------------------------------------------------------------ plan
struct Geom {
  int d;
  long long N;
  double L[3];
  int M[3];       // mode half-widths
  int nf[3];      // fine grid per dimension (nf[a] = 1 beyond d)
  int w;          // spreading kernel width
  double beta;    // ES shape parameter of the spreading kernel
  int wi;         // interpolation kernel width (w + 1)
  double beta_i;  // ES shape parameter of the interpolation kernel
  double icb;     // 1 / cosh(beta_i) (interpolation kernel normalisation)
  double gsc[3];  // -2 nf / (L wi): grid-to-position derivative scale of the
                  // interpolation (0 beyond d); per-plan constants, so that no
                  // thread computes them in FP64
  int T[3];       // tile size per dimension (1 beyond d)
  int nt[3];      // tiles per dimension (1 beyond d)
  int slack;      // cells a footprint start may lie outside its tile (cached
                  // tile order of the optimiser's trial steps; 0: none)
  int islack;     // of those, the cells the interpolation's field tiles cover
                  // on each side (slack for cached evaluations, else 0)
  int E[3];       // padded spreading tile extent T + 2 slack + w - 1 (1 beyond d)
  int Ei[3];      // interpolation field tile extent T + 2 islack + wi (1 beyond d)
  double ufac[3];   // nf / L: position -> grid coordinate
  FastDiv tdiv[3];  // division by T
  long long nbins;
  long long ngrid;  // prod nf
  long long nhalf;  // (M0+1) * prod_{a>0} (2M_a+1): half mode cube
  long long ncube;  // prod (2M_a+1): full mode cube
};

// Sorted per-point record: position of the point inside its kernel footprint and
// the local cell.
//   t[a]  = tau_a = l0_a - u_a + w/2 in [0, 1), u_a = grid coordinate of the point,
//           l0_a = ceil(u_a - w/2) = first grid index of its footprint;
//   cell  = local index of l0 inside its tile plus the slack (the padded tile
//           starts slack cells before the tile), 8 bits per dimension.
template <class R>
struct alignas(4 * sizeof(R)) Rec {
  R t[3];
  uint32_t cell;
};

// Record of a point kept in tile `tile` (cached tile order of the optimiser's
// trial steps): tau and the footprint start as the binning computes them, the
// start taken relative to that tile (periodically, within one grid period of
// it) and stored with the slack offset.  *bad: a coordinate is not finite;
// *off: a finite footprint start lies beyond the slack (clamped).
// tile coordinates, 10 bits per axis (a slack needs nt <= 1024)
__host__ __device__ inline uint32_t kept_tile_pack(const uint32_t* t) {
  return t[0] | (t[1] << 10) | (t[2] << 20);
}
template <class R, int D>
__device__ __forceinline__ Rec<R> kept_tile_record(const Geom& g, const R* x, uint32_t tile,
                                                    bool* bad, bool* off) {
  Rec<R> o;
  o.t[0] = o.t[1] = o.t[2] = R(0);
  o.cell = 0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    const uint32_t ta = (tile >> (10 * a)) & 1023u;
    const double nf = (double)g.nf[a];
    double u = (double)x[a] * g.ufac[a];
    if (!isfinite(u)) {
      *bad = true;
      u = 0.0;
    }
    if (!(u >= 0.0 && u < nf)) {
      u = fmod(u, nf);
      if (u < 0.0) u += nf;
      if (u >= nf) u = 0.0;
    }
    const double l0 = ceil(u - 0.5 * g.w);
    o.t[a] = (R)(l0 - u + 0.5 * g.w);
    int li = (int)l0;
    if (li < 0) li += g.nf[a];
    if (li >= g.nf[a]) li -= g.nf[a];
    int rel = li - (int)ta * g.T[a];
    if (rel < -g.slack) rel += g.nf[a];
    if (rel >= g.T[a] + g.slack) rel -= g.nf[a];
    if (rel < -g.slack || rel >= g.T[a] + g.slack) {
      *off = true;
      rel = rel < -g.slack ? -g.slack : g.T[a] + g.slack - 1;
    }
    o.cell |= (uint32_t)(rel + g.slack) << (8 * a);
  }
  return o;
}

// Fixed-point exponent for `cnt` contributions of at most 1 each:
// (cnt + 1) 2^ex <= 2^bits, ex = bits - ceil(log2(cnt + 1)), in integer
// arithmetic (the FP64 logarithm it replaces cost every thread of a block about
// a hundred instructions for the same value; equal for every cnt below 2^49)
__device__ __forceinline__ int fixed_exponent(long long cnt, int bits) {
  const unsigned long long v = (unsigned long long)cnt + 1ull;  // >= 1
  const int up = (v <= 1ull) ? 0 : 64 - __clzll((long long)(v - 1ull));
  return bits - up;
}

// sum of n partials in a fixed order by the first 256 threads of a block of 256
// or more (s: 256 doubles); every thread gets the sum
__device__ __forceinline__ double block_sum_256(const double* __restrict__ part, long long n,
                                                double* s) {
  if (threadIdx.x < 256) {
    double v = 0.0;
    for (long long i = threadIdx.x; i < n; i += 256) v += part[i];
    s[threadIdx.x] = v;
  }
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  const double r = s[0];
  __syncthreads();
  return r;
}

// The loss of an evaluation as its block partials (and those of an attached
// pair term, weight w2), summed by whoever finishes the evaluation: the loss is
// sum(part) + w2 sum(part2) (just sum(part) when n2 = 0), the non-finite flag is
// handed to flag_out and cleared.
struct LossParts {
  const double* part;
  long long n;
  const double* part2;
  long long n2;
  double w2;
  int* flag;
  int* flag_out;
};

// Trial steps of the optimiser that keep the tile order of the last binning:
// the spreading pass forms the trial point xt = x + alpha p of each of its
// slots (alpha: the decision's step length, or min(1, max_step / max |p|) from
// the direction pass's block maxima for a new direction, stored by block 0) and
// writes the point records in the kept order for itself and the interpolation.
template <class R>
struct KeptSpread {
  const R* x;
  const R* p;
  R* xt;
  const int* perm;         // slot -> point (the last binning)
  Rec<R>* rec;             // records, written
  const double* part1;     // block maxima of |p|
  int nb;
  double max_step;
  const int* step;         // the decision (LB_*)
  double* alpha;           // step length: read, or written for a new direction
  int* flag;               // a coordinate is not finite
  int* drift;              // a point beyond the slack
};

// FP32 kernels evaluate the spreading and interpolation kernels as per-cell
// polynomials of this degree in x = 2 tau - 1 (see plan.h, kernel_poly).
constexpr int kPolyDeg = 9;

// Counting sort of the points by tile.
//   BIN_TILES   block-private LDS histograms over the tiles (tiles <= 16384);
//   BIN_RANGES  two levels for larger grids: block-private histograms over
//               ranges of G consecutive tiles (at most 8192 ranges) place the
//               points by range (positions copied to tpos), then one
//               workgroup per range sorts its points by tile
//               in LDS.  perm then maps a sorted record to its tpos index;
//               interpolation writes through it into tpos and a gather pass
//               restores the caller's order;
//               With two levels (very many ranges), a first pass places the
//               points by coarse range (runs of consecutive ranges) the same
//               way, so that every chunk of the range pass meets few keys;
//   BIN_ATOMIC  global atomic counts per tile (grids beyond both).
enum BinMode { BIN_TILES = 0, BIN_RANGES = 1, BIN_ATOMIC = 2 };
// one histogram-and-scatter pass over keys tile / G
struct BinLevel {
  int nblk;         // blocks of the histogram pass
  long long chunk;  // points per histogram block (multiple of 256)
  long long nkeys;  // histogram keys
  long long G;      // tiles per key
  FastDiv kdiv;     // division by G
  int shift;        // kr = key | rank << shift
};
struct BinPlan {
  int mode;         // BinMode
  int nblk;         // blocks of the histogram pass
  long long chunk;  // points per histogram block (multiple of 256)
  long long nkeys;  // histogram keys: tiles (BIN_TILES) or ranges (BIN_RANGES)
  int G;            // tiles per range (BIN_RANGES), 1 otherwise
  FastDiv kdiv;     // division by G
  int shift;        // kr = key | rank << shift
  int levels;       // BIN_RANGES: 1, or 2 with the coarse pass `coarse` first
  BinLevel coarse;
};
struct BinBuffers {
  uint32_t* kr = nullptr;     // histogram passes: key | rank << shift; atomic: rank
  uint32_t* key = nullptr;    // atomic: tile per point
  uint32_t* H = nullptr;      // [key][block] counts, then offsets
  uint32_t* count = nullptr;  // points per key
  long long* start = nullptr; // tile starts (nbins + 1)
  long long* kstart = nullptr;  // BIN_RANGES: range starts (nkeys + 1)
  void* tpos = nullptr;       // BIN_RANGES: positions in range order [N][d]
  int* tidx = nullptr;        // BIN_RANGES: range order -> caller index (built
                              // only when an L-BFGS call fixes its internal order)
  // BIN_RANGES with two levels: the coarse pass (positions in coarse order,
  // reused for the gradient in coarse order)
  uint32_t* kr0 = nullptr;
  uint32_t* H0 = nullptr;
  uint32_t* count0 = nullptr;
  long long* kstart0 = nullptr;
  void* tpos0 = nullptr;
  int* tidx0 = nullptr;
  void* rec = nullptr;        // Rec<R>[N], sorted
  int* perm = nullptr;        // sorted position -> caller index (tpos index for BIN_RANGES)
  int* flag = nullptr;        // bit 0: a position is not finite
};

// For each axis, the padded spreading tiles that cover every grid coordinate:
// entries ent[a][off[a][y] .. off[a][y+1]) = (tile index, local index).
struct FoldTables {
  const int* off[3];
  const int2* ent[3];
};

// Point strengths of an evaluation (Methods, "Analytical gradients": the density
// sum_j c_j delta(r - r_j)); c == NULL means unit strengths.
//   c     strengths in the caller's order of the evaluation's positions
//   perm  sorted record -> caller index (the binning's permutation)
//   cmax  max |c| (fixed-point range of the spreading)
//   val   if not NULL: the field's value at each point (caller's order), for
//         the gradient with respect to the strengths
template <class R>
struct Strengths {
  const R* c = nullptr;
  const int* perm = nullptr;
  double cmax = 1.0;
  R* val = nullptr;
};
// Largest dynamic LDS of a spreading workgroup (bytes).
constexpr int kMaxSpreadLds = 160 * 1024;

// Launchers exported by the translation units (all enqueue on `st`).
void launch_bin(const Geom& g, const BinPlan& bp, const void* pos, bool f64, BinBuffers& b,
                hipStream_t st);

template <class R>
size_t spread_lds_bytes(const Geom& g, bool str);
template <class R>
size_t interp_lds_bytes(const Geom& g);
// the geometry an interpolation launch uses: field tiles covering the slack for
// a cached evaluation, the tiles alone otherwise
inline Geom interp_geom(const Geom& g, bool cached) {
  Geom h = g;
  h.islack = cached ? g.slack : 0;
  for (int a = 0; a < g.d; ++a) h.Ei[a] = g.T[a] + 2 * h.islack + g.wi;
  return h;
}
template <class R>
hipError_t spread_prepare(const Geom& g);
template <class R>
void launch_spread(const Geom& g, const Rec<R>* rec, const long long* start, R* tiles,
                   const Strengths<R>& cs, hipStream_t st,
                   const KeptSpread<R>* kept = nullptr);
template <class R>
void launch_fold(const Geom& g, const R* tiles, R* grid, const FoldTables& ft, hipStream_t st);
// interpolation of the field v at the binned points into grad (caller's order)
template <class R>
void launch_interp(const Geom& g, const BinPlan& bp, const BinBuffers& b, const R* v, R* grad,
                   const Strengths<R>& cs, hipStream_t st);
// out[j] = caller index of sorted record j
void launch_sorted_index(const Geom& g, const BinPlan& bp, const BinBuffers& b, int* out,
                         hipStream_t st);
// out[j] = caller index of slot j of a stable sort by the first-level key, after
// launch_bin (histogram passes) at the same positions; false for plans without
// first-level histograms of the caller's points (atomic sort, coarse pass) and
// when the kernel's LDS limit cannot be raised
bool launch_stable_index(const Geom& g, const BinPlan& bp, const BinBuffers& b, const void* pos,
                         bool f64, int* out, hipStream_t st);
template <class R>
void launch_fill(R* p, long long n, R v, hipStream_t st);
void launch_fill_u32(uint32_t* p, long long n, uint32_t v, hipStream_t st);

// FFT passes (see fft.hip)
struct FftTables;  // device twiddles and factors per axis
// GFIELD: (S - 1) g_scale from the saved rho as input of the inverse transform
// (the pair correlation function on the fine grid); GBACK: forward transform of
// a real grid b, then the backward of S with dF/dS = Re B g_scale.
enum ColMode {
  COL_FWD = 0,
  COL_INV = 1,
  COL_FUSED = 2,
  COL_SF = 3,
  COL_BWD = 4,
  COL_GFIELD = 5,
  COL_GBACK = 6
};

}  // namespace fresco
