// Point binning, spreading (type-1, first step) and interpolation (type-2,
// last step) for gfx950.
//
// Kernel: the exponential of semicircle  phi(z) = exp(beta (sqrt(1 - z^2) - 1))
// on |z| <= 1 (the kernel of the FINUFFT library used in the paper's Methods),
// scaled so that its support spans w grid cells: psi(x - l h) = phi((l - u) 2 / w)
// with u = x / h the coordinate in grid units.
//
// Binning.  Every point is mapped, in FP64, to u_a = r_a nf_a / L_a wrapped into
// [0, nf_a), the first index of its footprint l0_a = ceil(u_a - w/2) and the
// offset t_a = l0_a - u_a in [-w/2, -w/2 + 1) (kept in the working precision, so
// that large grids lose no phase accuracy).  Points are counting-sorted by the
// tile holding l0 with block-private LDS histograms (no global atomics):
//   hist     each block counts its chunk of points per tile in LDS; the LDS
//            atomic's return value is the point's rank inside (tile, block);
//   rowscan  per tile, exclusive scan over the blocks -> offset of each block;
//   scan     exclusive scan over tiles -> tile starts;
//   scatter  sorted record written at start[tile] + offset[tile][block] + rank.
// Grids with more tiles than an LDS histogram holds sort in two levels: the same
// four passes over ranges of G consecutive tiles move each point's position into
// its range's segment (runs of consecutive destinations, so the writes combine in
// the caches), then one workgroup per range counts its segment per tile in LDS,
// scans, and writes the sorted records (every write lands inside the segment).
// Interpolation then writes the gradient into the segment order and a gather
// pass, which recomputes each point's segment slot from the first level's
// histogram offsets, restores the caller's order with coalesced stores; a
// single-level sort would instead scatter every point's record and gradient to a
// random address over the whole array.
//
// Spreading.  One workgroup per tile accumulates its points into an LDS copy of
// the tile padded by w - 1 cells, in fixed point with integer LDS atomics
// (gfx950 executes integer LDS atomics far faster than float ones; the integer
// sum is exact and independent of order).  The scale is a power of two chosen
// per tile from a bound on the points that cover one cell (a box sum of the
// tile's footprint-start counts), so that no cell can exceed 2^31 while the
// rounding of each contribution stays far below the FP32 precision; two adjacent
// 32-bit cells therefore add as one 64-bit word without carries between them,
// which halves the atomic count.  The padded tile is stored as is; a fold
// kernel then sums, for every grid cell, the padded tiles that cover it
// (deterministic, no float atomics).
//
// Interpolation.  The gradient is the derivative of one interpolated field:
// dL/dr_a = d/dr_a Re sum_k C0(k) exp(-i k.r) with C0 = 2 G rho / N, evaluated
// with the derivative of the interpolation kernel,
//   d psi / d r_a = phi_c'(z_a) (-2/w_i) (nf_a / L_a) prod_{b != a} phi_c(z_b),
// at width w_i = w + 1 (one more cell keeps the derivative interpolation as
// accurate as the plain one) with the cosh form phi_c of the kernel (finite
// derivative at the support edge).  One workgroup per tile stages its padded
// field tile in LDS.
#include <cmath>
#include <cstring>
#include <type_traits>
#include <utility>

#include "common.h"
#include "kernels.h"
#include "lbfgs.h"

namespace fresco {

// ------------------------------------------------------------------ fill
template <class T>
__global__ void fill_kernel(T* p, long long n, T v) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  long long st = (long long)gridDim.x * blockDim.x;
  for (; i < n; i += st) p[i] = v;
}
template <class R>
void launch_fill(R* p, long long n, R v, hipStream_t st) {
  if (n <= 0) return;
  long long blocks = (n + 255) / 256;
  if (blocks > 8192) blocks = 8192;
  fill_kernel<R><<<(unsigned)blocks, 256, 0, st>>>(p, n, v);
}
void launch_fill_u32(uint32_t* p, long long n, uint32_t v, hipStream_t st) {
  launch_fill<uint32_t>(p, n, v, st);
}
template void launch_fill<float>(float*, long long, float, hipStream_t);
template void launch_fill<double>(double*, long long, double, hipStream_t);

// ------------------------------------------------------------- binning
struct PointBin {
  uint32_t bin;
  uint32_t cell;
  double t[3];
};

template <class R, int D>
__device__ __forceinline__ PointBin bin_point_d(const Geom& g, const R* r, bool* bad) {
  PointBin pb;
  pb.cell = 0;
  uint32_t tile[3] = {0, 0, 0};
  for (int a = 0; a < 3; ++a) pb.t[a] = 0.0;
#pragma unroll
  for (int a = 0; a < D; ++a) {
    double x = (double)r[a];
    const double nf = (double)g.nf[a];
    double u = x * g.ufac[a];
    if (!isfinite(u)) {
      *bad = true;
      u = 0.0;
    }
    if (!(u >= 0.0 && u < nf)) {  // outside the box: exact periodic reduction
      u = fmod(u, nf);
      if (u < 0.0) u += nf;
      if (u >= nf) u = 0.0;
    }
    double l0 = ceil(u - 0.5 * g.w);
    pb.t[a] = l0 - u + 0.5 * g.w;  // tau in [0, 1)
    int li = (int)l0;
    if (li < 0) li += g.nf[a];
    if (li >= g.nf[a]) li -= g.nf[a];
    uint32_t ta = fdiv((uint32_t)li, g.tdiv[a]);
    uint32_t loc = (uint32_t)li - ta * (uint32_t)g.T[a] + (uint32_t)g.slack;
    tile[a] = ta;
    pb.cell |= loc << (8 * a);
  }
  pb.bin = tile[0] + (uint32_t)g.nt[0] * (tile[1] + (uint32_t)g.nt[1] * tile[2]);
  return pb;
}
// g.d is uniform: both branches keep every index a compile-time constant
template <class R>
__device__ __forceinline__ PointBin bin_point(const Geom& g, const R* r, bool* bad) {
  return g.d == 2 ? bin_point_d<R, 2>(g, r, bad) : bin_point_d<R, 3>(g, r, bad);
}

// Block-private histogram over the keys tile / G (G = 1: the tiles).
// kr[i] = key | rank << shift (key < 2^shift, rank < 2^(32 - shift));
// H[key * nblk + block] = points of the block with that key.
template <class R>
__global__ void bin_hist_kernel(Geom g, const R* __restrict__ pos, long long chunk, int nblk,
                                int nkeys, FastDiv kdiv, int shift, uint32_t* __restrict__ kr,
                                uint32_t* __restrict__ H, int* __restrict__ flag) {
  extern __shared__ uint32_t hist[];
  // consecutive chunks on one XCD (chunk x per + l for workgroup 8 l + x), so
  // that the histogram entries of neighbouring chunks (one line of H holds 32)
  // are written through one L2; grid 8 ceil(nblk / 8)
  const int per = (nblk + 7) / 8;
  const int blk = (int)(blockIdx.x & 7u) * per + (int)(blockIdx.x >> 3);
  if (blk >= nblk) return;  // whole workgroup, before any barrier
  for (int i = threadIdx.x; i < nkeys; i += blockDim.x) hist[i] = 0;
  __syncthreads();
  const long long i0 = (long long)blk * chunk;
  long long i1 = i0 + chunk;
  if (i1 > g.N) i1 = g.N;
  bool bad = false;
  // four points per thread loaded before any is binned (the loop is otherwise
  // one dependent load at a time)
  const long long step = 4LL * blockDim.x;
  for (long long ib = i0 + threadIdx.x; ib < i1; ib += step) {
    R x[4][3];
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long long i = ib + (long long)u * blockDim.x;
#pragma unroll
      for (int a = 0; a < 3; ++a) x[u][a] = (i < i1 && a < g.d) ? pos[i * g.d + a] : R(0);
    }
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const long long i = ib + (long long)u * blockDim.x;
      if (i < i1) {
        PointBin pb = bin_point<R>(g, x[u], &bad);
        const uint32_t key = fdiv(pb.bin, kdiv);
        uint32_t r = atomicAdd(&hist[key], 1u);
        kr[i] = key | (r << shift);
      }
    }
  }
  if (bad) atomicOr(flag, 1);
  __syncthreads();
  for (int b = threadIdx.x; b < nkeys; b += blockDim.x)
    H[(long long)b * nblk + blk] = hist[b];
}

// Per tile: exclusive scan of H[tile][0..nblk) in place; count[tile] = total.
// One wavefront per tile.
__global__ void bin_rowscan_kernel(uint32_t* __restrict__ H, int nblk, long long nbins,
                                   uint32_t* __restrict__ count) {
  const long long tile = (long long)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6);
  if (tile >= nbins) return;
  const int lane = threadIdx.x & 63;
  uint32_t* row = H + tile * nblk;
  uint32_t carry = 0;
  for (int base = 0; base < nblk; base += 64) {
    const int i = base + lane;
    const uint32_t v = (i < nblk) ? row[i] : 0u;
    uint32_t x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      uint32_t y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (i < nblk) row[i] = carry + x - v;
    carry += __shfl(x, 63, 64);
  }
  if (lane == 0) count[tile] = carry;
}

// Workgroups are dispatched to the 8 XCDs round-robin by index.  The range
// passes give all 256-point blocks of one histogram chunk to one XCD (chunks
// x, x + 8, ... to XCD x, each in order), so that the runs of consecutive slots a
// chunk fills in every segment are written (or read) through one L2 and combine
// there into whole lines.  Grid: 8 ceil(nblk / 8) bpc workgroups; returns the
// point block of workgroup w and its chunk.
__device__ __forceinline__ long long xcd_point_block(uint32_t w, uint32_t bpc, uint32_t* chunk) {
  const uint32_t x = w & 7u, l = w >> 3;
  const uint32_t gc = l / bpc, k = l - gc * bpc;
  *chunk = gc * 8u + x;
  return (long long)(*chunk) * bpc + k;
}
inline unsigned xcd_grid(int nblk, long long chunk) {
  return (unsigned)(8ll * ((nblk + 7) / 8) * (chunk / 256));
}

// 256 threads per block; chunk is a multiple of 256, bpc = chunk / 256 blocks per
// histogram chunk, all on one XCD (xcd_point_block; grid xcd_grid(nblk, chunk))
template <class R>
__global__ void bin_scatter_kernel(Geom g, const R* __restrict__ pos, uint32_t bpc, int nblk,
                                   const uint32_t* __restrict__ kr,
                                   const uint32_t* __restrict__ H,
                                   const long long* __restrict__ start, Rec<R>* __restrict__ rec,
                                   int* __restrict__ perm) {
  uint32_t blk;
  const long long q = xcd_point_block(blockIdx.x, bpc, &blk);
  const long long i = q * 256 + threadIdx.x;
  if (blk >= (uint32_t)nblk || i >= g.N) return;
  bool bad = false;
  PointBin pb = bin_point<R>(g, pos + i * g.d, &bad);
  const uint32_t v = kr[i];
  const uint32_t tile = v & 0xffffu, rank = v >> 16;
  const long long dst = start[tile] + H[(long long)tile * nblk + blk] + rank;
  Rec<R> o;
  o.t[0] = (R)pb.t[0];
  o.t[1] = (R)pb.t[1];
  o.t[2] = (R)pb.t[2];
  o.cell = pb.cell;
  rec[dst] = o;
  perm[dst] = (int)i;
}

// Slot of point i in the range order (first level of BIN_RANGES); 256-thread
// blocks, bpc blocks per histogram chunk.
__device__ __forceinline__ long long range_slot(uint32_t v, int shift, uint32_t blk, int nblk,
                                                const uint32_t* __restrict__ H,
                                                const long long* __restrict__ kstart) {
  const uint32_t key = v & ((1u << shift) - 1u), rank = v >> shift;
  return kstart[key] + H[(long long)key * nblk + blk] + rank;
}


// Range pass: copy each point's position into its range's segment (one store
// per point: the writes are bound by their count, not their bytes).
template <class R>
__global__ void range_scatter_kernel(long long N, int d, const R* __restrict__ pos, uint32_t bpc,
                                     int nblk, int shift, const uint32_t* __restrict__ kr,
                                     const uint32_t* __restrict__ H,
                                     const long long* __restrict__ kstart, R* __restrict__ tpos) {
  uint32_t c;
  const long long q = xcd_point_block(blockIdx.x, bpc, &c);
  const long long i = q * 256 + threadIdx.x;
  if (c >= (uint32_t)nblk || i >= N) return;
  const long long dst = range_slot(kr[i], shift, c, nblk, H, kstart);
  if (d == 2) {
    using V2 = typename std::conditional<sizeof(R) == 4, float2, double2>::type;
    V2 v;
    v.x = pos[2 * i];
    v.y = pos[2 * i + 1];
    reinterpret_cast<V2*>(tpos)[dst] = v;
  } else {
    for (int a = 0; a < d; ++a) tpos[dst * d + a] = pos[i * d + a];
  }
}

// tidx[slot of i] = sidx[i] (or i): range order -> caller index, built when an
// L-BFGS call fixes its internal order
__global__ void range_index_kernel(long long N, uint32_t bpc, int nblk, int shift,
                                   const uint32_t* __restrict__ kr,
                                   const uint32_t* __restrict__ H,
                                   const long long* __restrict__ kstart,
                                   const int* __restrict__ sidx, int* __restrict__ tidx) {
  uint32_t c;
  const long long q = xcd_point_block(blockIdx.x, bpc, &c);
  const long long i = q * 256 + threadIdx.x;
  if (c >= (uint32_t)nblk || i >= N) return;
  tidx[range_slot(kr[i], shift, c, nblk, H, kstart)] = sidx ? sidx[i] : (int)i;
}

// Second level: one workgroup per range of G tiles sorts its segment
// tpos[kstart[s] .. kstart[s+1]) by tile.  LDS: cnt[G] counts, then the running
// write offsets.  Writes start[] of the range's tiles (and start[nbins]).  Each
// thread loads kRangeU positions before it bins them (several loads in flight
// per wave; the passes are otherwise latency-bound).
constexpr int kRangeU = 4;
template <class R, int D>
__device__ __forceinline__ int range_load(const R* __restrict__ tpos, long long j0, long long b,
                                          R (&x)[kRangeU][D]) {
  int n = 0;
#pragma unroll
  for (int u = 0; u < kRangeU; ++u) {
    const long long j = j0 + (long long)u * blockDim.x;
    if (j < b) {
      if constexpr (D == 2) {
        using V2 = typename std::conditional<sizeof(R) == 4, float2, double2>::type;
        const V2 v = reinterpret_cast<const V2*>(tpos)[j];
        x[u][0] = v.x;
        x[u][1] = v.y;
      } else {
#pragma unroll
        for (int a = 0; a < D; ++a) x[u][a] = tpos[j * D + a];
      }
      n = u + 1;
    }
  }
  return n;
}
template <class R, int D>
__global__ void range_sort_kernel(Geom g, int G, const R* __restrict__ tpos,
                                  const long long* __restrict__ kstart,
                                  long long* __restrict__ start, Rec<R>* __restrict__ rec,
                                  int* __restrict__ perm, int* __restrict__ flag) {
  extern __shared__ uint32_t cnt[];
  __shared__ uint32_t wsum[16];
  const long long t0 = (long long)blockIdx.x * G;
  const int nt = (int)((t0 + G <= g.nbins) ? G : g.nbins - t0);
  const long long a = kstart[blockIdx.x], b = kstart[blockIdx.x + 1];
  for (int i = threadIdx.x; i < G; i += blockDim.x) cnt[i] = 0;
  __syncthreads();
  bool bad = false, stray = false;
  const long long step = (long long)kRangeU * blockDim.x;
  for (long long j0 = a + threadIdx.x; j0 < b; j0 += step) {
    R x[kRangeU][D];
    const int n = range_load<R, D>(tpos, j0, b, x);
#pragma unroll
    for (int u = 0; u < kRangeU; ++u) {
      if (u < n) {
        PointBin pb = bin_point_d<R, D>(g, x[u], &bad);
        uint32_t loc = pb.bin - (uint32_t)t0;
        if (loc >= (uint32_t)nt) {  // the first level put it here from the same bits
          stray = true;
          loc = nt - 1;
        }
        atomicAdd(&cnt[loc], 1u);
      }
    }
  }
  __syncthreads();
  // exclusive scan of cnt[0..nt): contiguous chunks per thread, then the thread
  // sums across the block
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6, nw = blockDim.x >> 6;
  const int per = (nt + (int)blockDim.x - 1) / (int)blockDim.x;
  const int c0 = min((int)threadIdx.x * per, nt), c1 = min(c0 + per, nt);
  uint32_t sum = 0;
  for (int c = c0; c < c1; ++c) sum += cnt[c];
  uint32_t x = sum;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wsum[wv] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int k = 0; k < nw; ++k) {
      const uint32_t t = wsum[k];
      wsum[k] = run;
      run += t;
    }
  }
  __syncthreads();
  uint32_t base = wsum[wv] + x - sum;
  for (int c = c0; c < c1; ++c) {
    const uint32_t t = cnt[c];
    cnt[c] = base;
    start[t0 + c] = a + base;
    base += t;
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) start[g.nbins] = b;
  __syncthreads();
  for (long long j0 = a + threadIdx.x; j0 < b; j0 += step) {
    R x[kRangeU][D];
    const int n = range_load<R, D>(tpos, j0, b, x);
#pragma unroll
    for (int u = 0; u < kRangeU; ++u) {
      if (u < n) {
        PointBin pb = bin_point_d<R, D>(g, x[u], &bad);
        uint32_t loc = pb.bin - (uint32_t)t0;
        if (loc >= (uint32_t)nt) loc = nt - 1;
        const long long dst = a + atomicAdd(&cnt[loc], 1u);
        Rec<R> o;
        o.t[0] = (R)pb.t[0];
        o.t[1] = (R)pb.t[1];
        o.t[2] = (R)pb.t[2];
        o.cell = pb.cell;
        rec[dst] = o;
        perm[dst] = (int)(j0 + (long long)u * blockDim.x);
      }
    }
  }
  if (stray) atomicOr(flag, 2);
}

// grad[i] = gseg[slot of i] (caller's order from the range order)
template <class R>
__global__ void range_gather_kernel(long long N, int d, uint32_t bpc, int nblk, int shift,
                                    const uint32_t* __restrict__ kr,
                                    const uint32_t* __restrict__ H,
                                    const long long* __restrict__ kstart,
                                    const R* __restrict__ gseg, R* __restrict__ grad) {
  uint32_t c;
  const long long q = xcd_point_block(blockIdx.x, bpc, &c);
  const long long i = q * 256 + threadIdx.x;
  if (c >= (uint32_t)nblk || i >= N) return;
  const long long src = range_slot(kr[i], shift, c, nblk, H, kstart);
  if (d == 2) {
    using V2 = typename std::conditional<sizeof(R) == 4, float2, double2>::type;
    const V2 v = reinterpret_cast<const V2*>(gseg)[src];
    if (((uintptr_t)grad & (sizeof(V2) - 1)) == 0) {
      reinterpret_cast<V2*>(grad)[i] = v;
    } else {
      grad[2 * i] = v.x;
      grad[2 * i + 1] = v.y;
    }
  } else {
    for (int a = 0; a < d; ++a) grad[i * d + a] = gseg[src * d + a];
  }
}

// out[j] = tidx[perm[j]]
__global__ void compose_index_kernel(long long N, const int* __restrict__ perm,
                                     const int* __restrict__ tidx, int* __restrict__ out) {
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < N) out[j] = tidx[perm[j]];
}

// Fallback for very many tiles: global atomic counts (key, rank per point).
// Each run of consecutive lanes of a wavefront with the same tile takes its
// ranks with one atomic (points that arrive in tile order share few; in random
// order every run is one lane).
template <class R>
__global__ void bin_count_kernel(Geom g, const R* __restrict__ pos, uint32_t* __restrict__ key,
                                 uint32_t* __restrict__ rank, uint32_t* __restrict__ count,
                                 int* __restrict__ flag) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool valid = i < g.N;
  bool bad = false;
  uint32_t k = 0xffffffffu;
  if (valid) {
    PointBin pb = bin_point<R>(g, pos + i * g.d, &bad);
    k = pb.bin;
  }
  if (bad) atomicOr(flag, 1);
  // points past N sit at the end of the last wavefront: each is a run of its own
  // that takes no rank
  const int lane = threadIdx.x & 63;
  const uint32_t kp = __shfl_up(k, 1, 64);
  const bool vp = __shfl_up((int)valid, 1, 64) != 0;
  const bool head = lane == 0 || !valid || !vp || kp != k;
  const unsigned long long hm = __ballot(head);
  const unsigned long long upto = (lane == 63) ? ~0ull : ((2ull << lane) - 1ull);
  const int leader = 63 - __clzll(hm & upto);
  const unsigned long long above = hm & ~upto;
  const int end = above ? __ffsll((long long)above) - 1 : 64;
  uint32_t base = 0;
  if (head && valid) base = atomicAdd(&count[k], (uint32_t)(end - lane));
  base = __shfl(base, leader, 64);
  if (valid) {
    key[i] = k;
    rank[i] = base + (uint32_t)(lane - leader);
  }
}

template <class R>
__global__ void bin_scatter_atomic_kernel(Geom g, const R* __restrict__ pos,
                                          const uint32_t* __restrict__ key,
                                          const uint32_t* __restrict__ rank,
                                          const long long* __restrict__ start,
                                          Rec<R>* __restrict__ rec, int* __restrict__ perm) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  bool bad = false;
  PointBin pb = bin_point<R>(g, pos + i * g.d, &bad);
  const long long dst = start[key[i]] + rank[i];
  Rec<R> o;
  o.t[0] = (R)pb.t[0];
  o.t[1] = (R)pb.t[1];
  o.t[2] = (R)pb.t[2];
  o.cell = pb.cell;
  rec[dst] = o;
  perm[dst] = (int)i;
}

// Exclusive scan of the per-tile counts into start[0..nbins] (one workgroup,
// chunks of 1024 in order).
__global__ void scan_bins_kernel(const uint32_t* __restrict__ count, long long nb,
                                 long long* __restrict__ start) {
  // 1024 threads; each chunk of 1024 counts: wave scans by shuffles, then the 16
  // wave totals by one wave
  __shared__ long long wsum[16];
  __shared__ long long carry;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (long long base = 0; base < nb; base += 1024) {
    const long long i = base + threadIdx.x;
    const long long v = (i < nb) ? (long long)count[i] : 0;
    long long x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
      const long long y = __shfl_up(x, off, 64);
      if (lane >= off) x += y;
    }
    if (lane == 63) wsum[wv] = x;
    __syncthreads();
    if (wv == 0) {
      long long t = (lane < 16) ? wsum[lane] : 0;
#pragma unroll
      for (int off = 1; off < 16; off <<= 1) {
        const long long y = __shfl_up(t, off, 64);
        if (lane >= off) t += y;
      }
      if (lane < 16) wsum[lane] = t;  // inclusive totals of waves 0..lane
    }
    __syncthreads();
    const long long before = carry + (wv > 0 ? wsum[wv - 1] : 0);
    if (i < nb) start[i] = before + x - v;
    __syncthreads();
    if (threadIdx.x == 0) carry += wsum[15];
    __syncthreads();
  }
  if (threadIdx.x == 0) start[nb] = carry;
}

// BIN_RANGES after the range histogram: scatter into range order, then sort
// every range by tile
template <class R>
void range_finish(const Geom& g, const BinPlan& bp, const R* src, BinBuffers& b,
                  hipStream_t st) {
  const uint32_t bpc = (uint32_t)(bp.chunk / 256);
  range_scatter_kernel<R><<<xcd_grid(bp.nblk, bp.chunk), 256, 0, st>>>(
      g.N, g.d, src, bpc, bp.nblk, bp.shift, b.kr, b.H, b.kstart, (R*)b.tpos);
  const size_t lds2 = (size_t)bp.G * sizeof(uint32_t);
  if (g.d == 2)
    range_sort_kernel<R, 2><<<(unsigned)bp.nkeys, 512, lds2, st>>>(
        g, bp.G, (const R*)b.tpos, b.kstart, b.start, (Rec<R>*)b.rec, b.perm, b.flag);
  else
    range_sort_kernel<R, 3><<<(unsigned)bp.nkeys, 512, lds2, st>>>(
        g, bp.G, (const R*)b.tpos, b.kstart, b.start, (Rec<R>*)b.rec, b.perm, b.flag);
}

// BIN_RANGES, two levels: the coarse pass into tpos0 / tidx0
template <class R>
void range_coarse(const Geom& g, const BinLevel& c, const R* pos, BinBuffers& b,
                  hipStream_t st) {
  bin_hist_kernel<R><<<8 * ((c.nblk + 7) / 8), 1024, (size_t)c.nkeys * sizeof(uint32_t), st>>>(
      g, pos, c.chunk, c.nblk, (int)c.nkeys, c.kdiv, c.shift, b.kr0, b.H0, b.flag);
  bin_rowscan_kernel<<<(unsigned)((c.nkeys + 3) / 4), 256, 0, st>>>(b.H0, c.nblk, c.nkeys,
                                                                     b.count0);
  scan_bins_kernel<<<1, 1024, 0, st>>>(b.count0, c.nkeys, b.kstart0);
  range_scatter_kernel<R><<<xcd_grid(c.nblk, c.chunk), 256, 0, st>>>(
      g.N, g.d, pos, (uint32_t)(c.chunk / 256), c.nblk, c.shift, b.kr0, b.H0, b.kstart0,
      (R*)b.tpos0);
}

void launch_bin(const Geom& g, const BinPlan& bp, const void* pos, bool f64, BinBuffers& b,
                hipStream_t st) {
  const long long nblocks = (g.N + 255) / 256;
  if (bp.mode == BIN_TILES || bp.mode == BIN_RANGES) {
    // source of the (range or tile) histogram pass: the caller's positions, or
    // the coarse pass's output
    const void* src = pos;
    if (bp.mode == BIN_RANGES && bp.levels == 2) {
      if (f64) range_coarse<double>(g, bp.coarse, (const double*)pos, b, st);
      else range_coarse<float>(g, bp.coarse, (const float*)pos, b, st);
      src = b.tpos0;
    }
    const size_t lds = (size_t)bp.nkeys * sizeof(uint32_t);
    const int nk = (int)bp.nkeys;
    if (f64)
      bin_hist_kernel<double><<<8 * ((bp.nblk + 7) / 8), 1024, lds, st>>>(g, (const double*)src, bp.chunk,
                                                         bp.nblk, nk, bp.kdiv, bp.shift, b.kr,
                                                         b.H, b.flag);
    else
      bin_hist_kernel<float><<<8 * ((bp.nblk + 7) / 8), 1024, lds, st>>>(g, (const float*)src, bp.chunk,
                                                        bp.nblk, nk, bp.kdiv, bp.shift, b.kr,
                                                        b.H, b.flag);
    bin_rowscan_kernel<<<(unsigned)((bp.nkeys + 3) / 4), 256, 0, st>>>(b.H, bp.nblk, bp.nkeys,
                                                                        b.count);
    const uint32_t bpc = (uint32_t)(bp.chunk / 256);
    if (bp.mode == BIN_TILES) {
      scan_bins_kernel<<<1, 1024, 0, st>>>(b.count, g.nbins, b.start);
      if (f64)
        bin_scatter_kernel<double><<<xcd_grid(bp.nblk, bp.chunk), 256, 0, st>>>(
            g, (const double*)pos, bpc, bp.nblk, b.kr, b.H, b.start, (Rec<double>*)b.rec,
            b.perm);
      else
        bin_scatter_kernel<float><<<xcd_grid(bp.nblk, bp.chunk), 256, 0, st>>>(
            g, (const float*)pos, bpc, bp.nblk, b.kr, b.H, b.start, (Rec<float>*)b.rec,
            b.perm);
    } else {
      scan_bins_kernel<<<1, 1024, 0, st>>>(b.count, bp.nkeys, b.kstart);
      if (f64) range_finish<double>(g, bp, (const double*)src, b, st);
      else range_finish<float>(g, bp, (const float*)src, b, st);
    }
  } else {
    launch_fill<uint32_t>(b.count, g.nbins, 0u, st);
    if (f64)
      bin_count_kernel<double><<<(unsigned)nblocks, 256, 0, st>>>(g, (const double*)pos, b.key,
                                                                 b.kr, b.count, b.flag);
    else
      bin_count_kernel<float><<<(unsigned)nblocks, 256, 0, st>>>(g, (const float*)pos, b.key,
                                                                b.kr, b.count, b.flag);
    scan_bins_kernel<<<1, 1024, 0, st>>>(b.count, g.nbins, b.start);
    if (f64)
      bin_scatter_atomic_kernel<double><<<(unsigned)nblocks, 256, 0, st>>>(
          g, (const double*)pos, b.key, b.kr, b.start, (Rec<double>*)b.rec, b.perm);
    else
      bin_scatter_atomic_kernel<float><<<(unsigned)nblocks, 256, 0, st>>>(
          g, (const float*)pos, b.key, b.kr, b.start, (Rec<float>*)b.rec, b.perm);
  }
}

// ------------------------------------------------------------- spreading
__device__ __forceinline__ void tile_coords(const Geom& g, long long bin, int* t) {
  t[0] = (int)(bin % g.nt[0]);
  long long r = bin / g.nt[0];
  t[1] = (int)(r % g.nt[1]);
  t[2] = (int)(r / g.nt[1]);
}

// add a row of W fixed-point values starting at acc[rb] with 64-bit atomics on
// aligned pairs of 32-bit cells (no carry can cross: every cell stays < 2^32)
template <int W, int I>
__device__ __forceinline__ uint32_t q_at(const uint32_t* q) {
  if constexpr (I >= 0 && I < W) return q[I];
  else return 0u;
}
template <int W, int K>
__device__ __forceinline__ void add_pair(unsigned long long* p, int par, const uint32_t* q) {
  // cells rb - par + 2K and rb - par + 2K + 1 hold row elements 2K - par and 2K + 1 - par
  const uint32_t lo = par ? q_at<W, 2 * K - 1>(q) : q_at<W, 2 * K>(q);
  const uint32_t hi = par ? q_at<W, 2 * K>(q) : q_at<W, 2 * K + 1>(q);
  const unsigned long long v = (unsigned long long)lo | ((unsigned long long)hi << 32);
  if (v) atomicAdd(p + K, v);
}
template <int W, int... K>
__device__ __forceinline__ void add_pairs(unsigned long long* p, int par, const uint32_t* q,
                                          std::integer_sequence<int, K...>) {
  (add_pair<W, K>(p, par, q), ...);
}
template <int W>
__device__ __forceinline__ void add_row_pairs(uint32_t* acc, int rb, const uint32_t* q) {
  const int par = rb & 1;
  unsigned long long* p = reinterpret_cast<unsigned long long*>(acc + (rb - par));
  add_pairs<W>(p, par, q, std::make_integer_sequence<int, (W + 2) / 2>{});
}


// STR: point strengths c_j (any sign), read through the permutation; every cell
// is then one 64-bit two's-complement fixed-point word (in FP32 too), which adds
// signed contributions exactly; the scale also covers max |c|.
// KEPT: an optimiser trial step that keeps the tile order of the last binning
// (kp): the block first forms the trial point and the record of each of its
// slots (kept_tile_record, relative to this tile), writes both, and spreads
// from the records it wrote.
template <class R, int D, int W, bool STR, bool KEPT>
__device__ __forceinline__ void spread_body(const Geom& g, const Rec<R>* __restrict__ rec,
                                            const long long* __restrict__ start,
                                            R* __restrict__ tiles, const R* __restrict__ cstr,
                                            const int* __restrict__ perm, double cmax,
                                            const KeptSpread<R>& kp) {
  constexpr bool F32 = sizeof(R) == 4 && !STR;  // 32-bit cells added in pairs
  extern __shared__ unsigned long long smem_u64[];
  uint32_t* acc32 = reinterpret_cast<uint32_t*>(smem_u64);
  unsigned long long* acc64 = smem_u64;
  const long long bin = blockIdx.x;
  const int E0 = g.E[0], E1 = g.E[1], E2 = (D == 3) ? g.E[2] : 1;
  const int ncell = E0 * E1 * E2;
  R alpha = R(0);
  if constexpr (KEPT) {
    // step length, as the trial point pass takes it (every block; block 0
    // stores a new direction's)
    __shared__ double ksh[16];
    __shared__ double ka;
    const int step = *kp.step;
    if (step == LB_REJECT || step == LB_IDLE) {
      if (threadIdx.x == 0) ka = *kp.alpha;
    } else {
      double pm = 0.0;
      for (int b = threadIdx.x; b < kp.nb; b += blockDim.x) pm = fmax(pm, kp.part1[b]);
      for (int off = 32; off > 0; off >>= 1) pm = fmax(pm, __shfl_down(pm, off, 64));
      if ((threadIdx.x & 63) == 0) ksh[threadIdx.x >> 6] = pm;
      __syncthreads();
      if (threadIdx.x == 0) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t = fmax(t, ksh[w]);
        const double a = (t > kp.max_step) ? kp.max_step / t : 1.0;
        ka = a;
        if (blockIdx.x == 0) *kp.alpha = a;
      }
    }
    __syncthreads();
    alpha = (R)ka;
  }
  const long long s = start[bin], e = start[bin + 1];
  R* __restrict__ out = tiles + bin * (long long)ncell;
  if (e == s) {
    for (int c = threadIdx.x; c < ncell; c += blockDim.x) out[c] = R(0);
    return;  // uniform across the block
  }

  // Fixed-point scale from a bound on the number of points whose footprints
  // cover one cell (each contributes at most 1): a cell's contributors have
  // their footprint starts in one w x w window of start cells (over the last two
  // axes; in 3D every start of the column counts), and every such window lies
  // within K x K blocks of 2 x 2 start cells, K = w / 2 + 1.  The starts are
  // counted per block, and the largest sum over K x K blocks bounds every cell's
  // contributors (at most 64 / 49 of the exact w x w maximum in area at w = 7,
  // so the scale keeps all but a fraction of a bit; the exact box sums took 13%
  // of the spreading kernel).
  __shared__ uint32_t smax[16];
  uint32_t cov;
  {
    // footprint starts span the tile and the slack on both sides
    const int Ta = ((D == 3) ? g.T[1] : g.T[0]) + 2 * g.slack;
    const int Tb = ((D == 3) ? g.T[2] : g.T[1]) + 2 * g.slack;
    const int Sa = (Ta + 1) >> 1, Sb = (Tb + 1) >> 1;  // 2 x 2 blocks of start cells
    uint32_t* cnt = acc32;  // Sa Sb <= ncell words, before the accumulator is cleared
    for (int c = threadIdx.x; c < Sa * Sb; c += blockDim.x) cnt[c] = 0u;
    __syncthreads();
    auto count_cell = [&](uint32_t cl) {
      const int la = (D == 3) ? (int)((cl >> 8) & 0xff) : (int)(cl & 0xff);
      const int lb = (D == 3) ? (int)((cl >> 16) & 0xff) : (int)((cl >> 8) & 0xff);
      atomicAdd(cnt + (lb >> 1) * Sa + (la >> 1), 1u);
    };
    if constexpr (KEPT) {
      // the trial point and record of every slot of the tile, counted as they
      // are formed (the records are written for the spreading below, the
      // interpolation and the next update)
      int tcv[3];
      tile_coords(g, bin, tcv);
      const uint32_t tu[3] = {(uint32_t)tcv[0], (uint32_t)tcv[1], (uint32_t)tcv[2]};
      const uint32_t tc = kept_tile_pack(tu);
      bool bad = false, off = false;
      // two slots per thread and trip, every load of both issued before the
      // first use (the loads are a chain: slot -> point -> position)
      const long long bd = blockDim.x;
      for (long long j0 = s + threadIdx.x; j0 < e; j0 += 2 * bd) {
        const long long j1 = j0 + bd;
        const bool has1 = j1 < e;
        const long long i0 = kp.perm[j0];
        const long long i1 = has1 ? kp.perm[j1] : i0;
        R x0[D], p0[D], x1[D], p1[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
          x0[a] = kp.x[i0 * D + a];
          p0[a] = kp.p[i0 * D + a];
          x1[a] = kp.x[i1 * D + a];
          p1[a] = kp.p[i1 * D + a];
        }
        R v0[D], v1[D];
#pragma unroll
        for (int a = 0; a < D; ++a) {
          v0[a] = x0[a] + alpha * p0[a];
          v1[a] = x1[a] + alpha * p1[a];
          kp.xt[i0 * D + a] = v0[a];
          if (has1) kp.xt[i1 * D + a] = v1[a];
        }
        const Rec<R> r0 = kept_tile_record<R, D>(g, v0, tc, &bad, &off);
        kp.rec[j0] = r0;
        count_cell(r0.cell);
        if (has1) {
          const Rec<R> r1 = kept_tile_record<R, D>(g, v1, tc, &bad, &off);
          kp.rec[j1] = r1;
          count_cell(r1.cell);
        }
      }
      if (bad) atomicOr(kp.flag, 1);
      if (off && !bad) atomicOr(kp.drift, 1);
    } else {
      // four cells loaded per thread before the first count
      for (long long jb = s + threadIdx.x; jb < e; jb += 4LL * blockDim.x) {
        uint32_t cl[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const long long j = jb + (long long)u * blockDim.x;
          cl[u] = (j < e) ? rec[j].cell : 0u;
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (jb + (long long)u * blockDim.x < e) count_cell(cl[u]);
      }
    }
    __syncthreads();
    // largest sum over K x K blocks (K x all when the tile has fewer): a block
    // window that leaves the grid holds a subset of one that does not
    constexpr int K = W / 2 + 1;
    uint32_t mx = 0;
    {
      const int ka = K < Sa ? K : Sa, kb = K < Sb ? K : Sb;
      const int na = Sa - ka + 1, nb = Sb - kb + 1;
      for (int o = threadIdx.x; o < na * nb; o += blockDim.x) {
        const int jb = o / na, ia = o - jb * na;
        uint32_t sum = 0;
        for (int y = 0; y < kb; ++y)
          for (int x = 0; x < ka; ++x) sum += cnt[(jb + y) * Sa + ia + x];
        mx = sum > mx ? sum : mx;
      }
    }
    for (int off = 32; off > 0; off >>= 1) {
      const uint32_t o = (uint32_t)__shfl_down((int)mx, off, 64);
      mx = o > mx ? o : mx;
    }
    if ((threadIdx.x & 63) == 0) smax[threadIdx.x >> 6] = mx;
    __syncthreads();
    cov = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) cov = smax[w] > cov ? smax[w] : cov;
    __syncthreads();
  }
  for (int c = threadIdx.x; c < ncell + 2; c += blockDim.x) {
    if (F32) acc32[c] = 0u;
    else acc64[c] = 0ull;
  }
  // with strengths every contribution is at most max |c| in magnitude, and the
  // signed words keep one bit for the sign
  const int ex = STR ? (int)floor(log2(ldexp(1.0, 62) / ((double)(cov + 1) * cmax)))
                     : fixed_exponent((long long)cov, F32 ? 31 : 63);
  const R scale = (R)ldexp(1.0, ex);
  const double inv_scale = ldexp(1.0, -ex);
  const R beta = (R)g.beta;
  __syncthreads();
  for (long long j = s + threadIdx.x; j < e; j += blockDim.x) {
    const Rec<R> p = rec[j];
    const R cj = STR ? cstr[perm[j]] * scale : scale;
    R k0[W], k1[W], k2[W];
    spread_weights<R, W>(p.t[0], beta, k0);
    spread_weights<R, W>(p.t[1], beta, k1);
    if (D == 3) spread_weights<R, W>(p.t[2], beta, k2);
    const int l0 = p.cell & 0xff, l1 = (p.cell >> 8) & 0xff, l2 = (p.cell >> 16) & 0xff;
    const int zmax = (D == 3) ? W : 1;
    for (int dz = 0; dz < zmax; ++dz) {
      const R pz = (D == 3) ? k2[dz] * cj : cj;
#pragma unroll
      for (int dy = 0; dy < W; ++dy) {
        const R py = k1[dy] * pz;
        const int rb = ((D == 3 ? (l2 + dz) * E1 : 0) + (l1 + dy)) * E0 + l0;
        if (F32) {
          uint32_t q[W];
#pragma unroll
          for (int dx = 0; dx < W; ++dx) q[dx] = __float2uint_rn((float)(py * k0[dx]));
          add_row_pairs<W>(acc32, rb, q);
        } else if (STR) {
#pragma unroll
          for (int dx = 0; dx < W; ++dx)
            atomicAdd(acc64 + rb + dx,
                      (unsigned long long)(long long)llrint((double)(py * k0[dx])));
        } else {
#pragma unroll
          for (int dx = 0; dx < W; ++dx)
            atomicAdd(acc64 + rb + dx, (unsigned long long)((double)(py * k0[dx]) + 0.5));
        }
      }
    }
  }
  __syncthreads();
  for (int c = threadIdx.x; c < ncell; c += blockDim.x) {
    if (F32) out[c] = (R)((R)acc32[c] * (R)inv_scale);
    else if (STR) out[c] = (R)((double)(long long)acc64[c] * inv_scale);
    else out[c] = (R)((R)acc64[c] * (R)inv_scale);
  }
}

template <class R, int D, int W, bool STR, bool KEPT = false>
__global__ void spread_kernel(Geom g, const Rec<R>* __restrict__ rec,
                              const long long* __restrict__ start, R* __restrict__ tiles,
                              const R* __restrict__ cstr, const int* __restrict__ perm,
                              double cmax, KeptSpread<R> kp) {
  spread_body<R, D, W, STR, KEPT>(g, rec, start, tiles, cstr, perm, cmax, kp);
}
// The kept-order variant without strengths: its pointers took 83 scalar
// registers, with which only three of its 512-thread workgroups were resident
// per CU (a quarter of the tiles started when the first finished); within 64
// (the rest kept in vector lanes) all four are, 29.3 -> 26.2 us.
template <class R, int W>
__global__ __attribute__((amdgpu_num_sgpr(64))) void spread_kept_kernel(
    Geom g, const Rec<R>* __restrict__ rec, const long long* __restrict__ start,
    R* __restrict__ tiles, KeptSpread<R> kp) {
  spread_body<R, 2, W, false, true>(g, rec, start, tiles, nullptr, nullptr, 1.0, kp);
}

// Fold: grid cell (x, y, z) = sum over the padded tiles that cover it.  For each
// axis, cover[a] lists (tile, local index) pairs per grid coordinate (CSR).  One
// block per grid row (y, z); the y and z cover lists are uniform across it.
template <class R, int D>
__global__ void fold_kernel(Geom g, FoldTables ft, const R* __restrict__ tiles,
                            R* __restrict__ grid) {
  const long long ncell = (long long)g.E[0] * g.E[1] * (D == 3 ? g.E[2] : 1);
  const uint32_t row = blockIdx.x;
  const int y = (int)(row % (uint32_t)g.nf[1]);
  const int z = (int)(row / (uint32_t)g.nf[1]);
  const int yb = ft.off[1][y], ye = ft.off[1][y + 1];
  const int zb = (D == 3) ? ft.off[2][z] : 0, ze = (D == 3) ? ft.off[2][z + 1] : 1;
  R* __restrict__ out = grid + (long long)row * g.nf[0];
  for (int x = threadIdx.x; x < g.nf[0]; x += blockDim.x) {
    const int xb = ft.off[0][x], xe = ft.off[0][x + 1];
    R acc = R(0);
    for (int iz = zb; iz < ze; ++iz) {
      const int tz = (D == 3) ? ft.ent[2][iz].x : 0, lz = (D == 3) ? ft.ent[2][iz].y : 0;
      for (int iy = yb; iy < ye; ++iy) {
        const int ty = ft.ent[1][iy].x, ly = ft.ent[1][iy].y;
        const long long base = (long long)(g.nt[0] * (ty + g.nt[1] * tz)) * ncell +
                               (lz * g.E[1] + ly) * g.E[0];
        for (int ix = xb; ix < xe; ++ix) {
          const int2 ex = ft.ent[0][ix];
          acc += tiles[base + (long long)ex.x * ncell + ex.y];
        }
      }
    }
    out[x] = acc;
  }
}

// ---------------------------------------------------------- interpolation
// Field tile origin is one cell before the spreading tile (width w + 1), extent
// T + w + 1 per axis (g.Ei); with the cached tile order of the optimiser's trial
// steps, whose footprints may start g.slack cells outside their tile, the field
// tile grows by g.islack = g.slack on each side (Ei = T + 2 slack + w + 1).  In FP32 the LDS rows are padded to a multiple of
// four floats (zeros) and a point reads each row of its footprint as kRowQ
// aligned 16-byte words from the aligned cell at or below its first column; the
// x weights are shifted by the alignment offset once per point (zeros outside
// the footprint), so each row costs kRowQ LDS reads instead of w + 1 and the
// sum over the row keeps its order (the extra terms add exact zeros).
constexpr int interp_row_words(int wi) { return (wi + 3 + 3) / 4; }
// the words of a row reach at most 4 ceil((wi + 3) / 4) - wi <= 6 cells past its
// footprint
constexpr int kInterpTail = 8;
inline int interp_row_stride(const Geom& g, bool f32) {
  return f32 ? (g.Ei[0] + 3) / 4 * 4 : g.Ei[0];
}
// FP32 2D: the field tile is held four times in LDS, copy s shifted right by s
// cells (rows of interp_copy_stride words), so that every point reads its
// footprint rows as whole aligned 16-byte words of the copy s = -l0 mod 4, with
// its own weights, unshifted (footprints that are not a multiple of 4 cells read
// zero-filled cells past their end with weight 0)
template <class R, int D, int WI>
constexpr bool interp_shift4() {
  return sizeof(R) == 4 && D == 2;
}
// a row read spans cells l0 + s .. l0 + s + 4 ceil(WI / 4) - 1, l0 <= Ei0 - WI
constexpr int interp_copy_stride(int Ei0, int WI) {
  return (Ei0 - WI + (WI + 3) / 4 * 4 + 6) / 4 * 4;
}

// Register budget of the interpolation (workgroups of at most 512 threads, so
// up to 256 registers): FP32 kernels up to width 7 keep the occupancy they
// were tuned at, 4 waves per SIMD in 2D (128 registers) and 5 in 3D (92
// registers, no spill, against 105 at 4 waves: 3D interpolation 885 -> 809
// us; a 2D limit of 5 or more spills, and unrolling the 2D row loop less to
// free registers measured slower); wider and FP64 kernels take the registers
// they need instead of spilling under the 128 of a 1024-thread bound.
template <class R, int D, int W>
constexpr int interp_min_waves() {
  return (sizeof(R) == 4 && W <= 7) ? (D == 3 ? (W == 7 ? 5 : 1) : 4) : 1;
}
// footprint rows per unrolled step: all of them for FP32 up to width 8 (every
// row's LDS words in flight together); two for wider or FP64 footprints, whose
// hoisted rows would not fit in the registers
template <class R, int W>
constexpr int interp_row_unroll() {
  return (sizeof(R) == 4 && W <= 8) ? W + 1 : 2;
}

// LDS bytes of the field tile (the outlier list follows it)
template <class R>
__host__ __device__ inline size_t interp_tile_bytes(const Geom& g) {
  if (sizeof(R) == 4 && g.d == 2)  // four shifted copies
    return (size_t)4 * interp_copy_stride(g.Ei[0], g.wi) * g.Ei[1] * sizeof(R);
  // rows padded in FP32, plus the cells past the end
  const int rs = sizeof(R) == 4 ? (g.Ei[0] + 3) / 4 * 4 : g.Ei[0];
  return ((size_t)rs * g.Ei[1] * (g.d == 3 ? g.Ei[2] : 1) + kInterpTail) * sizeof(R);
}
template <class R, int D, int W>
__global__ __launch_bounds__(512)
__attribute__((amdgpu_waves_per_eu(interp_min_waves<R, D, W>())))
void interp_kernel(Geom g, const Rec<R>* __restrict__ rec,
                              const long long* __restrict__ start, const int* __restrict__ perm,
                              const R* __restrict__ v, R* __restrict__ grad,
                              const R* __restrict__ cstr, R* __restrict__ val) {
  constexpr int WI = W + 1;
  constexpr bool F32 = sizeof(R) == 4;
  constexpr int NQ = interp_row_words(WI);
  extern __shared__ float4 smem_f4[];
  R* sub = reinterpret_cast<R*>(smem_f4);
  const long long bin = blockIdx.x;
  const int E0 = g.Ei[0], E1 = g.Ei[1], E2 = (D == 3) ? g.Ei[2] : 1;
  const int E0s = F32 ? (E0 + 3) / 4 * 4 : E0;  // LDS row stride
  const int ncell = E0s * E1 * E2;
  constexpr bool SH4 = interp_shift4<R, D, WI>();
  const int Ec = interp_copy_stride(E0, WI);  // row stride of the shifted copies
  const int csz = Ec * E1;                // words per copy
  const long long s = start[bin], e = start[bin + 1];
  if (e == s) return;
  int t[3];
  tile_coords(g, bin, t);
  const int o0 = t[0] * g.T[0] - 1 - g.islack + g.nf[0];
  const int o1 = t[1] * g.T[1] - 1 - g.islack + g.nf[1];
  const int o2 = (D == 3) ? t[2] * g.T[2] - 1 - g.islack + g.nf[2] : 0;
  // the field over the tile, KB loads in flight per thread before the LDS
  // stores; row padding and the kInterpTail cells past the end (read by the last
  // row's words) are zero.  Cell c = (c2 E1 + c1) E0s + c0: one division per
  // thread, then the coordinates step by the block size.
  if constexpr (SH4 && WI % 4 != 0) {
    // cells the copies do not receive read as zero
    float4* z4 = reinterpret_cast<float4*>(sub);
    for (int i = threadIdx.x; i < csz; i += blockDim.x) z4[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    __syncthreads();
  }
  {
    constexpr int KB = 12;
    const int bd = (int)blockDim.x;
    const int total = ncell + kInterpTail;
    const int dr = bd / E0s, dc = bd - dr * E0s;
    int c0 = (int)threadIdx.x % E0s;
    int c1 = (int)threadIdx.x / E0s;
    int c2 = 0;
    while (c1 >= E1) {
      c1 -= E1;
      ++c2;
    }
    for (int cb = threadIdx.x; cb < total; cb += KB * bd) {
      R val[KB];
      int li[KB];  // shifted copies: index r Ec + x of the cell, or -1
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        const int c = cb + u * bd;
        val[u] = R(0);
        li[u] = (c < ncell && c0 < E0) ? (c2 * E1 + c1) * Ec + c0 : -1;
        if (c < ncell && c0 < E0) {
          int x = o0 + c0, y = o1 + c1, z = o2 + c2;
          while (x >= g.nf[0]) x -= g.nf[0];
          while (y >= g.nf[1]) y -= g.nf[1];
          while (z >= g.nf[2]) z -= g.nf[2];
          val[u] = v[((long long)z * g.nf[1] + y) * g.nf[0] + x];
        }
        c0 += dc;
        c1 += dr;
        if (c0 >= E0s) {
          c0 -= E0s;
          ++c1;
        }
        while (c1 >= E1) {
          c1 -= E1;
          ++c2;
        }
      }
      if constexpr (SH4) {
        // cell (row r, column x) to index r Ec + x + s of copy s, s = 0..3
#pragma unroll
        for (int u = 0; u < KB; ++u) {
          if (li[u] >= 0) {
            R* d0p = sub + li[u];
#pragma unroll
            for (int sc = 0; sc < 4; ++sc) d0p[sc * csz + sc] = val[u];
          }
        }
      } else {
#pragma unroll
        for (int u = 0; u < KB; ++u) {
          const int c = cb + u * bd;
          if (c < total) sub[c] = val[u];
        }
      }
    }
  }
  __syncthreads();
  const R beta = (R)g.beta_i;
  const R icb = (R)g.icb;
  R gs[3];
  for (int a = 0; a < 3; ++a) gs[a] = (a < D) ? (R)g.gsc[a] : R(0);
  // 2D rows stored as one pair when the output is aligned for it
  const bool pair_store = ((uintptr_t)grad & (2 * sizeof(R) - 1)) == 0;
  for (long long j = s + threadIdx.x; j < e; j += blockDim.x) {
    const Rec<R> p = rec[j];
    const int q = perm[j];
    R f0[WI], d0[WI], f1[WI], d1[WI], f2[WI], d2[WI];
    int l[3];
    const int cl[3] = {(int)(p.cell & 0xff), (int)((p.cell >> 8) & 0xff),
                       (int)((p.cell >> 16) & 0xff)};
    // footprint of width W + 1: tau_i = tau + 1/2 starting at l0 (tau < 1/2), or
    // tau - 1/2 starting one cell earlier
#pragma unroll
    for (int a = 0; a < D; ++a) {
      const int k = (p.t[a] >= R(0.5)) ? 1 : 0;
      const R ti = k ? p.t[a] - R(0.5) : p.t[a] + R(0.5);
      l[a] = cl[a] - (g.slack - g.islack) - k + 1;
      if (a == 0) interp_weights<R, WI>(ti, beta, icb, f0, d0);
      else if (a == 1) interp_weights<R, WI>(ti, beta, icb, f1, d1);
      else interp_weights<R, WI>(ti, beta, icb, f2, d2);
    }
    // FP32: x weights shifted by the alignment offset of the first column (or,
    // with the shifted copies, the copy that aligns it)
    const int xb = F32 ? (l[0] & ~3) : l[0];
    const int sc = (4 - (l[0] & 3)) & 3;
    const R* sub4 = sub + sc * csz + l[0] + sc;
    R f0s[4 * NQ], d0s[4 * NQ];
    if constexpr (F32 && !SH4) {
      const int sh = l[0] & 3;
#pragma unroll
      for (int k = 0; k < 4 * NQ; ++k) {
        R a = R(0), b = R(0);
#pragma unroll
        for (int q = 0; q < 4; ++q)
          if (k - q >= 0 && k - q < WI && sh == q) {
            a = f0[k - q];
            b = d0[k - q];
          }
        f0s[k] = a;
        d0s[k] = b;
      }
    }
    R gx = R(0), gy = R(0), gz = R(0), gv = R(0);
    const int zmax = (D == 3) ? WI : 1;
    // one footprint plane at a time: unrolled, the compiler hoists the row reads
    // of several planes and spills registers
#pragma nounroll
    for (int dz = 0; dz < zmax; ++dz) {
      R sxy = R(0), sdxy = R(0), sxdy = R(0);
#pragma unroll(interp_row_unroll<R, W>())
      for (int dy = 0; dy < WI; ++dy) {
        const R* row = sub + ((D == 3 ? (l[2] + dz) * E1 : 0) + (l[1] + dy)) * E0s + xb;
        R sx = R(0), sdx = R(0);
        if constexpr (SH4) {
          const float4* q4 = reinterpret_cast<const float4*>(sub4 + (l[1] + dy) * Ec);
          constexpr int NQ4 = (WI + 3) / 4;
#pragma unroll
          for (int k4 = 0; k4 < NQ4; ++k4) {
            const float4 w4 = q4[k4];
            const float v4[4] = {w4.x, w4.y, w4.z, w4.w};
#pragma unroll
            for (int i = 0; i < 4; ++i) {
              const int k = 4 * k4 + i;
              sx += v4[i] * (k < WI ? f0[k < WI ? k : 0] : R(0));
              sdx += v4[i] * (k < WI ? d0[k < WI ? k : 0] : R(0));
            }
          }
        } else if constexpr (F32) {
          const float4* q4 = reinterpret_cast<const float4*>(row);
#pragma unroll
          for (int k4 = 0; k4 < NQ; ++k4) {
            const float4 w4 = q4[k4];
            sx += w4.x * f0s[4 * k4];
            sdx += w4.x * d0s[4 * k4];
            sx += w4.y * f0s[4 * k4 + 1];
            sdx += w4.y * d0s[4 * k4 + 1];
            sx += w4.z * f0s[4 * k4 + 2];
            sdx += w4.z * d0s[4 * k4 + 2];
            sx += w4.w * f0s[4 * k4 + 3];
            sdx += w4.w * d0s[4 * k4 + 3];
          }
        } else {
#pragma unroll
          for (int dx = 0; dx < WI; ++dx) {
            const R vv = row[dx];
            sx += vv * f0[dx];
            sdx += vv * d0[dx];
          }
        }
        sxy += sx * f1[dy];
        sdxy += sdx * f1[dy];
        sxdy += sx * d1[dy];
      }
      if (D == 3) {
        gx += sdxy * f2[dz];
        gy += sxdy * f2[dz];
        gz += sxy * d2[dz];
        gv += sxy * f2[dz];
      } else {
        gx = sdxy;
        gy = sxdy;
        gv = sxy;
      }
    }
    // point strengths scale the position gradient (the field's value, for the
    // strength gradient, is not scaled)
    R sg[3] = {gs[0], gs[1], gs[2]};
    if (cstr) {
      const R cq = cstr[q];
      sg[0] *= cq;
      sg[1] *= cq;
      sg[2] *= cq;
    }
    if (val) val[q] = gv;
    const long long o = (long long)q * D;
    if (D == 2 && pair_store) {
      using V2 = typename std::conditional<sizeof(R) == 4, float2, double2>::type;
      V2 w2;
      w2.x = gx * sg[0];
      w2.y = gy * sg[1];
      reinterpret_cast<V2*>(grad)[q] = w2;
    } else {
      grad[o] = gx * sg[0];
      grad[o + 1] = gy * sg[1];
      if (D == 3) grad[o + 2] = gz * sg[2];
    }
  }
}

// --------------------------------------------------------------- launch
#define FRESCO_W_SWITCH(W_, CALL) \
  switch (W_) {                   \
    case 2: CALL(2); break;       \
    case 3: CALL(3); break;       \
    case 4: CALL(4); break;       \
    case 5: CALL(5); break;       \
    case 6: CALL(6); break;       \
    case 7: CALL(7); break;       \
    case 8: CALL(8); break;       \
    case 9: CALL(9); break;       \
    case 10: CALL(10); break;     \
    case 11: CALL(11); break;     \
    case 12: CALL(12); break;     \
    case 13: CALL(13); break;     \
    case 14: CALL(14); break;     \
    case 15: CALL(15); break;     \
    case 16: CALL(16); break;     \
  }

// accumulator (ncell + 2 words), then the coverage bound's row sums (Tb Ea
// 32-bit words over the last two axes)
template <class R>
size_t spread_lds_bytes(const Geom& g, bool str) {
  // the accumulator (the start-block counts of the coverage bound use its first
  // words before it is cleared)
  const size_t ncell = (size_t)g.E[0] * g.E[1] * (g.d == 3 ? g.E[2] : 1);
  return (ncell + 2) * (sizeof(R) == 4 && !str ? 4 : 8);
}
template <class R>
size_t interp_lds_bytes(const Geom& g) {
  return interp_tile_bytes<R>(g);
}

// one-time kernel attributes (dynamic LDS above the default limit); returns
// the first failure
template <class R>
hipError_t spread_prepare(const Geom& g) {
  const int sl = (int)spread_lds_bytes<R>(g, false);
  const int il = (int)std::max(interp_lds_bytes<R>(interp_geom(g, false)),
                               interp_lds_bytes<R>(interp_geom(g, true)));
  const int slc = (int)spread_lds_bytes<R>(g, true);
  hipError_t e = hipSuccess;
  auto lds = [&e](const void* f, int bytes) {
    if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  };
#define PREP(W)                                                 \
  do {                                                          \
    if (g.d == 2) {                                             \
      lds((const void*)spread_kernel<R, 2, W, false>, sl);      \
      lds((const void*)spread_kept_kernel<R, W>, sl);          \
      lds((const void*)interp_kernel<R, 2, W>, il);             \
      if (slc <= kMaxSpreadLds)                                 \
        lds((const void*)spread_kernel<R, 2, W, true>, slc);    \
      if (slc <= kMaxSpreadLds)                                 \
        lds((const void*)spread_kernel<R, 2, W, true, true>, slc); \
    } else {                                                    \
      lds((const void*)spread_kernel<R, 3, W, false>, sl);      \
      lds((const void*)interp_kernel<R, 3, W>, il);             \
      if (slc <= kMaxSpreadLds)                                 \
        lds((const void*)spread_kernel<R, 3, W, true>, slc);    \
    }                                                           \
  } while (0)
  FRESCO_W_SWITCH(g.w, PREP)
#undef PREP
  // block-private histograms: at most 16384 keys
  lds((const void*)bin_hist_kernel<R>, 16384 * 4);
  return e;
}

template <class R>
void launch_spread(const Geom& g, const Rec<R>* rec, const long long* start, R* tiles,
                   const Strengths<R>& cs, hipStream_t st, const KeptSpread<R>* kept) {
  const bool str = cs.c != nullptr;
  const size_t lds = spread_lds_bytes<R>(g, str);
  const int threads = 512;  // (2D: 26.7 -> 23.5 us against 256)
  KeptSpread<R> kp;
  std::memset(&kp, 0, sizeof(kp));
  if (kept) kp = *kept;
  // the kept tile order exists in 2D only (a slack)
#define SP(W)                                                                                 \
  do {                                                                                        \
    if (g.d == 2 && kept && !str)                                                             \
      spread_kept_kernel<R, W><<<(unsigned)g.nbins, threads, lds, st>>>(g, rec, start, tiles, \
                                                                        kp);                  \
    else if (g.d == 2 && kept)                                                                \
      spread_kernel<R, 2, W, true, true><<<(unsigned)g.nbins, threads, lds, st>>>(           \
          g, rec, start, tiles, cs.c, cs.perm, cs.cmax, kp);                                  \
    else if (g.d == 2 && !str)                                                                \
      spread_kernel<R, 2, W, false><<<(unsigned)g.nbins, threads, lds, st>>>(                \
          g, rec, start, tiles, nullptr, nullptr, 1.0, kp);                                   \
    else if (g.d == 2)                                                                        \
      spread_kernel<R, 2, W, true><<<(unsigned)g.nbins, threads, lds, st>>>(                 \
          g, rec, start, tiles, cs.c, cs.perm, cs.cmax, kp);                                  \
    else if (!str)                                                                            \
      spread_kernel<R, 3, W, false><<<(unsigned)g.nbins, threads, lds, st>>>(                \
          g, rec, start, tiles, nullptr, nullptr, 1.0, kp);                                   \
    else                                                                                      \
      spread_kernel<R, 3, W, true><<<(unsigned)g.nbins, threads, lds, st>>>(                 \
          g, rec, start, tiles, cs.c, cs.perm, cs.cmax, kp);                                  \
  } while (0)
  FRESCO_W_SWITCH(g.w, SP)
#undef SP
}

template <class R>
void launch_fold(const Geom& g, const R* tiles, R* grid, const FoldTables& ft, hipStream_t st) {
  const unsigned rows = (unsigned)(g.ngrid / g.nf[0]);
  int threads = ((g.nf[0] + 63) / 64) * 64;
  if (threads > 256) threads = 256;
  if (g.d == 2) fold_kernel<R, 2><<<rows, threads, 0, st>>>(g, ft, tiles, grid);
  else fold_kernel<R, 3><<<rows, threads, 0, st>>>(g, ft, tiles, grid);
}

template <class R>
void launch_interp(const Geom& g, const BinPlan& bp, const BinBuffers& b, const R* v, R* grad,
                   const Strengths<R>& cs, hipStream_t st) {
  const size_t lds = interp_lds_bytes<R>(g);
  // 2D: 256 threads, four workgroups per CU; field tiles covering a slack hold
  // more than a quarter of the LDS, so 512 threads, two workgroups per CU (whole
  // rounds of 512 tiles instead of 768 and a tail)
  const int threads = (g.d == 3 || g.islack > 0) ? 512 : 256;
  const Rec<R>* rec = (const Rec<R>*)b.rec;
  const long long* start = b.start;
  const int* perm = b.perm;
  // BIN_RANGES: the gradient goes to the range order first (tpos is free once
  // the records are sorted), then to the caller's order
  R* out = (bp.mode == BIN_RANGES) ? (R*)b.tpos : grad;
#define IP(W)                                                                                 \
  do {                                                                                        \
    if (g.d == 2)                                                                             \
      interp_kernel<R, 2, W><<<(unsigned)g.nbins, threads, lds, st>>>(                       \
          g, rec, start, perm, v, out, cs.c, cs.val);                                         \
    else                                                                                      \
      interp_kernel<R, 3, W><<<(unsigned)g.nbins, threads, lds, st>>>(                       \
          g, rec, start, perm, v, out, cs.c, cs.val);                                         \
  } while (0)
  FRESCO_W_SWITCH(g.w, IP)
#undef IP
  if (bp.mode == BIN_RANGES) {
    // range order -> source order of the range pass (the caller's, or the
    // coarse order, then the caller's)
    R* mid = (bp.levels == 2) ? (R*)b.tpos0 : grad;
    range_gather_kernel<R><<<xcd_grid(bp.nblk, bp.chunk), 256, 0, st>>>(
        g.N, g.d, (uint32_t)(bp.chunk / 256), bp.nblk, bp.shift, b.kr, b.H, b.kstart, out,
        mid);
    if (bp.levels == 2) {
      const BinLevel& c = bp.coarse;
      range_gather_kernel<R><<<xcd_grid(c.nblk, c.chunk), 256, 0, st>>>(
          g.N, g.d, (uint32_t)(c.chunk / 256), c.nblk, c.shift, b.kr0, b.H0, b.kstart0, mid,
          grad);
    }
  }
}

// Caller index per slot of a stable sort by the first-level key (the tile, or
// the range of tiles): the points of one key keep their caller order.  Slot =
// off[key] + H[key * nblk + chunk] (the histogram pass and its scans) + the
// number of earlier points of the chunk with that key, counted in index order:
// lanes of one wavefront with equal keys are grouped by ballots, and the
// wavefronts of the block add to the running counts one after the other.  One
// workgroup of 1024 threads per histogram chunk; LDS: nkeys running counts.
template <class R>
__global__ void bin_stable_kernel(Geom g, const R* __restrict__ pos, long long chunk, int nblk,
                                  int nkeys, FastDiv kdiv, const uint32_t* __restrict__ H,
                                  const long long* __restrict__ off, int* __restrict__ out) {
  extern __shared__ uint32_t run[];
  for (int k = threadIdx.x; k < nkeys; k += blockDim.x) run[k] = 0u;
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (int)(blockDim.x >> 6);
  const unsigned long long below = (1ull << lane) - 1ull;
  const long long i0 = (long long)blockIdx.x * chunk;
  long long i1 = i0 + chunk;
  if (i1 > g.N) i1 = g.N;
  for (long long sb = i0; sb < i1; sb += blockDim.x) {
    const long long i = sb + threadIdx.x;
    const bool valid = i < i1;
    uint32_t key = 0xffffffffu;
    if (valid) {
      bool bad = false;
      key = fdiv(bin_point<R>(g, pos + i * g.d, &bad).bin, kdiv);
    }
    // lanes of this wavefront with the same key (the lowest unassigned lane's
    // key per round)
    unsigned long long peers = 0ull;
    bool done = !valid;
    for (;;) {
      const unsigned long long act = __ballot(!done);
      if (act == 0ull) break;
      const int ld = __ffsll((long long)act) - 1;
      const uint32_t lk = (uint32_t)__shfl((int)key, ld, 64);
      const bool mine = !done && key == lk;
      const unsigned long long m = __ballot(mine);
      if (mine) {
        peers = m;
        done = true;
      }
    }
    const uint32_t wr = (uint32_t)__popcll(peers & below);
    const bool last = valid && (peers >> lane) == 1ull;
    uint32_t r = 0;
    for (int w = 0; w < nw; ++w) {
      if (wave == w && valid) r = run[key] + wr;
      __syncthreads();
      if (wave == w && last) run[key] += (uint32_t)__popcll(peers);
      __syncthreads();
    }
    if (valid) out[off[key] + H[(long long)key * nblk + blockIdx.x] + r] = (int)i;
  }
}

bool launch_stable_index(const Geom& g, const BinPlan& bp, const BinBuffers& b, const void* pos,
                         bool f64, int* out, hipStream_t st) {
  const bool ok = bp.mode == BIN_TILES || (bp.mode == BIN_RANGES && bp.levels == 1);
  if (!ok) return false;
  const long long* off = (bp.mode == BIN_TILES) ? b.start : b.kstart;
  const size_t lds = (size_t)bp.nkeys * sizeof(uint32_t);
  const int nk = (int)bp.nkeys;
  // at most 16384 keys, as for the histogram pass (never under stream capture:
  // called when an optimiser call fixes its order)
  const void* fn = f64 ? (const void*)bin_stable_kernel<double> : (const void*)bin_stable_kernel<float>;
  if (hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, 16384 * 4) != hipSuccess)
    return false;  // the caller takes the sorted-index path
  if (f64)
    bin_stable_kernel<double><<<bp.nblk, 1024, lds, st>>>(g, (const double*)pos, bp.chunk,
                                                         bp.nblk, nk, bp.kdiv, b.H, off, out);
  else
    bin_stable_kernel<float><<<bp.nblk, 1024, lds, st>>>(g, (const float*)pos, bp.chunk,
                                                        bp.nblk, nk, bp.kdiv, b.H, off, out);
  return true;
}

void launch_sorted_index(const Geom& g, const BinPlan& bp, const BinBuffers& b, int* out,
                         hipStream_t st) {
  if (bp.mode == BIN_RANGES) {
    // range order -> caller index (through the coarse order with two levels),
    // then sorted record -> caller index
    const int* sidx = nullptr;
    if (bp.levels == 2) {
      const BinLevel& c = bp.coarse;
      range_index_kernel<<<xcd_grid(c.nblk, c.chunk), 256, 0, st>>>(
          g.N, (uint32_t)(c.chunk / 256), c.nblk, c.shift, b.kr0, b.H0, b.kstart0, nullptr,
          b.tidx0);
      sidx = b.tidx0;
    }
    range_index_kernel<<<xcd_grid(bp.nblk, bp.chunk), 256, 0, st>>>(
        g.N, (uint32_t)(bp.chunk / 256), bp.nblk, bp.shift, b.kr, b.H, b.kstart, sidx, b.tidx);
    compose_index_kernel<<<(unsigned)((g.N + 255) / 256), 256, 0, st>>>(g.N, b.perm, b.tidx,
                                                                         out);
  } else
    (void)hipMemcpyAsync(out, b.perm, sizeof(int) * g.N, hipMemcpyDeviceToDevice, st);
}

template size_t spread_lds_bytes<float>(const Geom&, bool);
template size_t spread_lds_bytes<double>(const Geom&, bool);
template size_t interp_lds_bytes<float>(const Geom&);
template size_t interp_lds_bytes<double>(const Geom&);
template hipError_t spread_prepare<float>(const Geom&);
template hipError_t spread_prepare<double>(const Geom&);
template void launch_spread<float>(const Geom&, const Rec<float>*, const long long*, float*,
                                   const Strengths<float>&, hipStream_t,
                                   const KeptSpread<float>*);
template void launch_spread<double>(const Geom&, const Rec<double>*, const long long*, double*,
                                    const Strengths<double>&, hipStream_t,
                                    const KeptSpread<double>*);
template void launch_fold<float>(const Geom&, const float*, float*, const FoldTables&,
                                 hipStream_t);
template void launch_fold<double>(const Geom&, const double*, double*, const FoldTables&,
                                  hipStream_t);
template void launch_interp<float>(const Geom&, const BinPlan&, const BinBuffers&, const float*,
                                   float*, const Strengths<float>&, hipStream_t);
template void launch_interp<double>(const Geom&, const BinPlan&, const BinBuffers&,
                                    const double*, double*, const Strengths<double>&, hipStream_t);

}  // namespace fresco
