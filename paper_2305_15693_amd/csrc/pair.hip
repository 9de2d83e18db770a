// Soft-core pair repulsion for packings (Results, stealthy hyperuniform
// packings: a short-range repulsion added to the spectral loss so that
// particles keep a minimum distance):
//   U(r) = (eps / alpha) (1 - r / sigma)^alpha for r < sigma, else 0,
//   E = sum_{i<j} U(r_ij) under the minimum image convention (sigma < L_a / 2),
//   dE/dr_i = sum_{j != i} U'(r_ij) (r_i - r_j) / r_ij,
//   U'(r) = -(eps / sigma) (1 - r / sigma)^(alpha - 1).
// alpha = 2 is the harmonic soft core; alpha = 2.5 the Hertzian one.
//
// Cell list, one pass per evaluation (O(N)):
//   key      cell of every point (FP64 wrap into the box), arrival rank in its
//            cell from a global atomic counter;
//   scan     exclusive scan of the cell counts (three-phase, fixed order);
//   scatter  records (position as given, original index) into cell order;
//   order    each cell's records sorted by original index (the arrival order of
//            the atomics is not reproducible; after this step the layout is);
//   force    one thread per point visits the (up to 3^d distinct) neighbour
//            cells in a fixed order and accumulates its gradient in FP64 and
//            half of every pair energy into FP64 block partials.
// Cells have side L_a / nc_a >= sigma; when sigma-sized cells would exceed
// kMaxCells the side grows (more candidates per point, bounded memory).
// Differences are taken in FP64 from the stored coordinates, so wrapping and the
// minimum image add no error in the FP32 build.
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>

#include "common.h"
#include "pair.h"

namespace fresco {

constexpr long long kMaxCells = 1LL << 24;
constexpr int kScanPer = 4096;  // counts per scan block (1024 threads x 4)

template <class R>
struct alignas(sizeof(R) == 4 ? 16 : 32) PairRec {
  R x[3];
  int idx;
};

struct PairGeom {
  int d;
  long long n;
  double L[3];
  double cfac[3];  // nc / L
  double invL[3];  // 1 / L
  int nc[3];
  double sigma, eps, alpha;
};

template <class R>
__device__ __forceinline__ uint32_t pair_cell(const PairGeom& g, const R* r, int* k, bool* bad) {
  uint32_t c = 0;
  for (int a = 2; a >= 0; --a) {
    int ka = 0;
    if (a < g.d) {
      double x = (double)r[a];
      if (!isfinite(x)) {
        *bad = true;
        x = 0.0;
      }
      double u = x - g.L[a] * floor(x * g.invL[a]);  // clamped below if rounding lands on L
      ka = (int)(u * g.cfac[a]);
      if (ka < 0) ka = 0;
      if (ka >= g.nc[a]) ka = g.nc[a] - 1;
    }
    k[a] = ka;
    c = c * (uint32_t)g.nc[a] + (uint32_t)ka;
  }
  return c;
}

template <class R>
__global__ void pair_key_kernel(PairGeom g, const R* __restrict__ pos, uint32_t* __restrict__ key,
                                uint32_t* __restrict__ rank, uint32_t* __restrict__ count,
                                int* __restrict__ flag) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  bool bad = false;
  int k[3];
  const uint32_t c = pair_cell<R>(g, pos + i * g.d, k, &bad);
  if (bad) atomicOr(flag, 1);
  key[i] = c;
  rank[i] = atomicAdd(&count[c], 1u);
}

// --- three-phase exclusive scan of count[0..nc) into start[0..nc]
__device__ __forceinline__ uint32_t block_incl_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
  // 1024 threads: wave scans, then a scan of the 16 wave totals
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) sh[wave] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t run = 0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      const uint32_t t = sh[w];
      sh[w] = run;
      run += t;
    }
    sh[16] = run;
  }
  __syncthreads();
  x += sh[wave];
  *total = sh[16];
  __syncthreads();
  return x;
}

__global__ void scan_reduce_kernel(const uint32_t* __restrict__ count, long long nc,
                                   uint32_t* __restrict__ bsum) {
  __shared__ uint32_t sh[17];
  const long long base = (long long)blockIdx.x * kScanPer + threadIdx.x * 4;
  uint32_t v = 0;
  for (int q = 0; q < 4; ++q)
    if (base + q < nc) v += count[base + q];
  uint32_t tot;
  (void)block_incl_scan(v, sh, &tot);
  if (threadIdx.x == 0) bsum[blockIdx.x] = tot;
}

// one block: exclusive scan of the block sums in place; start[nc] = total
__global__ void scan_top_kernel(uint32_t* __restrict__ bsum, int nb, uint32_t* __restrict__ start,
                                long long nc) {
  __shared__ uint32_t sh[17];
  uint32_t carry = 0;
  for (int base = 0; base < nb; base += 1024) {
    const int i = base + threadIdx.x;
    const uint32_t v = (i < nb) ? bsum[i] : 0u;
    uint32_t tot;
    const uint32_t x = block_incl_scan(v, sh, &tot);
    if (i < nb) bsum[i] = carry + x - v;
    carry += tot;
  }
  if (threadIdx.x == 0) start[nc] = carry;
}

__global__ void scan_down_kernel(const uint32_t* __restrict__ count, long long nc,
                                 const uint32_t* __restrict__ bsum, uint32_t* __restrict__ start) {
  __shared__ uint32_t sh[17];
  const long long base = (long long)blockIdx.x * kScanPer + threadIdx.x * 4;
  uint32_t c4[4], v = 0;
  for (int q = 0; q < 4; ++q) {
    c4[q] = (base + q < nc) ? count[base + q] : 0u;
    v += c4[q];
  }
  uint32_t tot;
  uint32_t x = block_incl_scan(v, sh, &tot) - v + bsum[blockIdx.x];
  for (int q = 0; q < 4; ++q) {
    if (base + q < nc) start[base + q] = x;
    x += c4[q];
  }
}

template <class R>
__global__ void pair_scatter_kernel(PairGeom g, const R* __restrict__ pos,
                                    const uint32_t* __restrict__ key,
                                    const uint32_t* __restrict__ rank,
                                    const uint32_t* __restrict__ start,
                                    PairRec<R>* __restrict__ sorted) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.n) return;
  PairRec<R> o;
  for (int a = 0; a < 3; ++a) o.x[a] = (a < g.d) ? pos[i * g.d + a] : R(0);
  o.idx = (int)i;
  sorted[start[key[i]] + rank[i]] = o;
}

// insertion sort of each cell's records by original index
template <class R>
__global__ void pair_order_kernel(long long nc, const uint32_t* __restrict__ start,
                                  PairRec<R>* __restrict__ sorted) {
  const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= nc) return;
  const uint32_t b = start[c], e = start[c + 1];
  for (uint32_t i = b + 1; i < e; ++i) {
    const PairRec<R> r = sorted[i];
    uint32_t j = i;
    while (j > b && sorted[j - 1].idx > r.idx) {
      sorted[j] = sorted[j - 1];
      --j;
    }
    sorted[j] = r;
  }
}

template <class R>
__global__ void pair_force_kernel(PairGeom g, const PairRec<R>* __restrict__ sorted,
                                  const uint32_t* __restrict__ start, R* __restrict__ grad,
                                  int accumulate, double weight, double* __restrict__ part) {
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double e = 0.0;
  if (s < g.n) {
    const PairRec<R> me = sorted[s];
    bool bad = false;
    int k[3];
    (void)pair_cell<R>(g, me.x, k, &bad);
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      if (a >= g.d || g.nc[a] == 1) {
        lo[a] = 0;
        hi[a] = 0;
      } else if (g.nc[a] == 2) {
        lo[a] = 0;  // the two neighbours coincide
        hi[a] = 1;
      } else {
        lo[a] = -1;
        hi[a] = 1;
      }
    }
    const double s2 = g.sigma * g.sigma;
    const double isig = 1.0 / g.sigma;
    double acc[3] = {0.0, 0.0, 0.0};
    // the neighbour cells along x of one (y, z) row are consecutive in the cell
    // order: at most two runs of records per row (one more where the row wraps)
    int ra0[2], ra1[2], nrun;
    {
      const int n0 = g.nc[0], k0 = k[0];
      if (lo[0] == 0 && hi[0] == 0) {
        ra0[0] = 0; ra1[0] = 0; nrun = 1;
      } else if (lo[0] == 0) {  // two cells along x
        ra0[0] = 0; ra1[0] = 1; nrun = 1;
      } else if (k0 == 0) {
        ra0[0] = 0; ra1[0] = 1; ra0[1] = n0 - 1; ra1[1] = n0 - 1; nrun = 2;
      } else if (k0 == n0 - 1) {
        ra0[0] = n0 - 2; ra1[0] = n0 - 1; ra0[1] = 0; ra1[1] = 0; nrun = 2;
      } else {
        ra0[0] = k0 - 1; ra1[0] = k0 + 1; nrun = 1;
      }
    }
    for (int oz = lo[2]; oz <= hi[2]; ++oz) {
      int cz = k[2] + oz;
      if (cz < 0) cz += g.nc[2];
      if (cz >= g.nc[2]) cz -= g.nc[2];
      for (int oy = lo[1]; oy <= hi[1]; ++oy) {
        int cy = k[1] + oy;
        if (cy < 0) cy += g.nc[1];
        if (cy >= g.nc[1]) cy -= g.nc[1];
        const uint32_t row = (uint32_t)g.nc[0] * ((uint32_t)cy + (uint32_t)g.nc[1] * (uint32_t)cz);
        for (int rr = 0; rr < nrun; ++rr) {
          const uint32_t b = start[row + ra0[rr]], en = start[row + ra1[rr] + 1];
          for (uint32_t t = b; t < en; ++t) {
            const PairRec<R> o = sorted[t];
            if (o.idx == me.idx) continue;
            double dx[3], r2 = 0.0;
            for (int a = 0; a < 3; ++a) {
              if (a < g.d) {
                double v = (double)me.x[a] - (double)o.x[a];
                v -= g.L[a] * rint(v * g.invL[a]);
                dx[a] = v;
                r2 += v * v;
              } else {
                dx[a] = 0.0;
              }
            }
            if (r2 >= s2) continue;
            const double r = sqrt(r2);
            const double x = 1.0 - r * isig;
            double xa1;  // x^(alpha - 1)
            if (g.alpha == 2.0) xa1 = x;
            else xa1 = pow(x, g.alpha - 1.0);
            e += 0.5 * (g.eps / g.alpha) * xa1 * x;
            if (r > 0.0) {
              const double f = -g.eps * isig * xa1 / r;
              for (int a = 0; a < 3; ++a) acc[a] += f * dx[a];
            }
          }
        }
      }
    }
    for (int a = 0; a < g.d; ++a) {
      const long long o = (long long)me.idx * g.d + a;
      const double v = weight * acc[a];
      grad[o] = accumulate ? (R)((double)grad[o] + v) : (R)v;
    }
  }
  // block partial of the energy (fixed order)
  __shared__ double sh[4];
  for (int off = 32; off > 0; off >>= 1) e += __shfl_down(e, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = e;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// Overlaps (main text, quasicrystalline structures: points that end up on top
// of one another are removed and redrawn between minimisation cycles): flag[i]
// = 1 when a point of lower index lies closer than sqrt(thr2) to point i under
// the minimum image (thr at most the cell side, so that the neighbour cells hold
// every candidate).  Differences in FP64 from the stored coordinates.
template <class R>
__global__ void overlap_flag_kernel(PairGeom g, const PairRec<R>* __restrict__ sorted,
                                    const uint32_t* __restrict__ start, double thr2,
                                    uint32_t* __restrict__ flag) {
  const long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= g.n) return;
  const PairRec<R> me = sorted[s];
  bool bad = false;
  int k[3];
  (void)pair_cell<R>(g, me.x, k, &bad);
  // distinct neighbour cells per axis: all of them on an axis of one or two
  // cells, else k - 1, k, k + 1 (periodic)
  int lo[3], cnt[3];
  for (int a = 0; a < 3; ++a) {
    if (g.nc[a] <= 2) {
      lo[a] = 0;
      cnt[a] = g.nc[a];
    } else {
      lo[a] = k[a] - 1 + g.nc[a];
      cnt[a] = 3;
    }
  }
  uint32_t hit = 0;
  for (int iz = 0; iz < cnt[2] && !hit; ++iz) {
    const int cz = (lo[2] + iz) % g.nc[2];
    for (int iy = 0; iy < cnt[1] && !hit; ++iy) {
      const int cy = (lo[1] + iy) % g.nc[1];
      for (int ix = 0; ix < cnt[0] && !hit; ++ix) {
        const int cx = (lo[0] + ix) % g.nc[0];
        const uint32_t cell =
            (uint32_t)cx + (uint32_t)g.nc[0] * ((uint32_t)cy + (uint32_t)g.nc[1] * (uint32_t)cz);
        for (uint32_t t = start[cell]; t < start[cell + 1]; ++t) {
          const PairRec<R> o = sorted[t];
          if (o.idx >= me.idx) continue;
          double r2 = 0.0;
          for (int a = 0; a < g.d; ++a) {
            double v = (double)me.x[a] - (double)o.x[a];
            v -= g.L[a] * rint(v * g.invL[a]);
            r2 += v * v;
          }
          if (r2 < thr2) {
            hit = 1;
            break;
          }
        }
      }
    }
  }
  flag[me.idx] = hit;
}

// pos[i] = fresh[rank[i]] for every flagged point (rank: exclusive scan of the
// flags in index order)
template <class R>
__global__ void overlap_replace_kernel(R* __restrict__ pos, const uint32_t* __restrict__ flag,
                                       const uint32_t* __restrict__ rank,
                                       const R* __restrict__ fresh, long long n, int d) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !flag[i]) return;
  for (int a = 0; a < d; ++a) pos[i * d + a] = fresh[(long long)rank[i] * d + a];
}

__global__ void pair_fill_kernel(uint32_t* p, long long n) {
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x)
    p[i] = 0u;
}

// energy = sum of the partials (fixed order); flag handed over and cleared
__global__ void pair_finish_kernel(const double* __restrict__ part, int nb, double* __restrict__ out,
                                   int* __restrict__ flag, int* __restrict__ flag_out) {
  __shared__ double s[256];
  double v = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) v += part[i];
  s[threadIdx.x] = v;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = s[0];
    if (flag_out) flag_out[0] = flag[0];
    flag[0] = 0;
  }
}

static PairGeom pair_geom(const fresco_pair_ctx* pc) {
  PairGeom g;
  std::memset(&g, 0, sizeof(g));
  g.d = pc->d;
  g.n = pc->n;
  for (int a = 0; a < 3; ++a) {
    g.L[a] = pc->L[a];
    g.nc[a] = pc->nc[a];
    g.cfac[a] = (double)pc->nc[a] / pc->L[a];
    g.invL[a] = 1.0 / pc->L[a];
  }
  g.sigma = pc->sigma;
  g.eps = pc->eps;
  g.alpha = pc->alpha;
  return g;
}

// the cell list of pos: keys, scan, records in cell order sorted by index
template <class R>
static void pair_cells_t(fresco_pair_ctx* pc, const R* pos, hipStream_t st) {
  const PairGeom g = pair_geom(pc);
  const unsigned nb = (unsigned)((pc->n + 255) / 256);
  long long fb = (pc->ncell + 255) / 256;
  if (fb > 16384) fb = 16384;
  pair_fill_kernel<<<(unsigned)fb, 256, 0, st>>>(pc->count, pc->ncell);
  pair_key_kernel<R><<<nb, 256, 0, st>>>(g, pos, pc->key, pc->rank, pc->count, pc->flag);
  scan_reduce_kernel<<<pc->nscan_blocks, 1024, 0, st>>>(pc->count, pc->ncell, pc->bsum);
  scan_top_kernel<<<1, 1024, 0, st>>>(pc->bsum, pc->nscan_blocks, pc->start, pc->ncell);
  scan_down_kernel<<<pc->nscan_blocks, 1024, 0, st>>>(pc->count, pc->ncell, pc->bsum, pc->start);
  PairRec<R>* sorted = (PairRec<R>*)pc->sorted;
  pair_scatter_kernel<R><<<nb, 256, 0, st>>>(g, pos, pc->key, pc->rank, pc->start, sorted);
  pair_order_kernel<R><<<(unsigned)((pc->ncell + 255) / 256), 256, 0, st>>>(pc->ncell, pc->start,
                                                                            sorted);
}

template <class R>
static int pair_enqueue_t(fresco_pair_ctx* pc, const R* pos, R* grad, bool accumulate,
                          double weight, hipStream_t st) {
  const PairGeom g = pair_geom(pc);
  const unsigned nb = (unsigned)((pc->n + 255) / 256);
  pair_cells_t<R>(pc, pos, st);
  pair_force_kernel<R><<<nb, 256, 0, st>>>(g, (const PairRec<R>*)pc->sorted, pc->start, grad,
                                           accumulate ? 1 : 0, weight, pc->part);
  return hipGetLastError() == hipSuccess ? FRESCO_OK : FRESCO_EHIP;
}

static int pair_enqueue_cells(fresco_pair_ctx* pc, const void* pos, hipStream_t st) {
  if (pc->dtype == FRESCO_F32) pair_cells_t<float>(pc, (const float*)pos, st);
  else pair_cells_t<double>(pc, (const double*)pos, st);
  return hipGetLastError() == hipSuccess ? FRESCO_OK : FRESCO_EHIP;
}

int pair_enqueue(fresco_pair_ctx* pc, const void* pos, void* grad, bool accumulate, double weight,
                 hipStream_t st) {
  if (pc->dtype == FRESCO_F32)
    return pair_enqueue_t<float>(pc, (const float*)pos, (float*)grad, accumulate, weight, st);
  return pair_enqueue_t<double>(pc, (const double*)pos, (double*)grad, accumulate, weight, st);
}

}  // namespace fresco

using namespace fresco;

// Checks a pair problem and fills the cell geometry of pc: cells of side
// >= sigma, grown until there are at most kMaxCells; scan and force block counts.
static int pair_plan(const fresco_pair_problem* p, fresco_pair_ctx* pc) {
  if (!p) return FRESCO_EINVAL;
  if (p->dim != 2 && p->dim != 3) return FRESCO_EINVAL;
  if (p->dtype != FRESCO_F32 && p->dtype != FRESCO_F64) return FRESCO_EINVAL;
  if (p->n < 1) return FRESCO_EINVAL;
  if (p->n > 2147483647LL) return FRESCO_ENOTSUP;
  if (!(p->sigma > 0.0) || !std::isfinite(p->sigma) || !(p->eps > 0.0) || !std::isfinite(p->eps) ||
      !(p->alpha >= 1.0) || !std::isfinite(p->alpha))
    return FRESCO_EINVAL;
  for (int a = 0; a < p->dim; ++a)
    if (!(p->box[a] > 2.0 * p->sigma) || !std::isfinite(p->box[a])) return FRESCO_EINVAL;
  pc->d = p->dim;
  pc->dtype = p->dtype;
  pc->n = p->n;
  pc->sigma = p->sigma;
  pc->eps = p->eps;
  pc->alpha = p->alpha;
  double side = p->sigma;
  for (;;) {
    long long tot = 1;
    for (int a = 0; a < 3; ++a) {
      if (a < p->dim) {
        pc->L[a] = p->box[a];
        long long k = (long long)std::floor(p->box[a] / side);
        if (k < 1) k = 1;
        if (k > (1LL << 20)) k = 1LL << 20;
        pc->nc[a] = (int)k;
      } else {
        pc->L[a] = 1.0;
        pc->nc[a] = 1;
      }
      tot *= pc->nc[a];
    }
    if (tot <= kMaxCells) {
      pc->ncell = tot;
      break;
    }
    side *= 1.05;
  }
  pc->nscan_blocks = (int)((pc->ncell + kScanPer - 1) / kScanPer);
  pc->nblocks = (int)((pc->n + 255) / 256);
  return FRESCO_OK;
}

static void pair_copy_geometry(const fresco_pair_ctx& g, fresco_pair_ctx* pc) {
  pc->d = g.d;
  pc->dtype = g.dtype;
  pc->n = g.n;
  for (int a = 0; a < 3; ++a) {
    pc->L[a] = g.L[a];
    pc->nc[a] = g.nc[a];
  }
  pc->sigma = g.sigma;
  pc->eps = g.eps;
  pc->alpha = g.alpha;
  pc->ncell = g.ncell;
  pc->nscan_blocks = g.nscan_blocks;
  pc->nblocks = g.nblocks;
}

template <class T>
static int pair_alloc(fresco_pair_ctx* pc, T** p, size_t count) {
  void* q = nullptr;
  if (hipMalloc(&q, sizeof(T) * (count ? count : 1)) != hipSuccess) return FRESCO_ENOMEM;
  pc->allocs.push_back(q);
  *p = (T*)q;
  return FRESCO_OK;
}

// ---------------------------------------------------------------------------
// Scratch of fresco_pair_energy_grad_noalloc: the cell list of one evaluation
// (keys, ranks, counts, starts, scan sums, records, energy partials, flag) in a
// file-scope device array, so that the call allocates nothing.  Each GPU the
// library runs on holds its own copy until the process ends.  In host code the
// array's name is not a device address: the address is taken once per device
// with hipGetSymbolAddress (with that device current) and only that address is
// passed to kernels.
constexpr size_t kPairScratchBytes = size_t(32) << 20;
static __device__ __align__(256) unsigned char scratch[kPairScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch (looked up on the first call).
int scratch_address(int dev, void** out) {
  if (dev < 0 || dev >= kMaxDevices) return FRESCO_ENOTSUP;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* ptr = nullptr;
    if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) {
      (void)hipGetLastError();
      return FRESCO_EHIP;
    }
    g_scratch_ptr[dev] = ptr;
  }
  *out = g_scratch_ptr[dev];
  return FRESCO_OK;
}

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

// Carves the cell-list buffers of geometry pc out of base; returns the bytes
// used (the caller compares them with the scratch size before launching).
size_t pair_carve(fresco_pair_ctx* pc, unsigned char* base) {
  const size_t rs = (pc->dtype == FRESCO_F32) ? sizeof(PairRec<float>) : sizeof(PairRec<double>);
  size_t off = 0;
  auto take = [&](size_t bytes) {
    unsigned char* p = base ? base + off : nullptr;
    off = align256(off + bytes);
    return p;
  };
  pc->key = (uint32_t*)take(sizeof(uint32_t) * pc->n);
  pc->rank = (uint32_t*)take(sizeof(uint32_t) * pc->n);
  pc->count = (uint32_t*)take(sizeof(uint32_t) * pc->ncell);
  pc->start = (uint32_t*)take(sizeof(uint32_t) * (pc->ncell + 1));
  pc->bsum = (uint32_t*)take(sizeof(uint32_t) * pc->nscan_blocks);
  pc->sorted = take(rs * pc->n);
  pc->part = (double*)take(sizeof(double) * pc->nblocks);
  pc->flag = (int*)take(sizeof(int));
  return off;
}

}  // namespace

extern "C" {

int fresco_pair_energy_grad_noalloc(const fresco_pair_problem* p, const void* pos,
                                    double* energy_dev, void* grad, void* stream) {
  if (!pos || !energy_dev || !grad) return FRESCO_EINVAL;
  fresco_pair_ctx pc;  // geometry and scratch views only; owns nothing
  int st = pair_plan(p, &pc);
  if (st) return st;
  if (pair_carve(&pc, nullptr) > kPairScratchBytes) return FRESCO_ENOTSUP;
  hipStream_t hs = (hipStream_t)stream;
  int cur = -1, sdev = -1;
  if (hipGetDevice(&cur) != hipSuccess) return FRESCO_EHIP;
  if (hs) {
    if (hipStreamGetDevice(hs, &sdev) != hipSuccess) return FRESCO_EHIP;
    if (sdev != cur) return FRESCO_EINVAL;  // the stream must belong to the current device
  }
  void* base = nullptr;
  if ((st = scratch_address(cur, &base))) return st;
  pair_carve(&pc, (unsigned char*)base);
  pc.st = hs;
  // the flag must start at zero: the array keeps the previous call's contents
  // (a fill kernel rather than a memset node, so that the call can be captured)
  pair_fill_kernel<<<1, 64, 0, hs>>>((uint32_t*)pc.flag, 1);
  if ((st = pair_enqueue(&pc, pos, grad, false, 1.0, hs))) return st;
  pair_finish_kernel<<<1, 256, 0, hs>>>(pc.part, pc.nblocks, energy_dev, pc.flag, nullptr);
  return hipGetLastError() == hipSuccess ? FRESCO_OK : FRESCO_EHIP;
}

int fresco_pair_destroy(fresco_pair_ctx* pc) {
  if (!pc) return FRESCO_OK;
  (void)hipStreamSynchronize(pc->st);
  for (void* p : pc->allocs) (void)hipFree(p);
  if (pc->energy_host) (void)hipHostFree(pc->energy_host);
  if (pc->ocount_host) (void)hipHostFree(pc->ocount_host);
  delete pc;
  return FRESCO_OK;
}

int fresco_pair_create(fresco_pair_ctx** out, const fresco_pair_problem* p, void* stream) {
  if (!out) return FRESCO_EINVAL;
  *out = nullptr;
  fresco_pair_ctx geom;
  int vs = pair_plan(p, &geom);
  if (vs) return vs;
  fresco_pair_ctx* pc = new (std::nothrow) fresco_pair_ctx();
  if (!pc) return FRESCO_ENOMEM;
  pair_copy_geometry(geom, pc);
  pc->st = (hipStream_t)stream;
  const size_t rs = (p->dtype == FRESCO_F32) ? sizeof(PairRec<float>) : sizeof(PairRec<double>);
  int st = FRESCO_OK;
  void* sorted = nullptr;
  if (!st) st = pair_alloc(pc, &pc->key, pc->n);
  if (!st) st = pair_alloc(pc, &pc->rank, pc->n);
  if (!st) st = pair_alloc(pc, &pc->count, pc->ncell);
  if (!st) st = pair_alloc(pc, &pc->start, pc->ncell + 1);
  if (!st) st = pair_alloc(pc, &pc->bsum, pc->nscan_blocks);
  if (!st) st = pair_alloc(pc, (char**)&sorted, rs * pc->n);
  if (!st) st = pair_alloc(pc, &pc->part, pc->nblocks);
  if (!st) st = pair_alloc(pc, &pc->flag, 1);
  if (!st) st = pair_alloc(pc, &pc->edev, 1);
  if (!st) st = pair_alloc(pc, &pc->fout, 1);
  pc->sorted = sorted;
  if (!st && hipMemset(pc->flag, 0, sizeof(int)) != hipSuccess) st = FRESCO_EHIP;
  if (!st && hipHostMalloc((void**)&pc->energy_host, 2 * sizeof(double)) != hipSuccess)
    st = FRESCO_ENOMEM;
  if (st) {
    fresco_pair_destroy(pc);
    return st;
  }
  *out = pc;
  return FRESCO_OK;
}

int fresco_pair_energy_grad_async(fresco_pair_ctx* pc, const void* pos, double* energy_dev,
                                  void* grad) {
  if (!pc || !pos || !energy_dev || !grad) return FRESCO_EINVAL;
  int st = pair_enqueue(pc, pos, grad, false, 1.0, pc->st);
  if (st) return st;
  pair_finish_kernel<<<1, 256, 0, pc->st>>>(pc->part, pc->nblocks, energy_dev, pc->flag, nullptr);
  return hipGetLastError() == hipSuccess ? FRESCO_OK : FRESCO_EHIP;
}

int fresco_pair_replace_overlaps(fresco_pair_ctx* pc, void* pos, double threshold,
                                 const void* fresh, int64_t n_fresh, int64_t* n_replaced) {
  if (!pc || !pos || !n_replaced || n_fresh < 0 || (n_fresh > 0 && !fresh)) return FRESCO_EINVAL;
  if (!(threshold > 0.0) || threshold > pc->sigma) return FRESCO_EINVAL;
  *n_replaced = 0;
  const long long n = pc->n;
  const int nsb = (int)((n + kScanPer - 1) / kScanPer);
  int st = FRESCO_OK;
  if (!pc->oflag) {
    if (!st) st = pair_alloc(pc, &pc->oflag, n);
    if (!st) st = pair_alloc(pc, &pc->orank, n + 1);
    if (!st) st = pair_alloc(pc, &pc->obsum, nsb);
    if (!st && hipHostMalloc((void**)&pc->ocount_host, sizeof(uint32_t)) != hipSuccess)
      st = FRESCO_ENOMEM;
    if (st) return st;
  }
  hipStream_t hs = pc->st;
  // the cell list of the current positions (the gradient output is scratch here)
  st = pair_enqueue_cells(pc, pos, hs);
  if (st) return st;
  const PairGeom g = pair_geom(pc);
  const unsigned nb = (unsigned)((n + 255) / 256);
  if (pc->dtype == FRESCO_F32)
    overlap_flag_kernel<float><<<nb, 256, 0, hs>>>(g, (const PairRec<float>*)pc->sorted, pc->start,
                                                  threshold * threshold, pc->oflag);
  else
    overlap_flag_kernel<double><<<nb, 256, 0, hs>>>(
        g, (const PairRec<double>*)pc->sorted, pc->start, threshold * threshold, pc->oflag);
  scan_reduce_kernel<<<nsb, 1024, 0, hs>>>(pc->oflag, n, pc->obsum);
  scan_top_kernel<<<1, 1024, 0, hs>>>(pc->obsum, nsb, pc->orank, n);
  scan_down_kernel<<<nsb, 1024, 0, hs>>>(pc->oflag, n, pc->obsum, pc->orank);
  if (hipGetLastError() != hipSuccess) return FRESCO_EHIP;
  if (hipMemcpyAsync(pc->ocount_host, pc->orank + n, sizeof(uint32_t), hipMemcpyDeviceToHost,
                     hs) != hipSuccess ||
      hipStreamSynchronize(hs) != hipSuccess)
    return FRESCO_EHIP;
  const int64_t count = (int64_t)*pc->ocount_host;
  if (count > n_fresh) {
    *n_replaced = count;  // how many would be needed; positions untouched
    return FRESCO_EINVAL;
  }
  if (count > 0) {
    if (pc->dtype == FRESCO_F32)
      overlap_replace_kernel<float><<<nb, 256, 0, hs>>>((float*)pos, pc->oflag, pc->orank,
                                                        (const float*)fresh, n, pc->d);
    else
      overlap_replace_kernel<double><<<nb, 256, 0, hs>>>((double*)pos, pc->oflag, pc->orank,
                                                         (const double*)fresh, n, pc->d);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(hs) != hipSuccess)
      return FRESCO_EHIP;
  }
  *n_replaced = count;
  return FRESCO_OK;
}

int fresco_pair_energy_grad(fresco_pair_ctx* pc, const void* pos, double* energy, void* grad) {
  if (!pc || !pos || !energy || !grad) return FRESCO_EINVAL;
  int st = pair_enqueue(pc, pos, grad, false, 1.0, pc->st);
  if (st) return st;
  // energy and flag land in device scratch, then in the pinned host slots
  pair_finish_kernel<<<1, 256, 0, pc->st>>>(pc->part, pc->nblocks, pc->edev, pc->flag, pc->fout);
  if (hipMemcpyAsync(pc->energy_host, pc->edev, sizeof(double), hipMemcpyDeviceToHost, pc->st) !=
          hipSuccess ||
      hipMemcpyAsync(pc->energy_host + 1, pc->fout, sizeof(int), hipMemcpyDeviceToHost, pc->st) !=
          hipSuccess)
    return FRESCO_EHIP;
  if (hipGetLastError() != hipSuccess) return FRESCO_EHIP;
  if (hipStreamSynchronize(pc->st) != hipSuccess) return FRESCO_EHIP;
  *energy = pc->energy_host[0];
  if (*reinterpret_cast<int*>(pc->energy_host + 1)) return FRESCO_ENONFINITE;
  return FRESCO_OK;
}

}  // extern "C"
