// Batched evaluation of many independent small problems (a ragged batch of
// configurations with their own N, box and target), and L-BFGS over the batch
// with one captured graph per trial step.
//
// Every configuration is the problem of the main text (loss
// sum_K W (S - S0)^2 and its position gradient, evaluated through nonuniform
// FFTs as in the Methods); the mode cube, the accuracy and therefore the fine
// grid are shared by the batch, and a configuration's whole grid fits in LDS.
// The points of all configurations are cut into chunks (work items) of at most
// `chunk` points, so that a batch of very uneven configurations still spreads
// its work evenly over the CUs.  One evaluation is three launches:
//   spread   per work item: points -> fixed-point LDS grid with integer LDS
//            atomics (exact, order independent; scale 2^ex from a bound on the
//            points that cover one cell) -> the item's partial grid;
//   modes    per configuration: sum of its items' partial grids (fixed order),
//            full complex FFT in LDS (exp(+i k.r)), every mode of the cube:
//            rho = FFT * prod h / psihat, S = |rho|^2 / N, loss += W (S - S0)^2
//            (FP64), field coefficient C(n) = 4 W (S - S0) rho / N * prod h / psihat_i
//            (both n and -n are visited, no half-spectrum bookkeeping), inverse
//            FFT (exp(-i k.x)); the field is its real part;
//   interp   per work item: the configuration's field in LDS, derivative
//            interpolation at every point (cosh-form kernel of width w + 1).
// The chunk size and the workgroup size are picked by the autotuner.
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <type_traits>
#include <vector>

#include "common.h"
#include "fft_lds.h"
#include "kernels.h"
#include "lbfgs.h"
#include "plan.h"

namespace fresco {

constexpr int kBatchMaxB = 4;  // butterflies per thread per stage
constexpr int kChunkMin = 2048;
constexpr int kChunks[5] = {2048, 4096, 8192, 16384, 32768};

struct BatchTables {  // device memory, read with uniform loads
  FftFactors F[3];
};

struct BatchGeom {
  int d;
  int M[3];
  int P[3];   // 2 M + 1
  int nf[3];  // fine grid (1 beyond d)
  int JT[3];  // threads per line of the FFT along each axis
  int w, wi;
  double beta, beta_i;
  double icb;  // 1 / cosh(beta_i), set with the plan (no FP64 cosh per thread)
  int ngrid, ncube, nb;
  int lds_tw;  // twiddle slots in LDS (largest nf)
};

struct BatchItem {
  long long off;  // first row of the configuration in the concatenated arrays
  long long n;
  double ufac[3];  // nf / L
  double gs[3];    // -(nf / L) (2 / w_i)
  double invN;
};

template <class R>
struct BatchPtrs {
  const BatchTables* tab;
  const BatchItem* items;
  const R* W;        // [nb][ncube] weights (relative normalisation applied)
  const R* S0;       // [nb][ncube]
  const R* dec[3];   // h / psihat_a(|n|), n = 0..M_a (spreading kernel)
  const R* deci[3];  // h / psihat_i,a(|n|) (interpolation kernel)
  const cpx<R>* tw[3];  // exp(+2 pi i q / nf_a)
  const R* pos;
  R* grad;
  double* loss;  // [nb]
  int* flag;     // non-finite position seen
};

__device__ __forceinline__ int wrap_index(int x, int n) {
  x += (x < 0) ? n : 0;
  x -= (x >= n) ? n : 0;
  return x;
}

// grid coordinate of one position: l0 = ceil(u - w/2), tau = l0 - u + w/2 (FP64)
__device__ __forceinline__ double grid_split(double x, double ufac, int nf, double hw, int* l0,
                                             bool* bad) {
  double u = x * ufac;
  if (!isfinite(u)) {
    *bad = true;
    u = 0.0;
  }
  const double nfd = (double)nf;
  if (!(u >= 0.0 && u < nfd)) {
    u = fmod(u, nfd);
    if (u < 0.0) u += nfd;
    if (u >= nfd) u = 0.0;
  }
  const double l = ceil(u - hw);
  *l0 = (int)l;
  return l - u + hw;
}

// Transform every line of the LDS grid along axis a (all threads call it).
template <class R, bool INV>
__device__ void batch_fft_axis(cpx<R>* buf, cpx<R>* tws, const cpx<R>* __restrict__ twg,
                               const FftFactors& F, const BatchGeom& g, int a) {
  const int n = F.n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) tws[i] = twg[i];
  __syncthreads();
  const int nlines = g.ngrid / n;
  const int JT = g.JT[a];
  const int LP = blockDim.x / JT;
  const int es = (a == 0) ? 1 : (a == 1 ? g.nf[0] : g.nf[0] * g.nf[1]);
  const int lb = threadIdx.x / JT, tj = threadIdx.x - (threadIdx.x / JT) * JT;
  for (int l0 = 0; l0 < nlines; l0 += LP) {
    const int line = l0 + lb;
    const bool active = lb < LP && line < nlines;
    int base = 0;
    if (active) {
      if (a == 0) {
        base = line * n;
      } else if (a == 1) {
        const int x = line % g.nf[0], z = line / g.nf[0];
        base = z * g.nf[0] * g.nf[1] + x;
      } else {
        base = line;
      }
    }
    lds_fft<R, kBatchMaxB, INV>(buf + base, F, tws, active, 0, 0, es, tj, JT);
  }
  __syncthreads();
}

// grid index of mode q of the cube (C order over n_0..n_{d-1}, n_{d-1} fastest)
template <int D>
__device__ __forceinline__ int mode_grid_index(const BatchGeom& g, int q, int* na) {
  int rem = q;
  for (int a = D - 1; a >= 0; --a) {
    na[a] = rem % g.P[a] - g.M[a];
    rem /= g.P[a];
  }
  int idx = 0, stride = 1;
  for (int a = 0; a < D; ++a) {
    idx += (na[a] < 0 ? na[a] + g.nf[a] : na[a]) * stride;
    stride *= g.nf[a];
  }
  return idx;
}

// work item: x = configuration, y = first point inside it, z = points
template <class R, int D, int W>
__global__ void __launch_bounds__(1024)
    batch_spread_kernel(BatchGeom g, BatchPtrs<R> p, const int4* __restrict__ work, int nwork,
                        R* __restrict__ part) {
  using U = typename std::conditional<sizeof(R) == 4, uint32_t, unsigned long long>::type;
  constexpr bool F32 = sizeof(R) == 4;
  extern __shared__ unsigned long long smem_u64[];
  U* acc = reinterpret_cast<U*>(smem_u64);
  uint32_t* tmp = reinterpret_cast<uint32_t*>(acc + g.ngrid);
  __shared__ double red[16];
  const int nf0 = g.nf[0], nf1 = g.nf[1], nf2 = g.nf[2];
  const R beta = (R)g.beta;
  const double hw = 0.5 * W;
  for (int it = blockIdx.x; it < nwork; it += gridDim.x) {
    const int4 wk = work[it];
    const BatchItem item = p.items[wk.x];
    const R* __restrict__ pos = p.pos + (item.off + wk.y) * D;
    const int n = wk.z;
    bool bad = false;
    // fixed-point scale: cnt = footprint starts per cell, its periodic w^d box sum
    // bounds the points covering one cell (each contributes at most 1)
    uint32_t* cnt = reinterpret_cast<uint32_t*>(acc);
    for (int i = threadIdx.x; i < g.ngrid; i += blockDim.x) cnt[i] = 0u;
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      int c = 0, stride = 1;
#pragma unroll
      for (int a = 0; a < D; ++a) {
        int l0;
        (void)grid_split((double)pos[(long long)j * D + a], item.ufac[a], g.nf[a], hw, &l0, &bad);
        c += wrap_index(l0, g.nf[a]) * stride;
        stride *= g.nf[a];
      }
      atomicAdd(cnt + c, 1u);
    }
    __syncthreads();
    uint32_t* src = cnt;
    uint32_t* dst = tmp;
    int stride = 1;
    for (int a = 0; a < D; ++a) {
      const int nfa = g.nf[a];
      for (int i = threadIdx.x; i < g.ngrid; i += blockDim.x) {
        const int xa = (i / stride) % nfa;
        uint32_t s = 0;
        for (int t = 0; t < W; ++t) s += src[i + (wrap_index(xa - t, nfa) - xa) * stride];
        dst[i] = s;
      }
      __syncthreads();
      uint32_t* sw = src;
      src = dst;
      dst = sw;
      stride *= nfa;
    }
    uint32_t mx = 0;
    for (int i = threadIdx.x; i < g.ngrid; i += blockDim.x) mx = max(mx, src[i]);
    for (int off = 32; off > 0; off >>= 1) mx = max(mx, (uint32_t)__shfl_down((int)mx, off, 64));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = (double)mx;
    __syncthreads();
    double cov = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) cov = fmax(cov, red[w]);
    __syncthreads();

    for (int i = threadIdx.x; i < g.ngrid; i += blockDim.x) acc[i] = (U)0;
    const int ex = fixed_exponent((long long)cov, F32 ? 31 : 63);
    const R scale = (R)ldexp(1.0, ex);
    const R inv_scale = (R)ldexp(1.0, -ex);
    __syncthreads();
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
      int l0[3] = {0, 0, 0};
      R tau[3] = {R(0), R(0), R(0)};
#pragma unroll
      for (int a = 0; a < D; ++a)
        tau[a] = (R)grid_split((double)pos[(long long)j * D + a], item.ufac[a], g.nf[a], hw,
                               &l0[a], &bad);
      R k0[W], k1[W], k2[W];
      spread_weights<R, W>(tau[0], beta, k0);
      spread_weights<R, W>(tau[1], beta, k1);
      if (D == 3) spread_weights<R, W>(tau[2], beta, k2);
      int xs[W];
#pragma unroll
      for (int dx = 0; dx < W; ++dx) xs[dx] = wrap_index(l0[0] + dx, nf0);
      const int zmax = (D == 3) ? W : 1;
      for (int dz = 0; dz < zmax; ++dz) {
        const R pz = (D == 3) ? k2[dz] * scale : scale;
        const int z = (D == 3) ? wrap_index(l0[2] + dz, nf2) : 0;
#pragma unroll
        for (int dy = 0; dy < W; ++dy) {
          const R py = k1[dy] * pz;
          U* row = acc + (z * nf1 + wrap_index(l0[1] + dy, nf1)) * nf0;
#pragma unroll
          for (int dx = 0; dx < W; ++dx) {
            U q;
            if (F32) q = (U)__float2uint_rn((float)(py * k0[dx]));
            else q = (U)((double)(py * k0[dx]) + 0.5);
            if (q) atomicAdd(row + xs[dx], q);
          }
        }
      }
    }
    if (bad) atomicOr(p.flag, 1);
    __syncthreads();
    R* __restrict__ out = part + (long long)it * g.ngrid;
    for (int i = threadIdx.x; i < g.ngrid; i += blockDim.x) out[i] = (R)acc[i] * inv_scale;
    __syncthreads();  // LDS is reused by the next item
  }
}

// citems[b] = (first work item of configuration b, its number of items)
template <class R, int D>
__global__ void __launch_bounds__(1024)
    batch_modes_kernel(BatchGeom g, BatchPtrs<R> p, const int2* __restrict__ citems,
                       const R* __restrict__ part, R* __restrict__ field) {
  extern __shared__ unsigned long long smem_u64[];
  cpx<R>* tws = reinterpret_cast<cpx<R>*>(smem_u64);
  cpx<R>* buf = tws + g.lds_tw;
  cpx<R>* coef = buf + g.ngrid;
  __shared__ double red[16];
  for (int b = blockIdx.x; b < g.nb; b += gridDim.x) {
    const int2 ci = citems[b];
    const BatchItem item = p.items[b];
    for (int i = threadIdx.x; i < g.ngrid; i += blockDim.x) {
      R s = R(0);
      for (int c = 0; c < ci.y; ++c) s += part[(long long)(ci.x + c) * g.ngrid + i];
      buf[i] = cpx<R>{s, R(0)};
    }
    __syncthreads();
    for (int a = 0; a < D; ++a) batch_fft_axis<R, false>(buf, tws, p.tw[a], p.tab->F[a], g, a);
    double lsum = 0.0;
    const R* __restrict__ Wb = p.W + (long long)b * g.ncube;
    const R* __restrict__ S0b = p.S0 + (long long)b * g.ncube;
    for (int q = threadIdx.x; q < g.ncube; q += blockDim.x) {
      int na[3] = {0, 0, 0};
      const int idx = mode_grid_index<D>(g, q, na);
      R dec = R(1), deci = R(1);
      for (int a = 0; a < D; ++a) {
        const int an = na[a] < 0 ? -na[a] : na[a];
        dec *= p.dec[a][an];
        deci *= p.deci[a][an];
      }
      const cpx<R> rho = cscale(buf[idx], dec);
      const R S = (rho.x * rho.x + rho.y * rho.y) * (R)item.invN;
      const R Wq = Wb[q];
      const R res = S - S0b[q];
      lsum += (double)Wq * (double)res * (double)res;
      coef[q] = cscale(rho, R(4) * Wq * res * (R)item.invN * deci);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < g.ngrid; i += blockDim.x) buf[i] = cpx<R>{R(0), R(0)};
    __syncthreads();
    for (int q = threadIdx.x; q < g.ncube; q += blockDim.x) {
      int na[3];
      buf[mode_grid_index<D>(g, q, na)] = coef[q];
    }
    __syncthreads();
    for (int a = 0; a < D; ++a) batch_fft_axis<R, true>(buf, tws, p.tw[a], p.tab->F[a], g, a);
    R* __restrict__ out = field + (long long)b * g.ngrid;
    for (int i = threadIdx.x; i < g.ngrid; i += blockDim.x) out[i] = buf[i].x;
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_down(lsum, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lsum;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) t += red[w];
      p.loss[b] = t;
    }
    __syncthreads();  // LDS is reused by the next configuration
  }
}

template <class R, int D, int W>
__global__ void __launch_bounds__(1024)
    batch_interp_kernel(BatchGeom g, BatchPtrs<R> p, const int4* __restrict__ work, int nwork,
                        const R* __restrict__ field) {
  constexpr int WI = W + 1;
  extern __shared__ unsigned long long smem_u64[];
  R* fl = reinterpret_cast<R*>(smem_u64);
  const int nf0 = g.nf[0], nf1 = g.nf[1], nf2 = g.nf[2];
  const R beta_i = (R)g.beta_i;
  const R icb = (R)g.icb;
  const double hw = 0.5 * W;
  for (int it = blockIdx.x; it < nwork; it += gridDim.x) {
    const int4 wk = work[it];
    const BatchItem item = p.items[wk.x];
    const R* __restrict__ src = field + (long long)wk.x * g.ngrid;
    for (int i = threadIdx.x; i < g.ngrid; i += blockDim.x) fl[i] = src[i];
    __syncthreads();
    const R* __restrict__ pos = p.pos + (item.off + wk.y) * D;
    R* __restrict__ grad = p.grad + (item.off + wk.y) * D;
    bool bad = false;
    for (int j = threadIdx.x; j < wk.z; j += blockDim.x) {
      int s[3] = {0, 0, 0};
      R f0[WI], d0[WI], f1[WI], d1[WI], f2[WI], d2[WI];
#pragma unroll
      for (int a = 0; a < D; ++a) {
        int l0;
        const R t = (R)grid_split((double)pos[(long long)j * D + a], item.ufac[a], g.nf[a], hw,
                                  &l0, &bad);
        const int k = (t >= R(0.5)) ? 1 : 0;
        const R ti = k ? t - R(0.5) : t + R(0.5);
        s[a] = l0 - k;
        if (a == 0) interp_weights<R, WI>(ti, beta_i, icb, f0, d0);
        else if (a == 1) interp_weights<R, WI>(ti, beta_i, icb, f1, d1);
        else interp_weights<R, WI>(ti, beta_i, icb, f2, d2);
      }
      int xs[WI];
#pragma unroll
      for (int dx = 0; dx < WI; ++dx) xs[dx] = wrap_index(s[0] + dx, nf0);
      R gx = R(0), gy = R(0), gz = R(0);
      const int zmax = (D == 3) ? WI : 1;
      for (int dz = 0; dz < zmax; ++dz) {
        const int z = (D == 3) ? wrap_index(s[2] + dz, nf2) : 0;
        R sxy = R(0), sdxy = R(0), sxdy = R(0);
#pragma unroll
        for (int dy = 0; dy < WI; ++dy) {
          const R* row = fl + (z * nf1 + wrap_index(s[1] + dy, nf1)) * nf0;
          R sx = R(0), sdx = R(0);
#pragma unroll
          for (int dx = 0; dx < WI; ++dx) {
            const R vv = row[xs[dx]];
            sx += vv * f0[dx];
            sdx += vv * d0[dx];
          }
          sxy += sx * f1[dy];
          sdxy += sdx * f1[dy];
          sxdy += sx * d1[dy];
        }
        if (D == 3) {
          gx += sdxy * f2[dz];
          gy += sxdy * f2[dz];
          gz += sxy * d2[dz];
        } else {
          gx = sdxy;
          gy = sxdy;
        }
      }
      grad[(long long)j * D] = gx * (R)item.gs[0];
      grad[(long long)j * D + 1] = gy * (R)item.gs[1];
      if (D == 3) grad[(long long)j * D + 2] = gz * (R)item.gs[2];
    }
    __syncthreads();  // LDS is reused by the next item
  }
}

// total = sum of the per-configuration losses (fixed order); flag handed over
__global__ void batch_total_kernel(const double* __restrict__ loss, int nb, double* __restrict__ out,
                                   int* __restrict__ flag, int* __restrict__ flag_out) {
  __shared__ double s[256];
  double v = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) v += loss[i];
  s[threadIdx.x] = v;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    if (out) out[0] = s[0];
    flag_out[0] = flag[0];
    flag[0] = 0;
  }
}

}  // namespace fresco

using namespace fresco;

struct fresco_batch_ctx {
  int dtype = 0;
  BatchGeom g{};
  hipStream_t st = nullptr;
  long long ntot = 0;
  std::vector<long long> off;  // nb + 1
  std::vector<long long> npts;  // points per configuration
  std::vector<void*> allocs;
  long long bytes = 0;
  size_t lds_spread = 0, lds_modes = 0, lds_interp = 0;
  int threads = 1024;  // workgroup size of the spread and interp passes
  int chunk = 8192;    // points per work item
  int nwork = 0;
  BatchTables* tab = nullptr;
  BatchItem* items = nullptr;
  int4* work = nullptr;    // [max items]
  int2* citems = nullptr;  // [nb]
  void* part = nullptr;    // [max items][ngrid] partial grids
  void* field = nullptr;   // [nb][ngrid]
  void* W = nullptr;
  void* S0 = nullptr;
  void* dec[3] = {nullptr, nullptr, nullptr};
  void* deci[3] = {nullptr, nullptr, nullptr};
  void* tw[3] = {nullptr, nullptr, nullptr};
  double* loss = nullptr;   // [nb]
  double* total = nullptr;  // [1]
  int* flag = nullptr;
  int* flag_out = nullptr;
  double* host = nullptr;   // pinned [nb + 1] doubles, then the flag
  // L-BFGS over the concatenated batch
  void* lv = nullptr;       // LbfgsVec<R>
  LbfgsState* lst = nullptr;
  LbfgsState* lst_host = nullptr;  // pinned [2] (one per chunk in flight)
  hipEvent_t lb_ev[2] = {nullptr, nullptr};
  int lb_m = 0;
  bool lb_fresh = true;
  LbfgsOpts lb_opts{};
  hipGraphExec_t lb_graph = nullptr;
  bool use_graphs = true;
};

namespace {

int g_batch_hip = 0;

#define BHIP(x)                  \
  do {                           \
    hipError_t e_ = (x);         \
    if (e_ != hipSuccess) {      \
      g_batch_hip = (int)e_;     \
      return FRESCO_EHIP;        \
    }                            \
  } while (0)

template <class T>
int balloc(fresco_batch_ctx* c, T** p, size_t count) {
  void* q = nullptr;
  const size_t bytes = sizeof(T) * (count ? count : 1);
  if (hipMalloc(&q, bytes) != hipSuccess) return FRESCO_ENOMEM;
  c->allocs.push_back(q);
  c->bytes += (long long)bytes;
  *p = (T*)q;
  return FRESCO_OK;
}

template <class T>
int bupload(fresco_batch_ctx* c, T** p, const std::vector<T>& h) {
  int st = balloc(c, p, h.size());
  if (st) return st;
  BHIP(hipMemcpy(*p, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice));
  return FRESCO_OK;
}

template <class R>
int upload_as(fresco_batch_ctx* c, void** p, const std::vector<double>& h) {
  std::vector<R> v(h.begin(), h.end());
  R* q = nullptr;
  int st = bupload(c, &q, v);
  *p = q;
  return st;
}

#define BATCH_W_SWITCH(W_, CALL) \
  switch (W_) {                  \
    case 2: CALL(2); break;      \
    case 3: CALL(3); break;      \
    case 4: CALL(4); break;      \
    case 5: CALL(5); break;      \
    case 6: CALL(6); break;      \
    case 7: CALL(7); break;      \
    case 8: CALL(8); break;      \
    case 9: CALL(9); break;      \
    case 10: CALL(10); break;    \
    case 11: CALL(11); break;    \
    case 12: CALL(12); break;    \
    case 13: CALL(13); break;    \
    case 14: CALL(14); break;    \
    case 15: CALL(15); break;    \
    case 16: CALL(16); break;    \
  }

long long max_work_items(const fresco_batch_ctx* c) {
  long long m = 0;
  for (long long n : c->npts) m += (n + kChunkMin - 1) / kChunkMin;
  return m;
}

// work items of at most `chunk` points, configuration by configuration
int plan_work(fresco_batch_ctx* c, int chunk) {
  const int nb = c->g.nb;
  std::vector<int4> work;
  std::vector<int2> citems(nb);
  for (int b = 0; b < nb; ++b) {
    citems[b].x = (int)work.size();
    for (long long j = 0; j < c->npts[b]; j += chunk) {
      const long long cnt = std::min<long long>(chunk, c->npts[b] - j);
      work.push_back(make_int4(b, (int)j, (int)cnt, 0));
    }
    citems[b].y = (int)work.size() - citems[b].x;
  }
  BHIP(hipMemcpy(c->work, work.data(), sizeof(int4) * work.size(), hipMemcpyHostToDevice));
  BHIP(hipMemcpy(c->citems, citems.data(), sizeof(int2) * nb, hipMemcpyHostToDevice));
  c->chunk = chunk;
  c->nwork = (int)work.size();
  return FRESCO_OK;
}

template <class R>
BatchPtrs<R> batch_ptrs(fresco_batch_ctx* c, const void* pos, void* grad) {
  BatchPtrs<R> p;
  p.tab = c->tab;
  p.items = c->items;
  p.W = (const R*)c->W;
  p.S0 = (const R*)c->S0;
  for (int a = 0; a < 3; ++a) {
    p.dec[a] = (const R*)c->dec[a];
    p.deci[a] = (const R*)c->deci[a];
    p.tw[a] = (const cpx<R>*)c->tw[a];
  }
  p.pos = (const R*)pos;
  p.grad = (R*)grad;
  p.loss = c->loss;
  p.flag = c->flag;
  return p;
}

template <class R>
int batch_enqueue(fresco_batch_ctx* c, const void* pos, void* grad, double* total) {
  const BatchGeom& g = c->g;
  BatchPtrs<R> p = batch_ptrs<R>(c, pos, grad);
  const unsigned wgrid = (unsigned)std::min(c->nwork, 4096);
  R* part = (R*)c->part;
  R* field = (R*)c->field;
#define BL(W)                                                                                  \
  do {                                                                                         \
    if (g.d == 2)                                                                              \
      batch_spread_kernel<R, 2, W><<<wgrid, c->threads, c->lds_spread, c->st>>>(               \
          g, p, c->work, c->nwork, part);                                                      \
    else                                                                                       \
      batch_spread_kernel<R, 3, W><<<wgrid, c->threads, c->lds_spread, c->st>>>(               \
          g, p, c->work, c->nwork, part);                                                      \
  } while (0)
  BATCH_W_SWITCH(g.w, BL)
#undef BL
  if (g.d == 2)
    batch_modes_kernel<R, 2><<<g.nb, 1024, c->lds_modes, c->st>>>(g, p, c->citems, part, field);
  else
    batch_modes_kernel<R, 3><<<g.nb, 1024, c->lds_modes, c->st>>>(g, p, c->citems, part, field);
#define BI(W)                                                                                  \
  do {                                                                                         \
    if (g.d == 2)                                                                              \
      batch_interp_kernel<R, 2, W><<<wgrid, c->threads, c->lds_interp, c->st>>>(               \
          g, p, c->work, c->nwork, field);                                                     \
    else                                                                                       \
      batch_interp_kernel<R, 3, W><<<wgrid, c->threads, c->lds_interp, c->st>>>(               \
          g, p, c->work, c->nwork, field);                                                     \
  } while (0)
  BATCH_W_SWITCH(g.w, BI)
#undef BI
  batch_total_kernel<<<1, 256, 0, c->st>>>(c->loss, g.nb, total, c->flag, c->flag_out);
  BHIP(hipGetLastError());
  return FRESCO_OK;
}

int batch_enqueue_any(fresco_batch_ctx* c, const void* pos, void* grad, double* total) {
  if (c->dtype == FRESCO_F32) return batch_enqueue<float>(c, pos, grad, total);
  return batch_enqueue<double>(c, pos, grad, total);
}

template <class R>
hipError_t batch_prepare(fresco_batch_ctx* c) {
  const BatchGeom& g = c->g;
  hipError_t e = hipSuccess;
#define BP(W)                                                                                    \
  do {                                                                                           \
    const void* ks = (g.d == 2) ? (const void*)batch_spread_kernel<R, 2, W>                      \
                                : (const void*)batch_spread_kernel<R, 3, W>;                     \
    const void* ki = (g.d == 2) ? (const void*)batch_interp_kernel<R, 2, W>                      \
                                : (const void*)batch_interp_kernel<R, 3, W>;                     \
    e = hipFuncSetAttribute(ks, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds_spread); \
    if (e == hipSuccess)                                                                         \
      e = hipFuncSetAttribute(ki, hipFuncAttributeMaxDynamicSharedMemorySize,                    \
                              (int)c->lds_interp);                                               \
  } while (0)
  BATCH_W_SWITCH(g.w, BP)
#undef BP
  if (e != hipSuccess) return e;
  const void* km = (g.d == 2) ? (const void*)batch_modes_kernel<R, 2>
                              : (const void*)batch_modes_kernel<R, 3>;
  return hipFuncSetAttribute(km, hipFuncAttributeMaxDynamicSharedMemorySize, (int)c->lds_modes);
}

template <class R>
int batch_build(fresco_batch_ctx* c, int nb, const fresco_problem* ps) {
  BatchGeom& g = c->g;
  const int d = g.d;
  // shared tables: FFT plans
  BatchTables tab;
  std::memset(&tab, 0, sizeof(tab));
  int st;
  for (int a = 0; a < d; ++a) {
    int rmin = 1;
    if (!plan_factors(g.nf[a], &tab.F[a], &rmin)) return FRESCO_ENOTSUP;
    const int nr = g.nf[a] / (rmin > 0 ? rmin : 1);
    g.JT[a] = (nr + kBatchMaxB - 1) / kBatchMaxB;
    if (g.JT[a] > 256) return FRESCO_ENOTSUP;
    std::vector<double> t = twiddles(g.nf[a], g.nf[a]);
    if ((st = upload_as<R>(c, &c->tw[a], t))) return st;
    const double h = 2.0 * M_PI / g.nf[a];
    std::vector<double> ph = kernel_fourier(g.M[a], g.w, g.beta, g.nf[a], false);
    for (auto& x : ph) x = h / x;
    if ((st = upload_as<R>(c, &c->dec[a], ph))) return st;
    std::vector<double> pi = kernel_fourier(g.M[a], g.wi, g.beta_i, g.nf[a], true);
    for (auto& x : pi) x = h / x;
    if ((st = upload_as<R>(c, &c->deci[a], pi))) return st;
  }
  {
    std::vector<BatchTables> v(1, tab);
    if ((st = bupload(c, &c->tab, v))) return st;
  }
  // per-configuration items, targets and weights
  std::vector<BatchItem> items(nb);
  std::vector<double> Wall((size_t)nb * g.ncube), S0all((size_t)nb * g.ncube);
  for (int b = 0; b < nb; ++b) {
    const fresco_problem& p = ps[b];
    BatchItem& it = items[b];
    std::memset(&it, 0, sizeof(it));
    it.off = c->off[b];
    it.n = p.n;
    it.invN = 1.0 / (double)p.n;
    for (int a = 0; a < 3; ++a) {
      if (a < d) {
        it.ufac[a] = (double)g.nf[a] / p.box[a];
        it.gs[a] = -(double)g.nf[a] / p.box[a] * 2.0 / g.wi;
      }
    }
    for (long long i = 0; i < g.ncube; ++i) {
      long long r = i, n2 = 0;
      bool zero = true;
      for (int a = d - 1; a >= 0; --a) {
        const long long na = r % g.P[a] - g.M[a];
        r /= g.P[a];
        n2 += na * na;
        if (na != 0) zero = false;
      }
      const double s0 = p.s0 ? p.s0[i] : 0.0;
      double w = p.w ? p.w[i] : ((n2 > 0 && (double)n2 <= p.k_cut * p.k_cut) ? 1.0 : 0.0);
      if (!(w >= 0.0) || !std::isfinite(w) || !std::isfinite(s0)) return FRESCO_EINVAL;
      if (zero) w = 0.0;
      double W = w;
      if (p.weight_mode == FRESCO_WEIGHT_RELATIVE && s0 != 0.0) W = w / (s0 * s0);
      Wall[(size_t)b * g.ncube + i] = W;
      S0all[(size_t)b * g.ncube + i] = s0;
    }
  }
  if ((st = bupload(c, &c->items, items))) return st;
  if ((st = upload_as<R>(c, &c->W, Wall))) return st;
  if ((st = upload_as<R>(c, &c->S0, S0all))) return st;
  if ((st = balloc(c, &c->loss, nb))) return st;
  if ((st = balloc(c, &c->total, 1))) return st;
  if ((st = balloc(c, &c->flag, 1))) return st;
  if ((st = balloc(c, &c->flag_out, 1))) return st;
  BHIP(hipMemset(c->flag, 0, sizeof(int)));
  BHIP(hipMemset(c->flag_out, 0, sizeof(int)));
  // work items (room for the smallest chunk size), partial grids, fields
  const long long maxw = max_work_items(c);
  if ((st = balloc(c, &c->work, (size_t)maxw))) return st;
  if ((st = balloc(c, &c->citems, (size_t)nb))) return st;
  R* part = nullptr;
  if ((st = balloc(c, &part, (size_t)maxw * g.ngrid))) return st;
  c->part = part;
  R* field = nullptr;
  if ((st = balloc(c, &field, (size_t)nb * g.ngrid))) return st;
  c->field = field;
  if ((st = plan_work(c, 8192))) return st;
  // LDS of the three passes
  using U = typename std::conditional<sizeof(R) == 4, uint32_t, unsigned long long>::type;
  const size_t cs = sizeof(cpx<R>);
  c->lds_spread = (size_t)g.ngrid * (sizeof(U) + sizeof(uint32_t));
  c->lds_modes = ((size_t)g.lds_tw + g.ngrid + g.ncube) * cs;
  c->lds_interp = (size_t)g.ngrid * sizeof(R);
  const size_t lim = 160 * 1024 - 256;
  if (c->lds_spread > lim || c->lds_modes > lim || c->lds_interp > lim) return FRESCO_ENOTSUP;
  BHIP(batch_prepare<R>(c));
  return FRESCO_OK;
}

// ------------------------------------------------------------------ L-BFGS
template <class R>
int batch_lbfgs_setup(fresco_batch_ctx* c, int m) {
  if (c->lv && c->lb_m == m) return FRESCO_OK;
  if (c->lb_graph) {
    (void)hipGraphExecDestroy(c->lb_graph);
    c->lb_graph = nullptr;
  }
  if (!c->lv) c->lv = new (std::nothrow) LbfgsVec<R>();
  if (!c->lv) return FRESCO_ENOMEM;
  LbfgsVec<R>& v = *(LbfgsVec<R>*)c->lv;
  const long long n = c->ntot * c->g.d;
  int st;
  if ((st = balloc(c, &v.x, n))) return st;
  if ((st = balloc(c, &v.g, n))) return st;
  if ((st = balloc(c, &v.p, n))) return st;
  if ((st = balloc(c, &v.xt, n))) return st;
  if ((st = balloc(c, &v.gt, n))) return st;
  const long long ld = lbfgs_slot_stride(n);
  if ((st = balloc(c, &v.S, (size_t)ld * m))) return st;
  if ((st = balloc(c, &v.Y, (size_t)ld * m))) return st;
  const int nb = lbfgs_blocks(n);
  v.nb = nb;
  v.n = n;
  v.ld = ld;
  v.m = m;
  if ((st = balloc(c, &v.part0, (4 * (size_t)kLbfgsMaxM + 1) * nb))) return st;
  if ((st = balloc(c, &v.part1, (size_t)nb))) return st;
  if (!c->lst && (st = balloc(c, &c->lst, 2))) return st;  // the state and pass A's snapshot
  if (!c->lst_host) BHIP(hipHostMalloc((void**)&c->lst_host, 2 * sizeof(LbfgsState)));
  for (int i = 0; i < 2; ++i)
    if (!c->lb_ev[i]) BHIP(hipEventCreateWithFlags(&c->lb_ev[i], hipEventDisableTiming));
  c->lb_m = m;
  c->lb_fresh = true;
  return FRESCO_OK;
}

template <class R>
int batch_trial(fresco_batch_ctx* c) {
  LbfgsVec<R>& v = *(LbfgsVec<R>*)c->lv;
  int st = batch_enqueue<R>(c, v.xt, v.gt, &c->lst->f_trial);
  if (st) return st;
  launch_lbfgs_update<R>(v, c->lst, c->lb_opts, c->st);
  BHIP(hipGetLastError());
  return FRESCO_OK;
}

template <class R>
int batch_step_impl(fresco_batch_ctx* c, void* pos, const fresco_lbfgs_opts* o, int n_iter,
                    double* loss_out, int32_t* n_eval_out) {
  int st;
  if ((st = batch_lbfgs_setup<R>(c, o->m))) return st;
  LbfgsOpts lo;
  lo.m = o->m;
  lo.max_backtracks = o->max_backtracks;
  lo.max_step = o->max_step;
  lo.c1 = o->c1;
  lo.shrink = o->shrink;
  lo.gtol = o->gtol;
  if (std::memcmp(&lo, &c->lb_opts, sizeof(lo)) != 0 && c->lb_graph) {
    (void)hipGraphExecDestroy(c->lb_graph);
    c->lb_graph = nullptr;
  }
  c->lb_opts = lo;
  LbfgsVec<R>& v = *(LbfgsVec<R>*)c->lv;
  const size_t vbytes = sizeof(R) * (size_t)v.n;
  if (c->lb_fresh) {
    LbfgsState h;
    std::memset(&h, 0, sizeof(h));
    h.head = c->lb_m - 1;
    h.gamma = 1.0;
    BHIP(hipMemcpyAsync(c->lst, &h, sizeof(h), hipMemcpyHostToDevice, c->st));
    BHIP(hipStreamSynchronize(c->st));
    c->lb_fresh = false;
  }
  BHIP(hipMemcpyAsync(v.x, pos, vbytes, hipMemcpyDeviceToDevice, c->st));
  BHIP(hipMemcpyAsync(v.xt, pos, vbytes, hipMemcpyDeviceToDevice, c->st));
  launch_lbfgs_set_mode(c->lst, 4, n_iter, c->st);
  if ((st = batch_trial<R>(c))) return st;
  launch_lbfgs_set_mode(c->lst, 0, -1, c->st);
  const bool graphs = c->use_graphs && c->st != nullptr;
  if (graphs && !c->lb_graph) {
    hipGraph_t graph = nullptr;
    BHIP(hipStreamBeginCapture(c->st, hipStreamCaptureModeThreadLocal));
    st = batch_trial<R>(c);
    hipError_t e = hipStreamEndCapture(c->st, &graph);
    if (st) {
      if (graph) (void)hipGraphDestroy(graph);
      return st;
    }
    BHIP(e);
    e = hipGraphInstantiate(&c->lb_graph, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    BHIP(e);
  }
  auto replay = [&](int count) -> int {
    for (int r = 0; r < count; ++r) {
      if (graphs) {
        BHIP(hipGraphLaunch(c->lb_graph, c->st));
      } else {
        const int s2 = batch_trial<R>(c);
        if (s2) return s2;
      }
    }
    return FRESCO_OK;
  };
  st = lbfgs_replay_until_stop(c->st, c->lst, c->lst_host, c->lb_ev, n_iter, kLbfgsReplayChunk,
                               replay, &g_batch_hip);
  if (st) return st;
  BHIP(hipMemcpyAsync(pos, v.x, vbytes, hipMemcpyDeviceToDevice, c->st));
  BHIP(hipMemcpyAsync(c->lst_host, c->lst, sizeof(LbfgsState), hipMemcpyDeviceToHost, c->st));
  BHIP(hipStreamSynchronize(c->st));
  const LbfgsState& h = *c->lst_host;
  if (loss_out) *loss_out = h.f_cur;
  if (n_eval_out) *n_eval_out = h.nevals;
  if (h.fail) return FRESCO_ELINESEARCH;
  return FRESCO_OK;
}

}  // namespace

extern "C" {

int fresco_batch_destroy(fresco_batch_ctx* c) {
  if (!c) return FRESCO_OK;
  (void)hipStreamSynchronize(c->st);
  if (c->lb_graph) (void)hipGraphExecDestroy(c->lb_graph);
  for (void* p : c->allocs) (void)hipFree(p);
  if (c->host) (void)hipHostFree(c->host);
  if (c->lst_host) (void)hipHostFree(c->lst_host);
  for (hipEvent_t e : c->lb_ev)
    if (e) (void)hipEventDestroy(e);
  if (c->lv) {
    if (c->dtype == FRESCO_F32) delete (LbfgsVec<float>*)c->lv;
    else delete (LbfgsVec<double>*)c->lv;
  }
  delete c;
  return FRESCO_OK;
}

int fresco_batch_create(fresco_batch_ctx** out, int32_t nb, const fresco_problem* ps,
                        void* stream) {
  if (!out) return FRESCO_EINVAL;
  *out = nullptr;
  if (!ps || nb < 1) return FRESCO_EINVAL;
  const fresco_problem& p0 = ps[0];
  const int d = p0.dim;
  if (d != 2 && d != 3) return FRESCO_EINVAL;
  if (p0.dtype != FRESCO_F32 && p0.dtype != FRESCO_F64) return FRESCO_EINVAL;
  if (!(p0.tol > 0.0 && p0.tol <= 0.1) || p0.upsampfac != 2.0) return FRESCO_EINVAL;
  long long ntot = 0;
  for (int b = 0; b < nb; ++b) {
    const fresco_problem& p = ps[b];
    if (p.dim != d || p.dtype != p0.dtype || p.tol != p0.tol || p.upsampfac != p0.upsampfac)
      return FRESCO_EINVAL;
    if (p.n < 1) return FRESCO_EINVAL;
    if (p.weight_mode != FRESCO_WEIGHT_ABS && p.weight_mode != FRESCO_WEIGHT_RELATIVE)
      return FRESCO_EINVAL;
    if (!p.w && !(p.k_cut >= 0.0)) return FRESCO_EINVAL;
    for (int a = 0; a < d; ++a) {
      if (p.kmax[a] != p0.kmax[a] || p.kmax[a] < 0) return FRESCO_EINVAL;
      if (!(p.box[a] > 0.0) || !std::isfinite(p.box[a])) return FRESCO_EINVAL;
    }
    ntot += p.n;
  }
  if (ntot > 2147483647LL) return FRESCO_ENOTSUP;
  fresco_batch_ctx* c = new (std::nothrow) fresco_batch_ctx();
  if (!c) return FRESCO_ENOMEM;
  c->dtype = p0.dtype;
  c->st = (hipStream_t)stream;
  const char* eg = std::getenv("FRESCO_GRAPHS");
  c->use_graphs = !(eg && eg[0] == '0');
  BatchGeom& g = c->g;
  g.d = d;
  g.nb = nb;
  g.w = kernel_width(p0.tol);
  g.beta = kernel_beta(g.w);
  g.wi = g.w + 1;
  g.beta_i = kernel_beta(g.wi);
  g.icb = 1.0 / std::cosh(g.beta_i);
  g.ngrid = 1;
  g.ncube = 1;
  g.lds_tw = 1;
  for (int a = 0; a < 3; ++a) {
    if (a < d) {
      g.M[a] = p0.kmax[a];
      g.P[a] = 2 * g.M[a] + 1;
      long long need = 2LL * g.P[a];
      if (need < 2LL * g.wi) need = 2LL * g.wi;
      if (need > 4096) {
        delete c;
        return FRESCO_ENOTSUP;
      }
      g.nf[a] = next_smooth_even(need);
      g.ngrid *= g.nf[a];
      g.ncube *= g.P[a];
      if (g.nf[a] > g.lds_tw) g.lds_tw = g.nf[a];
    } else {
      g.M[a] = 0;
      g.P[a] = 1;
      g.nf[a] = 1;
      g.JT[a] = 1;
    }
  }
  c->off.assign(nb + 1, 0);
  c->npts.assign(nb, 0);
  for (int b = 0; b < nb; ++b) {
    c->off[b + 1] = c->off[b] + ps[b].n;
    c->npts[b] = ps[b].n;
  }
  c->ntot = ntot;
  int st = (c->dtype == FRESCO_F32) ? batch_build<float>(c, nb, ps) : batch_build<double>(c, nb, ps);
  if (!st && hipHostMalloc((void**)&c->host, sizeof(double) * (nb + 2)) != hipSuccess)
    st = FRESCO_ENOMEM;
  if (st) {
    fresco_batch_destroy(c);
    return st;
  }
  *out = c;
  return FRESCO_OK;
}

int fresco_batch_offsets(const fresco_batch_ctx* c, int64_t* offsets) {
  if (!c || !offsets) return FRESCO_EINVAL;
  for (size_t b = 0; b < c->off.size(); ++b) offsets[b] = c->off[b];
  return FRESCO_OK;
}

int fresco_batch_loss_grad_async(fresco_batch_ctx* c, const void* pos, double* losses_dev,
                                 void* grad) {
  if (!c || !pos || !grad) return FRESCO_EINVAL;
  int st = batch_enqueue_any(c, pos, grad, c->total);
  if (st) return st;
  if (losses_dev)
    BHIP(hipMemcpyAsync(losses_dev, c->loss, sizeof(double) * c->g.nb, hipMemcpyDeviceToDevice,
                        c->st));
  return FRESCO_OK;
}

int fresco_batch_loss_grad(fresco_batch_ctx* c, const void* pos, double* losses, void* grad) {
  if (!c || !pos || !grad) return FRESCO_EINVAL;
  int st = batch_enqueue_any(c, pos, grad, c->total);
  if (st) return st;
  const int nb = c->g.nb;
  BHIP(hipMemcpyAsync(c->host, c->loss, sizeof(double) * nb, hipMemcpyDeviceToHost, c->st));
  BHIP(hipMemcpyAsync(c->host + nb, c->flag_out, sizeof(int), hipMemcpyDeviceToHost, c->st));
  BHIP(hipStreamSynchronize(c->st));
  if (losses)
    for (int b = 0; b < nb; ++b) losses[b] = c->host[b];
  if (*reinterpret_cast<int*>(c->host + nb)) return FRESCO_ENONFINITE;
  return FRESCO_OK;
}

int fresco_batch_step(fresco_batch_ctx* c, void* pos, const fresco_lbfgs_opts* o, int32_t n_iter,
                      double* loss_out, int32_t* n_eval_out) {
  if (!c || !pos || !o || n_iter < 0) return FRESCO_EINVAL;
  if (o->m < 1 || o->m > kLbfgsMaxM || o->max_backtracks < 0) return FRESCO_EINVAL;
  if (!(o->max_step > 0.0) || !(o->c1 > 0.0 && o->c1 < 1.0) ||
      !(o->shrink > 0.0 && o->shrink < 1.0) || !(o->gtol >= 0.0))
    return FRESCO_EINVAL;
  if (c->dtype == FRESCO_F32) return batch_step_impl<float>(c, pos, o, n_iter, loss_out, n_eval_out);
  return batch_step_impl<double>(c, pos, o, n_iter, loss_out, n_eval_out);
}

int fresco_batch_reset_history(fresco_batch_ctx* c) {
  if (!c) return FRESCO_EINVAL;
  c->lb_fresh = true;
  return FRESCO_OK;
}

int fresco_batch_autotune(fresco_batch_ctx* c, const void* pos, void* grad, int32_t reps,
                          int32_t* threads_out) {
  if (!c || !pos || !grad || reps < 1) return FRESCO_EINVAL;
  const int cand_t[3] = {256, 512, 1024};
  hipEvent_t e0, e1;
  BHIP(hipEventCreate(&e0));
  BHIP(hipEventCreate(&e1));
  float best_ms = 0.f;
  int best_t = c->threads, best_c = c->chunk;
  int st = FRESCO_OK;
  for (int ch : kChunks) {
    if ((st = plan_work(c, ch))) break;
    for (int t : cand_t) {
      c->threads = t;
      if ((st = batch_enqueue_any(c, pos, grad, c->total))) break;  // warm
      if (hipEventRecord(e0, c->st) != hipSuccess) {
        st = FRESCO_EHIP;
        break;
      }
      for (int r = 0; r < reps && !st; ++r) st = batch_enqueue_any(c, pos, grad, c->total);
      if (st) break;
      if (hipEventRecord(e1, c->st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess) {
        st = FRESCO_EHIP;
        break;
      }
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (best_ms == 0.f || ms < best_ms) {
        best_ms = ms;
        best_t = t;
        best_c = ch;
      }
    }
    if (st) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  c->threads = best_t;
  const int st2 = plan_work(c, best_c);
  if (!st) st = st2;
  if (c->lb_graph) {  // captured with the previous launch shape
    (void)hipGraphExecDestroy(c->lb_graph);
    c->lb_graph = nullptr;
  }
  if (threads_out) *threads_out = best_t;
  return st;
}

int fresco_batch_last_hip_error(void) { return g_batch_hip; }

}  // extern "C"
