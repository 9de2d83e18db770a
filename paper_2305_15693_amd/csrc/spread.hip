// Point binning, spreading (type-1, first step) and interpolation (type-2,
// last step) for gfx950.
//
// Kernel: the exponential of semicircle  phi(z) = exp(beta (sqrt(1 - z^2) - 1))
// on |z| <= 1 (Barnett, Magland & af Klinteberg, the kernel of the FINUFFT
// library the paper's Methods use), scaled so that its support spans w grid
// cells: psi(x - l h) = phi((u - l) * 2 / w) with u = x / h the coordinate in grid
// units.
//
// Binning.  Every point is mapped, in FP64, to u_a = r_a nf_a / L_a wrapped into
// [0, nf_a), the first index of its footprint l0_a = ceil(u_a - w/2) and the
// offset t_a = l0_a - u_a in [-w/2, -w/2 + 1) (kept in the working precision, so
// that large grids lose no phase accuracy).  Points are counting-sorted by the
// tile holding l0.
//
// Spreading.  One workgroup per tile accumulates its points into an LDS copy of
// the tile padded by w - 1 cells.  Accumulation is in fixed point with integer
// LDS atomics (gfx950 executes integer LDS atomics far faster than float ones,
// and the integer sum is exact and order independent); the scale is a power of
// two chosen per tile from its point count so that no cell can overflow.  The
// padded tile is then added into the periodic fine grid with float atomics.
//
// Interpolation.  One workgroup per tile stages the padded tile of every
// gradient component grid in LDS and evaluates sum_l v(l) psi(x_j - l h) for its
// points, writing the result at the point's original index.
#include <cmath>

#include "common.h"

namespace fresco {

template <class R>
__device__ __forceinline__ R es_kernel(R z, R beta) {
  R s = (R(1) - z) * (R(1) + z);
  return s >= R(0) ? exp(beta * (sqrt(s) - R(1))) : R(0);
}

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

template <class R>
__device__ __forceinline__ PointBin bin_point(const Geom& g, const R* r, bool* bad) {
  PointBin pb;
  pb.bin = 0;
  pb.cell = 0;
  uint32_t tile[3] = {0, 0, 0};
  for (int a = 0; a < 3; ++a) pb.t[a] = 0.0;
  for (int a = 0; a < g.d; ++a) {
    double x = (double)r[a];
    const double nf = (double)g.nf[a];
    double u = x * (nf / g.L[a]);
    if (!isfinite(u)) {
      *bad = true;
      u = 0.0;
    }
    u = fmod(u, nf);
    if (u < 0.0) u += nf;
    if (u >= nf) u = 0.0;
    double l0 = ceil(u - 0.5 * g.w);
    pb.t[a] = l0 - u;
    long long li = (long long)l0;
    if (li < 0) li += g.nf[a];
    if (li >= g.nf[a]) li -= g.nf[a];
    uint32_t ta = (uint32_t)(li / g.T[a]);
    uint32_t loc = (uint32_t)(li - (long long)ta * g.T[a]);
    tile[a] = ta;
    pb.cell |= loc << (8 * a);
  }
  pb.bin = tile[0] + (uint32_t)g.nt[0] * (tile[1] + (uint32_t)g.nt[1] * tile[2]);
  return pb;
}

template <class R>
__global__ void bin_count_kernel(Geom g, const R* __restrict__ pos, uint32_t* __restrict__ key,
                                 uint32_t* __restrict__ rank, uint32_t* __restrict__ count,
                                 int* __restrict__ flag) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  bool bad = false;
  PointBin pb = bin_point<R>(g, pos + i * g.d, &bad);
  if (bad) atomicOr(flag, 1);
  key[i] = pb.bin;
  rank[i] = atomicAdd(&count[pb.bin], 1u);
}

template <class R>
void launch_bin_count(const Geom& g, const R* pos, uint32_t* key, uint32_t* rank,
                      uint32_t* count, int* flag, hipStream_t st) {
  long long blocks = (g.N + 255) / 256;
  bin_count_kernel<R><<<(unsigned)blocks, 256, 0, st>>>(g, pos, key, rank, count, flag);
}

template <class R>
__global__ void bin_scatter_kernel(Geom g, const R* __restrict__ pos,
                                   const uint32_t* __restrict__ key,
                                   const uint32_t* __restrict__ rank,
                                   const long long* __restrict__ start, Rec<R>* __restrict__ rec,
                                   int* __restrict__ perm) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= g.N) return;
  bool bad = false;
  PointBin pb = bin_point<R>(g, pos + i * g.d, &bad);
  long long dst = start[key[i]] + rank[i];
  Rec<R> o;
  o.t[0] = (R)pb.t[0];
  o.t[1] = (R)pb.t[1];
  o.t[2] = (R)pb.t[2];
  o.cell = pb.cell;
  rec[dst] = o;
  perm[dst] = (int)i;
}

template <class R>
void launch_bin_scatter(const Geom& g, const R* pos, const uint32_t* key, const uint32_t* rank,
                        const long long* start, Rec<R>* rec, int* perm, hipStream_t st) {
  long long blocks = (g.N + 255) / 256;
  bin_scatter_kernel<R><<<(unsigned)blocks, 256, 0, st>>>(g, pos, key, rank, start, rec, perm);
}

// Exclusive scan of the per-tile counts into start[0..nbins] (one workgroup,
// chunks of 1024 in order).
__global__ void scan_bins_kernel(const uint32_t* __restrict__ count, long long nb,
                                 long long* __restrict__ start) {
  __shared__ long long s[1024];
  __shared__ long long carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (long long base = 0; base < nb; base += 1024) {
    long long i = base + threadIdx.x;
    long long v = (i < nb) ? (long long)count[i] : 0;
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
      long long add = (threadIdx.x >= (unsigned)off) ? s[threadIdx.x - off] : 0;
      __syncthreads();
      s[threadIdx.x] += add;
      __syncthreads();
    }
    if (i < nb) start[i] = carry + s[threadIdx.x] - v;
    __syncthreads();
    if (threadIdx.x == 1023) carry += s[1023];
    __syncthreads();
  }
  if (threadIdx.x == 0) start[nb] = carry;
}

void launch_scan_bins(const Geom& g, const uint32_t* count, long long* start, hipStream_t st) {
  scan_bins_kernel<<<1, 1024, 0, st>>>(count, g.nbins, start);
}

// ------------------------------------------------------------- spreading
template <class R>
struct FixedPoint;
template <>
struct FixedPoint<float> {
  using T = uint32_t;
  static constexpr int bits = 31;
};
template <>
struct FixedPoint<double> {
  using T = unsigned long long;
  static constexpr int bits = 63;
};

__device__ __forceinline__ uint32_t to_fixed(float v) { return __float2uint_rn(v); }
__device__ __forceinline__ unsigned long long to_fixed(double v) {
  return (unsigned long long)(v + 0.5);
}

__device__ __forceinline__ void tile_coords(const Geom& g, long long bin, int* t) {
  t[0] = (int)(bin % g.nt[0]);
  long long r = bin / g.nt[0];
  t[1] = (int)(r % g.nt[1]);
  t[2] = (int)(r / g.nt[1]);
}

template <class R, int D, int W>
__global__ void spread_kernel(Geom g, const Rec<R>* __restrict__ rec,
                              const long long* __restrict__ start, R* __restrict__ grid) {
  using A = typename FixedPoint<R>::T;
  extern __shared__ unsigned char smem_raw[];
  A* acc = reinterpret_cast<A*>(smem_raw);
  const long long bin = blockIdx.x;
  const int E0 = g.E[0], E1 = g.E[1], E2 = (D == 3) ? g.E[2] : 1;
  const int ncell = E0 * E1 * E2;
  const long long s = start[bin], e = start[bin + 1];
  if (e == s) return;  // uniform across the block
  for (int c = threadIdx.x; c < ncell; c += blockDim.x) acc[c] = 0;
  // fixed-point scale 2^ex with (count + 1) 2^ex <= 2^bits: each contribution is
  // at most 1, so no cell of the tile can overflow
  const double cnt1 = (double)(e - s + 1);
  const int ex = (int)floor(log2(ldexp(1.0, FixedPoint<R>::bits) / cnt1));
  const R scale = (R)ldexp(1.0, ex);
  const R inv_scale = (R)ldexp(1.0, -ex);
  const R half_w_inv = R(2) / R(W);
  const R beta = (R)g.beta;
  __syncthreads();
  for (long long j = s + threadIdx.x; j < e; j += blockDim.x) {
    const Rec<R> p = rec[j];
    R k0[W], k1[W], k2[W];
#pragma unroll
    for (int i = 0; i < W; ++i) {
      k0[i] = es_kernel<R>((p.t[0] + R(i)) * half_w_inv, beta);
      k1[i] = es_kernel<R>((p.t[1] + R(i)) * half_w_inv, beta);
      if (D == 3) k2[i] = es_kernel<R>((p.t[2] + R(i)) * half_w_inv, beta);
    }
    const int l0 = p.cell & 0xff, l1 = (p.cell >> 8) & 0xff, l2 = (p.cell >> 16) & 0xff;
    if (D == 2) {
#pragma unroll
      for (int dy = 0; dy < W; ++dy) {
        const R py = k1[dy] * scale;
        A* row = acc + (l1 + dy) * E0 + l0;
#pragma unroll
        for (int dx = 0; dx < W; ++dx) atomicAdd(row + dx, to_fixed(py * k0[dx]));
      }
    } else {
      for (int dz = 0; dz < W; ++dz) {
        const R pz = k2[dz] * scale;
#pragma unroll
        for (int dy = 0; dy < W; ++dy) {
          const R py = k1[dy] * pz;
          A* row = acc + ((l2 + dz) * E1 + (l1 + dy)) * E0 + l0;
#pragma unroll
          for (int dx = 0; dx < W; ++dx) atomicAdd(row + dx, to_fixed(py * k0[dx]));
        }
      }
    }
  }
  __syncthreads();
  int t[3];
  tile_coords(g, bin, t);
  const int o0 = t[0] * g.T[0], o1 = t[1] * g.T[1], o2 = t[2] * g.T[2];
  for (int c = threadIdx.x; c < ncell; c += blockDim.x) {
    const A a = acc[c];
    if (a == 0) continue;
    const int c0 = c % E0;
    const int r = c / E0;
    const int c1 = r % E1;
    const int c2 = r / E1;
    int x = o0 + c0, y = o1 + c1, z = o2 + c2;
    while (x >= g.nf[0]) x -= g.nf[0];
    while (y >= g.nf[1]) y -= g.nf[1];
    while (z >= g.nf[2]) z -= g.nf[2];
    const long long gi = ((long long)z * g.nf[1] + y) * g.nf[0] + x;
    unsafeAtomicAdd(grid + gi, (R)a * inv_scale);
  }
}

// ---------------------------------------------------------- interpolation
template <class R, int D, int W>
__global__ void interp_kernel(Geom g, const Rec<R>* __restrict__ rec,
                              const long long* __restrict__ start, const int* __restrict__ perm,
                              const R* __restrict__ v0, const R* __restrict__ v1,
                              const R* __restrict__ v2, int c_first, int nc,
                              R* __restrict__ grad) {
  extern __shared__ unsigned char smem_raw[];
  R* sub = reinterpret_cast<R*>(smem_raw);
  const long long bin = blockIdx.x;
  const int E0 = g.E[0], E1 = g.E[1], E2 = (D == 3) ? g.E[2] : 1;
  const int ncell = E0 * E1 * E2;
  const long long s = start[bin], e = start[bin + 1];
  if (e == s) return;
  int t[3];
  tile_coords(g, bin, t);
  const int o0 = t[0] * g.T[0], o1 = t[1] * g.T[1], o2 = t[2] * g.T[2];
  const R* src[3] = {v0, v1, v2};
  for (int k = 0; k < nc; ++k) {
    const R* __restrict__ v = src[c_first + k];
    for (int c = threadIdx.x; c < ncell; c += blockDim.x) {
      const int c0 = c % E0;
      const int r = c / E0;
      const int c1 = r % E1;
      const int c2 = r / E1;
      int x = o0 + c0, y = o1 + c1, z = o2 + c2;
      while (x >= g.nf[0]) x -= g.nf[0];
      while (y >= g.nf[1]) y -= g.nf[1];
      while (z >= g.nf[2]) z -= g.nf[2];
      sub[k * ncell + c] = v[((long long)z * g.nf[1] + y) * g.nf[0] + x];
    }
  }
  __syncthreads();
  const R half_w_inv = R(2) / R(W);
  const R beta = (R)g.beta;
  for (long long j = s + threadIdx.x; j < e; j += blockDim.x) {
    const Rec<R> p = rec[j];
    R k0[W], k1[W], k2[W];
#pragma unroll
    for (int i = 0; i < W; ++i) {
      k0[i] = es_kernel<R>((p.t[0] + R(i)) * half_w_inv, beta);
      k1[i] = es_kernel<R>((p.t[1] + R(i)) * half_w_inv, beta);
      if (D == 3) k2[i] = es_kernel<R>((p.t[2] + R(i)) * half_w_inv, beta);
    }
    const int l0 = p.cell & 0xff, l1 = (p.cell >> 8) & 0xff, l2 = (p.cell >> 16) & 0xff;
    const long long o = (long long)perm[j] * D;
    for (int k = 0; k < nc; ++k) {
      const R* sg = sub + k * ncell;
      R acc = R(0);
      if (D == 2) {
#pragma unroll
        for (int dy = 0; dy < W; ++dy) {
          const R* row = sg + (l1 + dy) * E0 + l0;
          R rs = R(0);
#pragma unroll
          for (int dx = 0; dx < W; ++dx) rs += row[dx] * k0[dx];
          acc += rs * k1[dy];
        }
      } else {
        for (int dz = 0; dz < W; ++dz) {
          R ps = R(0);
#pragma unroll
          for (int dy = 0; dy < W; ++dy) {
            const R* row = sg + ((l2 + dz) * E1 + (l1 + dy)) * E0 + l0;
            R rs = R(0);
#pragma unroll
            for (int dx = 0; dx < W; ++dx) rs += row[dx] * k0[dx];
            ps += rs * k1[dy];
          }
          acc += ps * k2[dz];
        }
      }
      grad[o + c_first + k] = acc;
    }
  }
}

// --------------------------------------------------------------- launch
template <class R, int D, int W>
static void spread_launch_w(const Geom& g, const Rec<R>* rec, const long long* start, R* grid,
                            hipStream_t st) {
  using A = typename FixedPoint<R>::T;
  const size_t lds = (size_t)g.E[0] * g.E[1] * (D == 3 ? g.E[2] : 1) * sizeof(A);
  hipFuncSetAttribute((const void*)spread_kernel<R, D, W>,
                      hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  spread_kernel<R, D, W><<<(unsigned)g.nbins, 256, lds, st>>>(g, rec, start, grid);
}

template <class R, int D, int W>
static void interp_launch_w(const Geom& g, const Rec<R>* rec, const long long* start,
                            const int* perm, const R* const* comps, int ncomp, R* grad,
                            hipStream_t st) {
  const size_t cell = (size_t)g.E[0] * g.E[1] * (D == 3 ? g.E[2] : 1) * sizeof(R);
  int per = (int)((160 * 1024) / cell);
  if (per > ncomp) per = ncomp;
  if (per < 1) per = 1;
  for (int c0 = 0; c0 < ncomp; c0 += per) {
    const int nc = (ncomp - c0 < per) ? ncomp - c0 : per;
    const size_t lds = cell * nc;
    hipFuncSetAttribute((const void*)interp_kernel<R, D, W>,
                        hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    interp_kernel<R, D, W><<<(unsigned)g.nbins, 256, lds, st>>>(
        g, rec, start, perm, comps[0], ncomp > 1 ? comps[1] : nullptr,
        ncomp > 2 ? comps[2] : nullptr, c0, nc, grad);
  }
}

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

template <class R>
void launch_spread(const Geom& g, const Rec<R>* rec, const long long* start, R* grid,
                   hipStream_t st) {
  if (g.d == 2) {
#define SP2(W) spread_launch_w<R, 2, W>(g, rec, start, grid, st)
    FRESCO_W_SWITCH(g.w, SP2)
#undef SP2
  } else {
#define SP3(W) spread_launch_w<R, 3, W>(g, rec, start, grid, st)
    FRESCO_W_SWITCH(g.w, SP3)
#undef SP3
  }
}

template <class R>
void launch_interp(const Geom& g, const Rec<R>* rec, const long long* start, const int* perm,
                   const R* const* comps, int ncomp, R* grad, hipStream_t st) {
  if (g.d == 2) {
#define IP2(W) interp_launch_w<R, 2, W>(g, rec, start, perm, comps, ncomp, grad, st)
    FRESCO_W_SWITCH(g.w, IP2)
#undef IP2
  } else {
#define IP3(W) interp_launch_w<R, 3, W>(g, rec, start, perm, comps, ncomp, grad, st)
    FRESCO_W_SWITCH(g.w, IP3)
#undef IP3
  }
}

template void launch_bin_count<float>(const Geom&, const float*, uint32_t*, uint32_t*, uint32_t*,
                                      int*, hipStream_t);
template void launch_bin_count<double>(const Geom&, const double*, uint32_t*, uint32_t*,
                                       uint32_t*, int*, hipStream_t);
template void launch_bin_scatter<float>(const Geom&, const float*, const uint32_t*,
                                        const uint32_t*, const long long*, Rec<float>*, int*,
                                        hipStream_t);
template void launch_bin_scatter<double>(const Geom&, const double*, const uint32_t*,
                                         const uint32_t*, const long long*, Rec<double>*, int*,
                                         hipStream_t);
template void launch_spread<float>(const Geom&, const Rec<float>*, const long long*, float*,
                                   hipStream_t);
template void launch_spread<double>(const Geom&, const Rec<double>*, const long long*, double*,
                                    hipStream_t);
template void launch_interp<float>(const Geom&, const Rec<float>*, const long long*, const int*,
                                   const float* const*, int, float*, hipStream_t);
template void launch_interp<double>(const Geom&, const Rec<double>*, const long long*,
                                    const int*, const double* const*, int, double*, hipStream_t);

}  // namespace fresco
