// LDS-staged mixed-radix Stockham FFT passes for gfx950, and the pointwise
// mode stage fused into the last forward pass.
//
// The uniform part of the nonuniform transforms (Methods: type-1 = spread,
// FFT, deconvolve; type-2 = pre-deconvolve, FFT, interpolate) runs as one pass
// per axis over the fine grid, pruned to the |n_a| <= M_a modes that the loss
// uses:
//   rows (axis 0)  real <-> half spectrum n_0 in [0, M_0], through a complex FFT
//                  of half the length (even/odd packing);
//   columns        complex lines along axis 1 or 2, loading only the nonzero
//                  modes on the inverse side and storing only the needed ones
//                  on the forward side.
// Forward passes use exp(+i n l h) (the paper's rho(k) sign), inverse passes
// exp(-i n l h).  Every line is transformed inside LDS by a Stockham
// autosort FFT whose stages read all their inputs into registers before any
// write, so one LDS buffer suffices.
#include <cmath>

#include "common.h"
#include "fft.h"
#include "fft_lds.h"

namespace fresco {

// ------------------------------------------------------------ row passes
// Forward rows: real line x[0..nf) -> X[k] = sum_l x_l exp(+2 pi i k l / nf) for
// k in [0, M0], via z_m = x_2m + i x_2m+1 and a complex FFT of length H = nf/2:
//   X[k] = (Z[k] + conj Z[H-k]) / 2 + exp(+2 pi i k / nf) (Z[k] - conj Z[H-k]) / (2i).
// LDS: [twiddles H][lines x (H + 1)].
// Copy src[k * sstride] to dst[k * dstride] for k = k0, k0 + step, ... < cnt,
// four loads in flight per thread before the first store (line loads are
// latency-bound otherwise).
template <class T>
__device__ __forceinline__ void copy_strided4(T* __restrict__ dst, long long dstride,
                                              const T* __restrict__ src, long long sstride,
                                              int k0, int step, int cnt) {
  for (int k = k0; k < cnt; k += 4 * step) {
    T v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (k + u * step < cnt) v[u] = src[(long long)(k + u * step) * sstride];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (k + u * step < cnt) dst[(long long)(k + u * step) * dstride] = v[u];
  }
}

// One grid line of the folded spread: cell (x, y, z) = sum over the padded
// tiles that cover it, in the order of the stand-alone fold.  xoff / xent: the
// first axis's cover lists in LDS.  Cells covered at most twice along every axis
// (all but those next to the wrap of a grid that is not a whole number of tiles)
// take a fixed set of loads issued together; the others walk their lists.
template <class R>
__device__ __forceinline__ R fold_cell_any(const RowFold<R>& f, int x, int yb, int ye, int zb,
                                           int ze, const int* xoff, const int2* xent) {
  R acc = R(0);
  for (int iz = zb; iz < ze; ++iz) {
    int tz = 0, lz = 0;
    if (f.d == 3) {
      const int2 e = f.ent[2][iz];
      tz = e.x;
      lz = e.y;
    }
    for (int iy = yb; iy < ye; ++iy) {
      const int2 ey = f.ent[1][iy];
      const long long base = (long long)f.nt0 * (ey.x + f.nt1 * tz) * f.ncell +
                             (long long)(lz * f.E1 + ey.y) * f.E0;
      for (int ix = xoff[x]; ix < xoff[x + 1]; ++ix) {
        const int2 ex = xent[ix];
        acc += f.tiles[base + (long long)ex.x * f.ncell + ex.y];
      }
    }
  }
  return acc;
}

template <class R>
__device__ __forceinline__ void fold_line(const RowFold<R>& f, long long row, const int* xoff,
                                          const int2* xent, cpx<R>* __restrict__ line, int tj,
                                          int JT, int H) {
  const int y = (f.d == 3) ? (int)(row % f.nf1) : (int)row;
  const int z = (f.d == 3) ? (int)(row / f.nf1) : 0;
  const int yb = f.off[1][y], ye = f.off[1][y + 1];
  const int zb = (f.d == 3) ? f.off[2][z] : 0;
  const int ze = (f.d == 3) ? f.off[2][z + 1] : 1;
  const int ny = ye - yb, nz = ze - zb;
  const bool fast_yz = ny <= 2 && nz <= 2;
  long long base[2][2];
  bool ok[2][2];
#pragma unroll
  for (int kz = 0; kz < 2; ++kz) {
    int tz = 0, lz = 0;
    if (f.d == 3 && kz < nz) {
      const int2 e = f.ent[2][zb + kz];
      tz = e.x;
      lz = e.y;
    }
#pragma unroll
    for (int ky = 0; ky < 2; ++ky) {
      ok[kz][ky] = kz < nz && ky < ny;
      base[kz][ky] = 0;
      if (ok[kz][ky]) {
        const int2 e = f.ent[1][yb + ky];
        base[kz][ky] = (long long)f.nt0 * (e.x + f.nt1 * tz) * f.ncell +
                       (long long)(lz * f.E1 + e.y) * f.E0;
      }
    }
  }
  for (int m = tj; m < H; m += JT) {
    R acc[2];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int x = 2 * m + h;
      const int xb = xoff[x], nx = xoff[x + 1] - xb;
      if (fast_yz && nx <= 2) {
        // every load issued (unused taps read the first cell), then summed
        const int2 e0 = xent[xb], e1 = xent[xb + (nx > 1 ? 1 : 0)];
        R v[2][2][2];
#pragma unroll
        for (int kz = 0; kz < 2; ++kz)
#pragma unroll
          for (int ky = 0; ky < 2; ++ky) {
            const long long b0 = ok[kz][ky] ? base[kz][ky] + e0.x * f.ncell + e0.y : 0;
            const long long b1 = (ok[kz][ky] && nx > 1) ? base[kz][ky] + e1.x * f.ncell + e1.y : 0;
            v[kz][ky][0] = f.tiles[b0];
            v[kz][ky][1] = f.tiles[b1];
          }
        R a = R(0);
#pragma unroll
        for (int kz = 0; kz < 2; ++kz)
#pragma unroll
          for (int ky = 0; ky < 2; ++ky)
            if (ok[kz][ky]) {
              a += v[kz][ky][0];
              if (nx > 1) a += v[kz][ky][1];
            }
        acc[h] = a;
      } else {
        acc[h] = fold_cell_any(f, x, yb, ye, zb, ze, xoff, xent);
      }
    }
    line[m] = cpx<R>{acc[0], acc[1]};
  }
}

// row served by line b of this workgroup
template <class R>
__device__ __forceinline__ long long row_of_block(const RowParams<R>& p, int b) {
  if (!p.xcd16) return (long long)blockIdx.x * p.lines_per_block + b;
  const uint32_t w = blockIdx.x, x = w & 7u, l = w >> 3;
  return ((long long)((l >> 4) * 8u + x) << 4) + (l & 15u);
}

template <class R, int MAXB>
__global__ void rows_r2c_kernel(RowParams<R> p, FftFactors F, const cpx<R>* __restrict__ twH,
                                const cpx<R>* __restrict__ twN) {
  extern __shared__ unsigned long long smem_u64[];
  cpx<R>* tws = reinterpret_cast<cpx<R>*>(smem_u64);
  const int H = F.n;
  const bool twl = p.tw_lds;  // twiddles staged in LDS (long lines read them from L2)
  cpx<R>* buf = twl ? tws + H : tws;
  const int ls = H + 1;
  const int JT = blockDim.x / p.lines_per_block;
  const int b = threadIdx.x / JT, tj = threadIdx.x % JT;
  const long long row = row_of_block(p, b);
  if (p.xcd16 && row >= p.nrows) return;  // whole workgroup
  const bool active = row < p.nrows;
  if (twl) load_twiddles(tws, twH, H);
  if (p.fold.tiles) {
    int* xoff = reinterpret_cast<int*>(buf + (long long)p.lines_per_block * ls);
    int2* xent = reinterpret_cast<int2*>(xoff + ((2 * H + 2) & ~1));
    copy_strided4(xoff, 1ll, p.fold.off[0], 1ll, (int)threadIdx.x, (int)blockDim.x, 2 * H + 1);
    copy_strided4(xent, 1ll, p.fold.ent[0], 1ll, (int)threadIdx.x, (int)blockDim.x,
                  p.fold.nent0);
    __syncthreads();
    if (active) fold_line(p.fold, row, xoff, xent, buf + b * ls, tj, JT, H);
  } else if (active) {
    const R* __restrict__ x = p.rin + row * (2LL * H);
    copy_strided4(buf + b * ls, 1ll, reinterpret_cast<const cpx<R>*>(x), 1ll, tj, JT, H);
  }
  __syncthreads();
  if (twl) lds_fft<R, MAXB, false>(buf, F, tws, active, b, ls, 1, tj, JT);
  else lds_fft<R, MAXB, false>(buf, F, twH, active, b, ls, 1, tj, JT);
  if (active) {
    cpx<R>* __restrict__ out = p.cout + row * p.rstride;
    for (int k = tj; k <= p.M0; k += JT) {
      cpx<R> Zk = buf[b * ls + k];
      cpx<R> Zc = cconj(buf[b * ls + (k == 0 ? 0 : H - k)]);
      cpx<R> E = cscale(cadd(Zk, Zc), R(0.5));
      cpx<R> O = cscale(cmul_mi(csub(Zk, Zc)), R(0.5));  // (Zk - Zc) / (2i)
      out[k * p.kstride] = cadd(E, cmul(twN[k], O));
    }
  }
}

// Inverse rows: half spectrum X[0..M0] (Hermitian extension implied) ->
// real x_l = sum_n X[n] exp(-2 pi i n l / nf), through
//   Z[k] = E[k] + i O[k],  E[k] = X[k] + X[k-H],
//   O[k] = exp(-2 pi i k / nf) (X[k] - X[k-H]),  X[k-H] = conj X[H-k],
// and x_2m + i x_2m+1 = sum_k Z[k] exp(-2 pi i k m / H).  The imaginary part of
// X[0] is not part of a real field and is dropped.
template <class R, int MAXB>
__global__ void rows_c2r_kernel(RowParams<R> p, FftFactors F, const cpx<R>* __restrict__ twH,
                                const cpx<R>* __restrict__ twN) {
  extern __shared__ unsigned long long smem_u64[];
  cpx<R>* tws = reinterpret_cast<cpx<R>*>(smem_u64);
  const int H = F.n;
  const bool twl = p.tw_lds;
  cpx<R>* buf = twl ? tws + H : tws;
  const int ls = H + 1;
  const int JT = blockDim.x / p.lines_per_block;
  const int b = threadIdx.x / JT, tj = threadIdx.x % JT;
  const long long row = row_of_block(p, b);
  if (p.xcd16 && row >= p.nrows) return;  // whole workgroup
  const bool active = row < p.nrows;
  const int comp = blockIdx.y;
  const int M0 = p.M0;
  if (twl) load_twiddles(tws, twH, H);
  if (active) {
    const cpx<R>* __restrict__ X = p.cin[comp] + row * p.rstride;
    const long long ks = p.kstride;
    // four iterations' strided loads are issued before any of them is used
    constexpr int U = 4;
    for (int k0 = tj; k0 < H; k0 += U * JT) {
      cpx<R> xk[U], xm[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = k0 + u * JT;
        xk[u] = cpx<R>{R(0), R(0)};
        xm[u] = cpx<R>{R(0), R(0)};
        if (k < H && k <= M0) xk[u] = X[k * ks];
        if (k < H && k > 0 && H - k <= M0) xm[u] = cconj(X[(H - k) * ks]);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int k = k0 + u * JT;
        if (k >= H) break;
        if (k == 0) xk[u].y = R(0);
        cpx<R> E = cadd(xk[u], xm[u]);
        cpx<R> O = cmulc(csub(xk[u], xm[u]), twN[k]);  // * exp(-2 pi i k / nf)
        buf[b * ls + k] = cadd(E, cmul_i(O));
      }
    }
  }
  __syncthreads();
  if (twl) lds_fft<R, MAXB, true>(buf, F, tws, active, b, ls, 1, tj, JT);
  else lds_fft<R, MAXB, true>(buf, F, twH, active, b, ls, 1, tj, JT);
  if (active) {
    R* __restrict__ y = p.rout[comp] + row * (2LL * H);
    for (int m = tj; m < H; m += JT) *reinterpret_cast<cpx<R>*>(y + 2 * m) = buf[b * ls + m];
  }
}

// --------------------------------------------------------- column passes
// Columns c in [0, ncols): element i of column c sits at
//   base(c) + i * line,  base(c) = (c / cdiv) * outer + c % cdiv.
// A block serves `bc` consecutive columns (bc a power of two); LDS holds the
// block as [i][b] so neighbouring threads touch neighbouring words.
// LDS: [twiddles n][n x bc data][(2M+1) x bc mode factors (FUSED, BWD)].

template <class R>
__device__ __forceinline__ long long col_base(long long c, const FastDiv& cdiv, long long outer) {
  uint32_t q = fdiv((uint32_t)c, cdiv);
  return (long long)q * outer + (c - (long long)q * cdiv.d);
}

// Mode-stage operands of up to kModePre modes per thread, loaded before the
// forward transform so that their latency overlaps it.
constexpr int kModePre = 4;

template <class R, int MAXB, int MODE>
__global__ void cols_kernel(ColParams<R> p, FftFactors F, const cpx<R>* __restrict__ twg) {
  extern __shared__ unsigned long long smem_u64[];
  const int n = F.n;
  const int bc = p.bc;
  cpx<R>* tws = reinterpret_cast<cpx<R>*>(smem_u64);
  const bool twl = p.tw_lds;  // twiddles staged in LDS (long lines read them from L2)
  cpx<R>* buf = twl ? tws + n : tws;
  cpx<R>* qbuf = buf + (long long)n * bc;  // [m][b], FUSED / BWD only
  const int P = 2 * p.M + 1;               // modes along this axis
  const int JT = blockDim.x / bc;
  const int b = threadIdx.x % bc, tj = threadIdx.x / bc;
  const long long c = (long long)blockIdx.x * bc + b;
  const bool active = c < p.ncols;
  const int comp = (MODE == COL_INV) ? blockIdx.y : 0;
  const long long ib = active ? col_base<R>(c, p.cdiv, p.in_outer) : 0;
  const long long ob = active ? col_base<R>(c, p.cdiv, p.out_outer) : 0;
  if (twl) load_twiddles(tws, twg, n);
#define COL_FFT(INV)                                                             \
  do {                                                                           \
    if (twl) lds_fft<R, MAXB, INV>(buf, F, tws, active, b, 1, bc, tj, JT);       \
    else lds_fft<R, MAXB, INV>(buf, F, twg, active, b, 1, bc, tj, JT);           \
  } while (0)

  // Mode stage (FUSED, SF, BWD; this is the last axis): column c holds the
  // half-spectrum modes (n_0, n_1[, n_2]) with n_last = m - M, where
  // c = n0 + H0 * (n1 + M1) in 3D, c = n0 in 2D.  Its column factors, and in
  // FUSED the weights, targets and kernel factors of this thread's modes
  // m = tj + u JT, are loaded before the forward transform.
  constexpr bool kModes = MODE == COL_FUSED || MODE == COL_SF || MODE == COL_BWD ||
                          MODE == COL_GFIELD || MODE == COL_GBACK;
  int n0 = 0, n1 = 0;
  R dlead = R(0), ilead = R(0);
  if (kModes && active) {
    if (p.d == 2) {
      n0 = (int)c;
    } else {
      uint32_t q = fdiv((uint32_t)c, p.h0div);
      n0 = (int)(c - (long long)q * p.h0div.d);
      n1 = (int)q - p.M1;
    }
    const int a1 = n1 < 0 ? -n1 : n1;
    dlead = p.dec[0][n0] * ((p.d == 3) ? p.dec[1][a1] : R(1));
    ilead = p.deci[0][n0] * ((p.d == 3) ? p.deci[1][a1] : R(1));
  }
  const bool pre = (MODE == COL_FUSED) && P <= kModePre * JT;
  R pwp[kModePre], pwm[kModePre], psp[kModePre], psm[kModePre], pdc[kModePre], pdi[kModePre];
  if (MODE == COL_FUSED && pre) {
#pragma unroll
    for (int u = 0; u < kModePre; ++u) {
      const int m = tj + u * JT;
      const long long h = p.mcol ? c * P + m : c + (long long)p.ncols * m;
      const bool ok = active && m < P;
      const int nl = m - p.M;
      const int al = ok ? (nl < 0 ? -nl : nl) : 0;
      pwp[u] = ok ? p.Wp[h] : R(0);
      pwm[u] = ok ? p.Wm[h] : R(0);
      psp[u] = ok ? p.S0p[h] : R(0);
      psm[u] = ok ? p.S0m[h] : R(0);
      pdc[u] = ok ? p.dec[p.d - 1][al] : R(0);
      pdi[u] = ok ? p.deci[p.d - 1][al] : R(0);
    }
  }
  if (MODE == COL_FWD || MODE == COL_FUSED || MODE == COL_SF || MODE == COL_GBACK) {
    // forward: load the full spatial line, transform with exp(+i ...)
    if (active) copy_strided4(buf + b, (long long)bc, p.in[0] + ib, p.in_line, tj, JT, n);
    __syncthreads();
    COL_FFT(false);
  }
  if (MODE == COL_FWD) {
    if (active) {
      cpx<R>* __restrict__ out = p.out[0];
      for (int m = tj; m < P; m += JT) {
        int i = m - p.M;
        if (i < 0) i += n;
        out[ob + (long long)m * p.out_line] = buf[i * bc + b];
      }
    }
    return;
  }
  if (MODE == COL_INV) {
    // inverse: scatter the 2M+1 modes into a zeroed line, transform with exp(-i ...)
    for (int i = tj; i < n; i += JT) buf[i * bc + b] = cpx<R>{R(0), R(0)};
    __syncthreads();
    if (active) {
      const cpx<R>* __restrict__ in = p.in[comp];
      for (int m0 = tj; m0 < P; m0 += 4 * JT) {
        cpx<R> v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
          if (m0 + u * JT < P) v[u] = in[ib + (long long)(m0 + u * JT) * p.in_line];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          const int m = m0 + u * JT;
          if (m < P) {
            int i = m - p.M;
            if (i < 0) i += n;
            buf[i * bc + b] = v[u];
          }
        }
      }
    }
    __syncthreads();
    COL_FFT(true);
    if (active) {
      cpx<R>* __restrict__ out = p.out[comp];
      for (int i = tj; i < n; i += JT) out[ob + (long long)i * p.out_line] = buf[i * bc + b];
    }
    return;
  }

  // ---- mode stage
  double lsum = 0.0, fsum = 0.0;
  if (active) {
    // dk, dik: kernel factors of the last axis at |n_last|
    auto mode_body = [&](int m, R wp, R wm, R s0p, R s0m, R dk, R dik) {
      const int nl = m - p.M;
      const R dec = dlead * dk;
      // half-spectrum index of the mode-stage arrays
      const long long hidx = p.mcol ? c * P + m : c + (long long)p.ncols * m;
      cpx<R> rho;
      if (MODE == COL_BWD || MODE == COL_GFIELD || MODE == COL_GBACK) {
        rho = p.rho_save[hidx];
      } else {
        const int i = nl < 0 ? nl + n : nl;
        rho = cscale(buf[i * bc + b], dec);
        if (p.rho_save) p.rho_save[hidx] = rho;
      }
      const R S = (rho.x * rho.x + rho.y * rho.y) * p.invN;
      // full-cube indices of n and -n (C order over n_0..n_{d-1})
      long long cp, cm;
      if (p.d == 2) {
        cp = (long long)(n0 + p.M0) * p.P1 + (nl + p.M1);
        cm = (long long)(-n0 + p.M0) * p.P1 + (-nl + p.M1);
      } else {
        cp = ((long long)(n0 + p.M0) * p.P1 + (n1 + p.M1)) * p.P2 + (nl + p.M2);
        cm = ((long long)(-n0 + p.M0) * p.P1 + (-n1 + p.M1)) * p.P2 + (-nl + p.M2);
      }
      // the n_0 = 0 plane lists both members of each pair: each writes its own
      // entry only (two writers of one entry would race)
      if ((MODE == COL_SF || MODE == COL_FUSED) && p.S_cube) {
        p.S_cube[cp] = S;
        if (n0 > 0) p.S_cube[cm] = S;
      }
      if (MODE == COL_GFIELD) {
        // g(x) = (1/N) sum_n (S(n) - 1) exp(-i k.x): plain coefficients, no
        // kernel deconvolution (the inverse transform lands on grid points)
        qbuf[m * bc + b] = cpx<R>{(S - R(1)) * p.g_scale, R(0)};
      }
      if (MODE == COL_GBACK) {
        // dL_g/dS(n) = g_scale Re B(n), B the forward transform of b = 2 W_g (g - g0)
        // (real and even in n); S(0) = N does not depend on the positions
        const int i = nl < 0 ? nl + n : nl;
        const R G = (cp == cm) ? R(0) : buf[i * bc + b].x * p.g_scale;
        const R f = R(2) * G * p.invN * ilead * dik;
        qbuf[m * bc + b] = cscale(rho, f);
      }
      if (MODE == COL_FUSED || MODE == COL_BWD) {
        // G: dL/dS symmetrised over the pair (n, -n)
        R G;
        if (MODE == COL_FUSED) {
          const R rp = S - s0p, rm = S - s0m;
          // loss over the full set: n and -n both when n_0 > 0; the n_0 = 0 plane
          // lists both members of every pair itself
          lsum += (double)wp * (double)rp * (double)rp;
          if (n0 > 0) lsum += (double)wm * (double)rm * (double)rm;
          if (p.fsum_part) {
            fsum += (double)wp * (double)S * (double)rp;
            if (n0 > 0) fsum += (double)wm * (double)S * (double)rm;
          }
          G = wp * rp + wm * rm;
        } else {
          // S(0) = N does not depend on the positions
          G = (cp == cm) ? R(0) : R(0.5) * (p.g_cube[cp] + p.g_cube[cm]);
        }
        // type-2 input of the field whose derivative is the gradient:
        // C0 = 2 G rho / N, divided by psihat_i and scaled by h^d
        const R f = R(2) * G * p.invN * ilead * dik;
        qbuf[m * bc + b] = cscale(rho, f);
      }
    };
    if (MODE == COL_FUSED && pre) {
#pragma unroll
      for (int u = 0; u < kModePre; ++u) {
        const int m = tj + u * JT;
        if (m < P) mode_body(m, pwp[u], pwm[u], psp[u], psm[u], pdc[u], pdi[u]);
      }
    } else {
      for (int m = tj; m < P; m += JT) {
        const long long h = p.mcol ? c * P + m : c + (long long)p.ncols * m;
        const int nl = m - p.M;
        const int al = nl < 0 ? -nl : nl;
        const R dk = p.dec[p.d - 1][al], dik = p.deci[p.d - 1][al];
        if (MODE == COL_FUSED) mode_body(m, p.Wp[h], p.Wm[h], p.S0p[h], p.S0m[h], dk, dik);
        else mode_body(m, R(0), R(0), R(0), R(0), dk, dik);
      }
    }
  }
  if (MODE == COL_SF) return;
  if (MODE == COL_FUSED) {
    // block reduction of the loss partial (FP64), fixed order
    __shared__ double red[1024 / 64];
    double v = lsum;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
      p.loss_part[blockIdx.x] = t;
    }
    if (p.fsum_part) {  // uniform: the strength gradient's sum, same order
      __syncthreads();
      double f = fsum;
      for (int off = 32; off > 0; off >>= 1) f += __shfl_down(f, off, 64);
      if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = f;
      __syncthreads();
      if (threadIdx.x == 0) {
        double t = 0.0;
        for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
        p.fsum_part[blockIdx.x] = t;
      }
    }
  }
  // inverse transform of the field coefficients along this axis
  __syncthreads();
  for (int i = tj; i < n; i += JT) buf[i * bc + b] = cpx<R>{R(0), R(0)};
  __syncthreads();
  if (active) {
    for (int m = tj; m < P; m += JT) {
      int i = m - p.M;
      if (i < 0) i += n;
      buf[i * bc + b] = qbuf[m * bc + b];
    }
  }
  __syncthreads();
  COL_FFT(true);
  if (active) {
    cpx<R>* __restrict__ out = p.out[0];
    for (int i = tj; i < n; i += JT) out[ob + (long long)i * p.out_line] = buf[i * bc + b];
  }
}
#undef COL_FFT

// ------------------------------------------------- 2D columns too long for LDS
// A column of length n = 2m (2D, last axis) is split by decimation in time:
//   X[k] = Y0[k mod m] + exp(+2 pi i k / n) Y1[k mod m],
// Y_r = the length-m transform of the entries 2 i + r, computed by the column pass
// (pruned to |k| <= M, which needs 2M + 1 <= m).  The field coefficients q(k) go
// back by decimation in frequency: the entries 2 j + r of the inverse transform
// are the length-m inverse transforms of q(k) exp(-2 pi i k r / n).
// This kernel recombines X, runs the mode stage of the fused pass on it (S,
// loss, coefficients; or S only, or the backward's coefficients) and writes the
// two pre-twiddled coefficient sets.  Layout of Y0, Y1, Q0, Q1 and of the
// mode-stage arrays: [m][c], m = k + M, c = n0 in [0, M0].
template <class R, int MODE>
__global__ void long_modes_kernel(ColParams<R> p, const cpx<R>* __restrict__ Y,
                                  cpx<R>* __restrict__ Q, const cpx<R>* __restrict__ twn, int n) {
  const int P = 2 * p.M + 1;
  const long long H0 = p.ncols;
  const long long total = (long long)P * H0;
  double lsum = 0.0;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int m = (int)(e / H0);
    const int n0 = (int)(e - (long long)m * H0);
    const int nl = m - p.M;
    const int al = nl < 0 ? -nl : nl;
    const int ki = nl < 0 ? nl + n : nl;  // exp(+2 pi i k / n) = twn[k mod n]
    const long long hidx = e;              // [m][c]
    cpx<R> rho;
    if (MODE == COL_BWD) {
      rho = p.rho_save[hidx];
    } else {
      const cpx<R> X = cadd(Y[e], cmul(twn[ki], Y[total + e]));
      rho = cscale(X, p.dec[0][n0] * p.dec[1][al]);
      if (p.rho_save) p.rho_save[hidx] = rho;
    }
    const R S = (rho.x * rho.x + rho.y * rho.y) * p.invN;
    const long long cp = (long long)(n0 + p.M0) * p.P1 + (nl + p.M1);
    const long long cm = (long long)(-n0 + p.M0) * p.P1 + (-nl + p.M1);
    if ((MODE == COL_SF || MODE == COL_FUSED) && p.S_cube) {
      p.S_cube[cp] = S;
      if (n0 > 0) p.S_cube[cm] = S;  // the n_0 = 0 plane writes each entry itself
    }
    if (MODE == COL_FUSED || MODE == COL_BWD) {
      R G;
      if (MODE == COL_FUSED) {
        const R wp = p.Wp[hidx], wm = p.Wm[hidx];
        const R rp = S - p.S0p[hidx], rm = S - p.S0m[hidx];
        lsum += (double)wp * (double)rp * (double)rp;
        if (n0 > 0) lsum += (double)wm * (double)rm * (double)rm;
        G = wp * rp + wm * rm;
      } else {
        G = (cp == cm) ? R(0) : R(0.5) * (p.g_cube[cp] + p.g_cube[cm]);
      }
      const cpx<R> q = cscale(rho, R(2) * G * p.invN * p.deci[0][n0] * p.deci[1][al]);
      Q[e] = q;
      Q[total + e] = cmulc(q, twn[ki]);  // q exp(-2 pi i k / n)
    }
  }
  if (MODE != COL_FUSED) return;
  __shared__ double red[1024 / 64];
  for (int off = 32; off > 0; off >>= 1) lsum += __shfl_down(lsum, off, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = lsum;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
    p.loss_part[blockIdx.x] = t;
  }
}

template <class R>
hipError_t launch_long_modes(int mode, const ColParams<R>& p, const cpx<R>* Y, cpx<R>* Q,
                             const cpx<R>* twn, int n, int blocks, hipStream_t st) {
  if (mode == COL_FUSED)
    long_modes_kernel<R, COL_FUSED><<<blocks, 256, 0, st>>>(p, Y, Q, twn, n);
  else if (mode == COL_SF)
    long_modes_kernel<R, COL_SF><<<blocks, 256, 0, st>>>(p, Y, Q, twn, n);
  else
    long_modes_kernel<R, COL_BWD><<<blocks, 256, 0, st>>>(p, Y, Q, twn, n);
  return hipGetLastError();
}

// ------------------------------------------------------------ launchers
static int pick_maxb(int need) {
  if (need <= 1) return 1;
  if (need <= 2) return 2;
  if (need <= 4) return 4;
  if (need <= 8) return 8;
  return -1;
}

template <class R>
size_t rows_lds_bytes(const RowParams<R>& p, const AxisFft<R>& ax) {
  const int H = ax.F.n;
  size_t b = ((p.tw_lds ? (size_t)H : 0) + (size_t)p.lines_per_block * (H + 1)) * sizeof(cpx<R>);
  if (p.fold.tiles)  // first-axis cover lists (offsets padded to an even count)
    b += (size_t)((2 * H + 2) & ~1) * sizeof(int) + (size_t)p.fold.nent0 * sizeof(int2);
  return b;
}
template <class R>
size_t cols_lds_bytes(int mode, const ColParams<R>& p, const AxisFft<R>& ax) {
  const int n = ax.F.n;
  size_t e = (p.tw_lds ? (size_t)n : 0) + (size_t)n * p.bc;
  if (mode == COL_FUSED || mode == COL_BWD || mode == COL_GFIELD || mode == COL_GBACK)
    e += (size_t)(2 * p.M + 1) * p.bc;
  return e * sizeof(cpx<R>);
}

template <class R>
static int rows_maxb(const RowParams<R>& p, const AxisFft<R>& ax) {
  const int JT = p.threads / p.lines_per_block;
  return pick_maxb((ax.F.n + ax.rmin * JT - 1) / (ax.rmin * JT));
}
template <class R>
static int cols_maxb(const ColParams<R>& p, const AxisFft<R>& ax) {
  const int JT = p.threads / p.bc;
  return pick_maxb((ax.F.n + ax.rmin * JT - 1) / (ax.rmin * JT));
}

#define FRESCO_MB_SWITCH(MB_, CALL) \
  switch (MB_) {                    \
    case 1: CALL(1); break;         \
    case 2: CALL(2); break;         \
    case 4: CALL(4); break;         \
    case 8: CALL(8); break;         \
  }

template <class R>
hipError_t prepare_rows(const RowParams<R>& p, const AxisFft<R>& ax) {
  const int mb = rows_maxb(p, ax);
  if (mb < 0) return hipErrorInvalidValue;
  const int lds = (int)rows_lds_bytes(p, ax);
#define PREP(MB)                                                                      \
  do {                                                                                \
    hipFuncSetAttribute((const void*)rows_c2r_kernel<R, MB>,                         \
                        hipFuncAttributeMaxDynamicSharedMemorySize, lds);             \
    hipFuncSetAttribute((const void*)rows_r2c_kernel<R, MB>,                         \
                        hipFuncAttributeMaxDynamicSharedMemorySize, lds);             \
  } while (0)
  FRESCO_MB_SWITCH(mb, PREP)
#undef PREP
  return hipGetLastError();
}

template <class R>
hipError_t prepare_cols(int mode, const ColParams<R>& p, const AxisFft<R>& ax) {
  const int mb = cols_maxb(p, ax);
  if (mb < 0) return hipErrorInvalidValue;
  const int lds = (int)cols_lds_bytes(mode, p, ax);
#define PREP1(MB, MD)                                                                  \
  hipFuncSetAttribute((const void*)cols_kernel<R, MB, MD>,                            \
                      hipFuncAttributeMaxDynamicSharedMemorySize, lds)
#define PREP(MB)                                        \
  do {                                                  \
    switch (mode) {                                     \
      case COL_FWD: PREP1(MB, COL_FWD); break;          \
      case COL_INV: PREP1(MB, COL_INV); break;          \
      case COL_FUSED: PREP1(MB, COL_FUSED); break;      \
      case COL_SF: PREP1(MB, COL_SF); break;            \
      case COL_BWD: PREP1(MB, COL_BWD); break;          \
      case COL_GFIELD: PREP1(MB, COL_GFIELD); break;    \
      case COL_GBACK: PREP1(MB, COL_GBACK); break;      \
    }                                                   \
  } while (0)
  FRESCO_MB_SWITCH(mb, PREP)
#undef PREP
#undef PREP1
  return hipGetLastError();
}

template <class R>
hipError_t launch_rows(bool inverse, const RowParams<R>& p, const AxisFft<R>& ax, int ncomp,
                       hipStream_t st) {
  const int mb = rows_maxb(p, ax);
  if (mb < 0) return hipErrorInvalidValue;
  const size_t lds = rows_lds_bytes(p, ax);
  const long long groups = (p.nrows + 15) / 16;
  const long long nblk = p.xcd16 ? 128 * ((groups + 7) / 8)
                                 : (p.nrows + p.lines_per_block - 1) / p.lines_per_block;
  dim3 grid((unsigned)nblk, inverse ? ncomp : 1);
  dim3 block(p.threads);
#define ROWS(MB)                                                                   \
  do {                                                                             \
    if (inverse)                                                                   \
      rows_c2r_kernel<R, MB><<<grid, block, lds, st>>>(p, ax.F, ax.tw, ax.twN);   \
    else                                                                           \
      rows_r2c_kernel<R, MB><<<grid, block, lds, st>>>(p, ax.F, ax.tw, ax.twN);   \
  } while (0)
  FRESCO_MB_SWITCH(mb, ROWS)
#undef ROWS
  return hipGetLastError();
}

template <class R>
hipError_t launch_cols(int mode, const ColParams<R>& p, const AxisFft<R>& ax, int ncomp,
                       hipStream_t st) {
  const int mb = cols_maxb(p, ax);
  if (mb < 0) return hipErrorInvalidValue;
  const size_t lds = cols_lds_bytes(mode, p, ax);
  dim3 grid((unsigned)((p.ncols + p.bc - 1) / p.bc), mode == COL_INV ? ncomp : 1);
  dim3 block(p.threads);
#define COLS1(MB, MD) cols_kernel<R, MB, MD><<<grid, block, lds, st>>>(p, ax.F, ax.tw)
#define COLS(MB)                                        \
  do {                                                  \
    switch (mode) {                                     \
      case COL_FWD: COLS1(MB, COL_FWD); break;          \
      case COL_INV: COLS1(MB, COL_INV); break;          \
      case COL_FUSED: COLS1(MB, COL_FUSED); break;      \
      case COL_SF: COLS1(MB, COL_SF); break;            \
      case COL_BWD: COLS1(MB, COL_BWD); break;          \
      case COL_GFIELD: COLS1(MB, COL_GFIELD); break;    \
      case COL_GBACK: COLS1(MB, COL_GBACK); break;      \
    }                                                   \
  } while (0)
  FRESCO_MB_SWITCH(mb, COLS)
#undef COLS
#undef COLS1
  return hipGetLastError();
}

#define FRESCO_FFT_INST(R)                                                                        \
  template size_t rows_lds_bytes<R>(const RowParams<R>&, const AxisFft<R>&);                      \
  template size_t cols_lds_bytes<R>(int, const ColParams<R>&, const AxisFft<R>&);                 \
  template hipError_t prepare_rows<R>(const RowParams<R>&, const AxisFft<R>&);                    \
  template hipError_t prepare_cols<R>(int, const ColParams<R>&, const AxisFft<R>&);               \
  template hipError_t launch_rows<R>(bool, const RowParams<R>&, const AxisFft<R>&, int,           \
                                     hipStream_t);                                                \
  template hipError_t launch_cols<R>(int, const ColParams<R>&, const AxisFft<R>&, int, hipStream_t); \
  template hipError_t launch_long_modes<R>(int, const ColParams<R>&, const cpx<R>*, cpx<R>*,      \
                                           const cpx<R>*, int, int, hipStream_t);
FRESCO_FFT_INST(float)
FRESCO_FFT_INST(double)

}  // namespace fresco
