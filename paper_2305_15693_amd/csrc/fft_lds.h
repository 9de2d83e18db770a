// Device building blocks of the LDS-staged Stockham FFT (shared by the
// per-axis passes and the batched small-grid evaluation): radix-2/3/4/5 DFTs and
// the in-LDS transform of a set of lines.
#pragma once

#include "common.h"

namespace fresco {

// ----------------------------------------------------------- small DFTs
template <class R>
struct Consts;
template <>
struct Consts<float> {
  static constexpr float c3 = 0.86602540378443864676f;  // sin(2 pi / 3)
  static constexpr float c51 = 0.30901699437494742410f;  // cos(2 pi / 5)
  static constexpr float c52 = -0.80901699437494742410f; // cos(4 pi / 5)
  static constexpr float s51 = 0.95105651629515357212f;  // sin(2 pi / 5)
  static constexpr float s52 = 0.58778525229247312917f;  // sin(4 pi / 5)
};
template <>
struct Consts<double> {
  static constexpr double c3 = 0.86602540378443864676;
  static constexpr double c51 = 0.30901699437494742410;
  static constexpr double c52 = -0.80901699437494742410;
  static constexpr double s51 = 0.95105651629515357212;
  static constexpr double s52 = 0.58778525229247312917;
};

// V[u] = sum_t v[t] exp(s 2 pi i t u / r), s = +1 (forward) or -1 (inverse)
template <class R, bool INV>
__device__ __forceinline__ void dft2(cpx<R>* v) {
  cpx<R> a = v[0], b = v[1];
  v[0] = cadd(a, b);
  v[1] = csub(a, b);
}
template <class R, bool INV>
__device__ __forceinline__ void dft3(cpx<R>* v) {
  cpx<R> t1 = cadd(v[1], v[2]), t2 = csub(v[1], v[2]);
  cpx<R> a = {v[0].x - R(0.5) * t1.x, v[0].y - R(0.5) * t1.y};
  cpx<R> b = cscale(t2, Consts<R>::c3);
  b = INV ? cmul_mi(b) : cmul_i(b);
  v[0] = cadd(v[0], t1);
  v[1] = cadd(a, b);
  v[2] = csub(a, b);
}
template <class R, bool INV>
__device__ __forceinline__ void dft4(cpx<R>* v) {
  cpx<R> s02 = cadd(v[0], v[2]), d02 = csub(v[0], v[2]);
  cpx<R> s13 = cadd(v[1], v[3]), d13 = csub(v[1], v[3]);
  cpx<R> id13 = INV ? cmul_mi(d13) : cmul_i(d13);
  v[0] = cadd(s02, s13);
  v[1] = cadd(d02, id13);
  v[2] = csub(s02, s13);
  v[3] = csub(d02, id13);
}
template <class R, bool INV>
__device__ __forceinline__ void dft5(cpx<R>* v) {
  const R c1 = Consts<R>::c51, c2 = Consts<R>::c52, s1 = Consts<R>::s51, s2 = Consts<R>::s52;
  cpx<R> b1 = cadd(v[1], v[4]), b2 = cadd(v[2], v[3]);
  cpx<R> d1 = csub(v[1], v[4]), d2 = csub(v[2], v[3]);
  cpx<R> A = {v[0].x + c1 * b1.x + c2 * b2.x, v[0].y + c1 * b1.y + c2 * b2.y};
  cpx<R> C = {v[0].x + c2 * b1.x + c1 * b2.x, v[0].y + c2 * b1.y + c1 * b2.y};
  cpx<R> B = {s1 * d1.x + s2 * d2.x, s1 * d1.y + s2 * d2.y};
  cpx<R> D = {s2 * d1.x - s1 * d2.x, s2 * d1.y - s1 * d2.y};
  B = INV ? cmul_mi(B) : cmul_i(B);
  D = INV ? cmul_mi(D) : cmul_i(D);
  v[0] = cadd(v[0], cadd(b1, b2));
  v[1] = cadd(A, B);
  v[4] = csub(A, B);
  v[2] = cadd(C, D);
  v[3] = csub(C, D);
}

template <class R, bool INV, int RAD>
__device__ __forceinline__ void dft(cpx<R>* v) {
  if constexpr (RAD == 2) dft2<R, INV>(v);
  else if constexpr (RAD == 3) dft3<R, INV>(v);
  else if constexpr (RAD == 4) dft4<R, INV>(v);
  else dft5<R, INV>(v);
}

// One radix-RAD Stockham stage s (radix fixed at compile time, so that the
// loads, twiddles and butterfly carry no run-time radix tests); both barriers
// inside.
template <class R, int MAXB, bool INV, int RAD>
__device__ __forceinline__ void lds_stage(cpx<R>* buf, const FftFactors& F, int s,
                                          const cpx<R>* __restrict__ tw, bool active, int b,
                                          int ls, int es, int tj, int JT) {
  const int nr = F.n / RAD;
  const FastDiv nsd = F.ns[s];
  const uint32_t tstep = F.twstep[s];
  cpx<R> v[MAXB][RAD];
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int j = tj + q * JT;
    if (active && j < nr) {
#pragma unroll
      for (int t = 0; t < RAD; ++t) v[q][t] = buf[b * ls + (j + t * nr) * es];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int j = tj + q * JT;
    if (active && j < nr) {
      const uint32_t jd = fdiv((uint32_t)j, nsd);
      const uint32_t k = (uint32_t)j - jd * nsd.d;
      const uint32_t step = k * tstep;
#pragma unroll
      for (int t = 1; t < RAD; ++t) {
        const cpx<R> w = tw[t * step];
        v[q][t] = INV ? cmulc(v[q][t], w) : cmul(v[q][t], w);
      }
      dft<R, INV, RAD>(v[q]);
      const uint32_t ob = jd * nsd.d * RAD + k;
#pragma unroll
      for (int u = 0; u < RAD; ++u) buf[b * ls + (ob + u * nsd.d) * es] = v[q][u];
    }
  }
  __syncthreads();
}

// One Stockham stage of run-time radix r (every radix's loads and butterflies
// behind run-time tests): fewer registers than the fixed-radix stage when a
// thread serves many butterflies (MAXB > 2: all its loads are issued together).
template <class R, int MAXB, bool INV>
__device__ __forceinline__ void lds_stage_any(cpx<R>* buf, const FftFactors& F, int s,
                                              const cpx<R>* __restrict__ tw, bool active, int b,
                                              int ls, int es, int tj, int JT) {
  const int n = F.n;
  const int r = F.radix[s];
  const int nr = n / r;
  cpx<R> v[MAXB][5];
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    int j = tj + q * JT;
    if (active && j < nr) {
#pragma unroll
      for (int t = 0; t < 5; ++t)
        if (t < r) v[q][t] = buf[b * ls + (j + t * nr) * es];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    int j = tj + q * JT;
    if (active && j < nr) {
      uint32_t jd = fdiv((uint32_t)j, F.ns[s]);
      uint32_t k = (uint32_t)j - jd * F.ns[s].d;
      uint32_t step = k * F.twstep[s];
#pragma unroll
      for (int t = 1; t < 5; ++t) {
        if (t < r) {
          cpx<R> w = tw[t * step];
          v[q][t] = INV ? cmulc(v[q][t], w) : cmul(v[q][t], w);
        }
      }
      if (r == 2) dft2<R, INV>(v[q]);
      else if (r == 3) dft3<R, INV>(v[q]);
      else if (r == 4) dft4<R, INV>(v[q]);
      else dft5<R, INV>(v[q]);
      uint32_t ob = jd * F.ns[s].d * r + k;
#pragma unroll
      for (int u = 0; u < 5; ++u)
        if (u < r) buf[b * ls + (ob + u * F.ns[s].d) * es] = v[q][u];
    }
  }
  __syncthreads();
}

// A stage of a plan fixed at compile time (length N, NS = product of the earlier
// radices): the index arithmetic folds to constants, bitwise the same results as
// lds_stage.
template <class R, int MAXB, bool INV, int RAD, int N, int NS>
__device__ __forceinline__ void lds_stage_fixed(cpx<R>* buf, const cpx<R>* __restrict__ tw,
                                                bool active, int b, int ls, int es, int tj,
                                                int JT) {
  constexpr int nr = N / RAD;
  constexpr uint32_t tstep = N / (NS * RAD);
  cpx<R> v[MAXB][RAD];
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int j = tj + q * JT;
    if (active && j < nr) {
#pragma unroll
      for (int t = 0; t < RAD; ++t) v[q][t] = buf[b * ls + (j + t * nr) * es];
    }
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < MAXB; ++q) {
    const int j = tj + q * JT;
    if (active && j < nr) {
      const uint32_t jd = (uint32_t)j / NS;
      const uint32_t k = (uint32_t)j - jd * NS;
      const uint32_t step = k * tstep;
#pragma unroll
      for (int t = 1; t < RAD; ++t) {
        const cpx<R> w = tw[t * step];
        v[q][t] = INV ? cmulc(v[q][t], w) : cmul(v[q][t], w);
      }
      dft<R, INV, RAD>(v[q]);
      const uint32_t ob = jd * NS * RAD + k;
#pragma unroll
      for (int u = 0; u < RAD; ++u) buf[b * ls + (ob + u * NS) * es] = v[q][u];
    }
  }
  __syncthreads();
}

template <int... RS>
constexpr int plan_length() {
  return (RS * ... * 1);
}
// the stages of the fixed plan RS... (NS: product of the radices before RAD)
template <class R, int MAXB, bool INV, int N, int NS, int RAD, int... REST>
__device__ __forceinline__ void lds_fixed_plan(cpx<R>* buf, const cpx<R>* __restrict__ tw,
                                               bool active, int b, int ls, int es, int tj,
                                               int JT) {
  lds_stage_fixed<R, MAXB, INV, RAD, N, NS>(buf, tw, active, b, ls, es, tj, JT);
  if constexpr (sizeof...(REST) > 0)
    lds_fixed_plan<R, MAXB, INV, N, NS * RAD, REST...>(buf, tw, active, b, ls, es, tj, JT);
}
template <int... RS>
__device__ __forceinline__ bool plan_is(const FftFactors& F) {
  constexpr int rs[] = {RS...};
  if (F.nfac != (int)sizeof...(RS)) return false;
  bool same = true;
#pragma unroll
  for (int s = 0; s < (int)sizeof...(RS); ++s) same = same && F.radix[s] == rs[s];
  return same;
}
// Runs the transform if F is the fixed plan RS...; returns whether it did.
template <class R, int MAXB, bool INV, int... RS>
__device__ __forceinline__ bool lds_try_plan(cpx<R>* buf, const FftFactors& F,
                                             const cpx<R>* __restrict__ tw, bool active, int b,
                                             int ls, int es, int tj, int JT) {
  if (!plan_is<RS...>(F)) return false;  // uniform across the block
  lds_fixed_plan<R, MAXB, INV, plan_length<RS...>(), 1, RS...>(buf, tw, active, b, ls, es, tj,
                                                                JT);
  return true;
}

// In-LDS Stockham FFT of the lines this thread group serves.
// buf element (line b, index i) lives at buf[b * ls + i * es]; this thread works
// on line `b` and on butterflies j = tj, tj + JT, ... of every stage.  All
// threads of the block must call it (it contains barriers).  Up to two
// butterflies per thread and stage (the 2D row and column passes) the stages
// are specialised by radix, and the plans of the lengths the planner picks for
// the 2D and 3D workloads (1250 = 5 5 5 5 2, 625, 250, 125) run as fixed stage
// sequences, their index arithmetic folded to constants (forward and inverse
// column FFTs of the 2D mode pass 3.4 and 2.9 -> 2.5 and 2.1 us); more
// butterflies per thread (the 3D column passes) take the run-time radix stage,
// whose registers fit.
template <class R, int MAXB, bool INV>
__device__ void lds_fft(cpx<R>* buf, const FftFactors& F, const cpx<R>* __restrict__ tw,
                        bool active, int b, int ls, int es, int tj, int JT) {
  if constexpr (MAXB <= 2) {
    if (lds_try_plan<R, MAXB, INV, 5, 5, 5, 5, 2>(buf, F, tw, active, b, ls, es, tj, JT)) return;
    if (lds_try_plan<R, MAXB, INV, 5, 5, 5, 5>(buf, F, tw, active, b, ls, es, tj, JT)) return;
    if (lds_try_plan<R, MAXB, INV, 5, 5, 5, 2>(buf, F, tw, active, b, ls, es, tj, JT)) return;
    if (lds_try_plan<R, MAXB, INV, 5, 5, 5>(buf, F, tw, active, b, ls, es, tj, JT)) return;
  }
  for (int s = 0; s < F.nfac; ++s) {
    if constexpr (MAXB <= 2) {
      switch (F.radix[s]) {
        case 2: lds_stage<R, MAXB, INV, 2>(buf, F, s, tw, active, b, ls, es, tj, JT); break;
        case 3: lds_stage<R, MAXB, INV, 3>(buf, F, s, tw, active, b, ls, es, tj, JT); break;
        case 4: lds_stage<R, MAXB, INV, 4>(buf, F, s, tw, active, b, ls, es, tj, JT); break;
        default: lds_stage<R, MAXB, INV, 5>(buf, F, s, tw, active, b, ls, es, tj, JT); break;
      }
    } else {
      lds_stage_any<R, MAXB, INV>(buf, F, s, tw, active, b, ls, es, tj, JT);
    }
  }
}

// Copy a twiddle table into LDS (all threads; followed by a barrier in caller),
// four loads in flight per thread before the first store.
template <class R>
__device__ __forceinline__ void load_twiddles(cpx<R>* dst, const cpx<R>* __restrict__ src,
                                              int n) {
  const int step = (int)blockDim.x;
  for (int i = threadIdx.x; i < n; i += 4 * step) {
    cpx<R> v[4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i + u * step < n) v[u] = src[i + u * step];
#pragma unroll
    for (int u = 0; u < 4; ++u)
      if (i + u * step < n) dst[i + u * step] = v[u];
  }
}

}  // namespace fresco
