// Kernel evaluation shared by the per-tile spreading/interpolation passes and
// the batched small-grid evaluation.
//
// Spreading kernel: the exponential of semicircle
//   phi(z) = exp(beta (sqrt(1 - z^2) - 1)) on |z| <= 1
// (the kernel of the FINUFFT library the paper's Methods use), its support
// spanning w grid cells.  Interpolation kernel: its cosh form (finite
// derivative at the support edge), width w + 1.
#pragma once

#include "common.h"
#include "kernel_tables.h"

namespace fresco {

template <class R>
__device__ __forceinline__ R es_kernel(R z, R beta) {
  R s = (R(1) - z) * (R(1) + z);
  return s >= R(0) ? exp(beta * (sqrt(s) - R(1))) : R(0);
}

// Interpolation kernel and its derivative: phi_c(z) = cosh(beta s) / cosh(beta),
// s = sqrt(1 - z^2).  It is the exponential of semicircle up to terms of order
// exp(-2 beta s - beta), but even in s, so phi_c' = -beta z sinh(beta s) / (s cosh beta)
// stays finite at |z| = 1 (the plain exponential's derivative diverges there,
// which would make the gradient of points sitting on a grid node inaccurate).
template <class R>
__device__ __forceinline__ void cosh_kernel_d(R z, R beta, R inv_cosh_beta, R* f, R* df) {
  const R s2 = (R(1) - z) * (R(1) + z);
  if (!(s2 >= R(0))) {
    *f = R(0);
    *df = R(0);
    return;
  }
  const R s = sqrt(s2);
  const R bs = beta * s;
  const R e = exp(bs);
  const R ei = R(1) / e;
  R shs;  // sinh(beta s) / s
  if (bs > R(1e-2)) {
    shs = R(0.5) * (e - ei) / s;
  } else {
    const R b2 = bs * bs;
    shs = beta * (R(1) + b2 * (R(1) / R(6) + b2 * (R(1) / R(120))));
  }
  *f = R(0.5) * (e + ei) * inv_cosh_beta;
  *df = -beta * z * shs * inv_cosh_beta;
}

// Kernel values on the W footprint cells of one axis from tau in [0, 1):
// FP32 evaluates the per-cell polynomials in x = 2 tau - 1 (coefficients are
// compile-time literals from the generated kernel_tables.h), FP64 the closed forms.
template <class R, int W>
__device__ __forceinline__ void spread_weights(R tau, R beta, R* k) {
  if constexpr (sizeof(R) == 4) {
    tab::Poly<W>::es(2.f * tau - 1.f, k);
  } else {
    const R hw = R(2) / R(W);
#pragma unroll
    for (int i = 0; i < W; ++i) k[i] = es_kernel<R>((tau - R(0.5) * R(W) + R(i)) * hw, beta);
  }
}
// interpolation kernel (width WI) and its z-derivative
template <class R, int WI>
__device__ __forceinline__ void interp_weights(R tau, R beta, R icb, R* f, R* df) {
  if constexpr (sizeof(R) == 4) {
    const float x = 2.f * tau - 1.f;
    tab::Poly<WI>::ch(x, f);
    tab::Poly<WI>::dch(x, df);
  } else {
    const R hw = R(2) / R(WI);
#pragma unroll
    for (int i = 0; i < WI; ++i)
      cosh_kernel_d<R>((tau - R(0.5) * R(WI) + R(i)) * hw, beta, icb, f + i, df + i);
  }
}

}  // namespace fresco
