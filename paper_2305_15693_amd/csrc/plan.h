// Host-side planning: fine-grid sizes, kernel parameters, deconvolution
// factors, FFT stage plans and launch shapes.
#pragma once

#include <vector>

#include "common.h"

namespace fresco {

// smallest even integer >= n whose only prime factors are 2, 3 and 5
int next_smooth_even(long long n);

// kernel width for a requested accuracy at upsampling 2 (w = ceil(log10 1/tol) + 1)
int kernel_width(double tol);

// ES shape parameter at upsampling 2
double kernel_beta(int w);

// psihat(n) = alpha * int_{-1}^{1} phi(z) cos(n alpha z) dz with alpha = w h / 2,
// h = 2 pi / nf, for n = 0..nmax (FP64 Gauss-Legendre in z = sin(theta), where
// the integrand is smooth).  phi is the exponential of semicircle, or with
// cosh_form its even-in-sqrt(1 - z^2) variant cosh(beta sqrt(1 - z^2)) / cosh(beta).
std::vector<double> kernel_fourier(int nmax, int w, double beta, int nf, bool cosh_form);

// Piecewise-polynomial form of a kernel for fast evaluation.  For a point with
// footprint offset tau in [0, 1) (tau = t + w/2), the value on footprint cell j is
// phi(z_j), z_j = (tau - w/2 + j) 2 / w.  Returns, for each j, the monomial
// coefficients c[j][0..deg] of the degree-deg Chebyshev interpolant of phi(z_j)
// in x = 2 tau - 1 (row-major, w x (deg + 1)).
// kind: 0 exponential of semicircle, 1 cosh form, 2 derivative d/dz of the cosh form.
std::vector<double> kernel_poly(int w, double beta, int kind, int deg);

// radix plan of a complex FFT of length n (radices 2, 3, 4, 5); false if n has
// another prime factor or needs too many stages
bool plan_factors(int n, FftFactors* F, int* rmin);

// exp(+2 pi i q / n) for q in [0, count)
std::vector<double> twiddles(int n, int count);

}  // namespace fresco
