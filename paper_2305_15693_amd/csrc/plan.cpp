// Host-side planning for the FReSCo nonuniform FFTs.
//
// Kernel choice (the FINUFFT framework of the paper's Methods, following
// Barnett, Magland & af Klinteberg): exponential of semicircle
// phi(z) = exp(beta (sqrt(1 - z^2) - 1)), width w = ceil(log10(1/tol)) + 1 grid
// cells and beta = 2.30 w at upsampling factor 2; fine grid at least twice the
// number of modes per dimension, rounded up to an even 5-smooth size.
#include "plan.h"

#include <cmath>

namespace fresco {

int next_smooth_even(long long n) {
  if (n < 2) n = 2;
  for (long long m = n + (n & 1);; m += 2) {
    long long k = m;
    for (int p : {2, 3, 5})
      while (k % p == 0) k /= p;
    if (k == 1) return (int)m;
  }
}

int kernel_width(double tol) {
  int w = (int)std::ceil(std::log10(1.0 / tol)) + 1;
  if (w < 2) w = 2;
  if (w > 16) w = 16;
  return w;
}

double kernel_beta(int w) { return 2.30 * (double)w; }

// Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_q)
static void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& wt) {
  x.resize(q);
  wt.resize(q);
  for (int i = 0; i < q; ++i) {
    double z = std::cos(M_PI * (i + 0.75) / (q + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= q; ++k) {
        double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      double dp = q * (z * p1 - p0) / (z * z - 1.0);
      double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p0 = 1.0, p1 = z;
    for (int k = 2; k <= q; ++k) {
      double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    double dp = q * (z * p1 - p0) / (z * z - 1.0);
    x[i] = z;
    wt[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

std::vector<double> kernel_fourier(int nmax, int w, double beta, int nf, bool cosh_form) {
  // z = sin(theta), theta in [-pi/2, pi/2]:
  //   int phi(z) cos(c z) dz = int phi(sin theta) cos(c sin theta) cos theta dtheta
  // with phi(sin theta) = exp(beta (cos theta - 1))            (spreading kernel)
  //   or cosh(beta cos theta) / cosh(beta)                     (interpolation kernel)
  const int q = 2 * w + 60;
  std::vector<double> x, wt;
  gauss_legendre(q, x, wt);
  const double h = 2.0 * M_PI / nf;
  const double alpha = 0.5 * w * h;
  std::vector<double> out(nmax + 1);
  std::vector<double> th(q), f(q), sn(q);
  for (int i = 0; i < q; ++i) {
    th[i] = 0.5 * M_PI * x[i];
    sn[i] = std::sin(th[i]);
    const double ct = std::cos(th[i]);
    const double ph = cosh_form ? std::exp(beta * (ct - 1.0)) * (1.0 + std::exp(-2.0 * beta * ct)) /
                                      (1.0 + std::exp(-2.0 * beta))
                                : std::exp(beta * (ct - 1.0));
    f[i] = ph * ct * wt[i] * 0.5 * M_PI;
  }
  for (int n = 0; n <= nmax; ++n) {
    double s = 0.0;
    for (int i = 0; i < q; ++i) s += f[i] * std::cos(n * alpha * sn[i]);
    out[n] = alpha * s;
  }
  return out;
}

static double kernel_value(double z, double beta, int kind) {
  const double s2 = (1.0 - z) * (1.0 + z);
  if (s2 < 0.0) return 0.0;
  const double s = std::sqrt(s2);
  if (kind == 0) return std::exp(beta * (s - 1.0));
  const double cb = std::cosh(beta);
  if (kind == 1) return std::cosh(beta * s) / cb;
  const double bs = beta * s;
  const double shs = (bs > 1e-6) ? std::sinh(bs) / s : beta * (1.0 + bs * bs / 6.0);
  return -beta * z * shs / cb;
}

std::vector<double> kernel_poly(int w, double beta, int kind, int deg) {
  const int np = deg + 1;
  std::vector<double> out((size_t)w * np, 0.0);
  std::vector<double> xk(np), fk(np), a(np);
  for (int k = 0; k < np; ++k) xk[k] = std::cos(M_PI * (k + 0.5) / np);
  for (int j = 0; j < w; ++j) {
    for (int k = 0; k < np; ++k) {
      const double tau = 0.5 * (xk[k] + 1.0);
      const double z = (tau - 0.5 * w + j) * 2.0 / w;
      fk[k] = kernel_value(z, beta, kind);
    }
    // Chebyshev coefficients of the interpolant
    for (int m = 0; m < np; ++m) {
      double s = 0.0;
      for (int k = 0; k < np; ++k) s += fk[k] * std::cos(M_PI * m * (k + 0.5) / np);
      a[m] = s * 2.0 / np;
    }
    a[0] *= 0.5;
    // sum a_m T_m(x) -> monomials, T_{m+1} = 2 x T_m - T_{m-1}
    std::vector<double> tm1(np, 0.0), tm(np, 0.0), tn(np, 0.0), c(np, 0.0);
    tm1[0] = 1.0;  // T_0
    if (np > 1) tm[1] = 1.0;  // T_1
    for (int k = 0; k < np; ++k) c[k] += a[0] * tm1[k];
    if (np > 1)
      for (int k = 0; k < np; ++k) c[k] += a[1] * tm[k];
    for (int m = 2; m < np; ++m) {
      for (int k = 0; k < np; ++k) tn[k] = -tm1[k] + ((k > 0) ? 2.0 * tm[k - 1] : 0.0);
      for (int k = 0; k < np; ++k) c[k] += a[m] * tn[k];
      tm1 = tm;
      tm = tn;
    }
    for (int k = 0; k < np; ++k) out[(size_t)j * np + k] = c[k];
  }
  return out;
}

bool plan_factors(int n, FftFactors* F, int* rmin) {
  int fac[64];
  int nf = 0;
  int m = n;
  while (m % 5 == 0) { fac[nf++] = 5; m /= 5; }
  while (m % 3 == 0) { fac[nf++] = 3; m /= 3; }
  while (m % 4 == 0) { fac[nf++] = 4; m /= 4; }
  while (m % 2 == 0) { fac[nf++] = 2; m /= 2; }
  if (m != 1 || nf > kMaxFactors) return false;
  F->n = n;
  F->nfac = nf;
  int ns = 1;
  int rm = 5;
  for (int s = 0; s < nf; ++s) {
    F->radix[s] = fac[s];
    F->ns[s] = make_fastdiv((uint32_t)ns);
    F->twstep[s] = (uint32_t)(n / (ns * fac[s]));
    ns *= fac[s];
    if (fac[s] < rm) rm = fac[s];
  }
  if (nf == 0) rm = 1;
  *rmin = rm;
  return true;
}

std::vector<double> twiddles(int n, int count) {
  std::vector<double> t(2 * (size_t)count);
  for (int q = 0; q < count; ++q) {
    double a = 2.0 * M_PI * (double)q / (double)n;
    t[2 * q] = std::cos(a);
    t[2 * q + 1] = std::sin(a);
  }
  return t;
}

}  // namespace fresco
