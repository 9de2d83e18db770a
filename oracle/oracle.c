/*
 * oracle.c -- FP64 CPU oracle for the FReSCo structure-factor loss and its
 * position gradient (Shih, Casiulis & Martiniani, "Fast Generation of
 * Spectrally-Shaped Disorder", arXiv 2305.15693).
 *
 * TEST INFRASTRUCTURE ONLY.  This file exists so that tests, the smoke check
 * and the CPU-baseline leg of the benchmark have an independent, plainly
 * correct reference.  The product (the HIP library) never links, loads or
 * calls it, and it shares no code, header, table or constant with the HIP
 * path.
 *
 * Everything is evaluated by direct sums straight from the definitions; no
 * nonuniform FFT, no grids, no approximation:
 *
 *   rho(k)  = sum_j c_j exp(+i k.r_j)                 (Methods, Eq. ft; c_j = 1)
 *   S(k)    = |rho(k)|^2 / N                          (Eq. structure_factor)
 *   L       = sum_{k in K} W(k) (S(k) - S0(k))^2      (Methods, loss with W)
 *   C_a(k)  = -4 i k_a W(k) (S(k) - S0(k)) rho(k) / N
 *   dL/dr_ja = Re sum_{k in K} C_a(k) exp(-i k.r_j)   (Eq. gradient /
 *                                                      Eq. losspositiongradient)
 *
 * Wave vectors are k = 2 pi n / L_a for integer mode vectors n; the caller
 * passes the constrained set K as an explicit list of mode vectors (the full
 * set, both n and -n, exactly as the sum in the loss runs).  Positions are read
 * exactly as given (fp32 inputs are widened to fp64 by the caller, which is
 * exact) and are not wrapped: exp(i k.r) has period L in every coordinate.
 *
 * The per-point factors exp(i 2 pi m r_a / L_a), m = -M..M, are taken from
 * direct libm cos/sin calls (no recurrences), and the multi-dimensional
 * exponential is their product, which is the same number up to rounding.
 *
 * Determinism: points are processed in fixed blocks; within a block each mode
 * is owned by one thread and summed in point order, so results do not depend
 * on the thread count.
 *
 * Pinning: see tests/test_oracle_pins.py (lattice Bragg values, N=1 and N=2
 * closed forms, the pair form of S, Friedel/translation/permutation
 * invariance, the gradient sum rule, Poisson statistics and finite
 * differences).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_OK 0
#define OR_EINVAL -1
#define OR_ENOMEM -2

static const double TWO_PI = 6.283185307179586476925286766559;

int oracle_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* largest |n_a| over the mode list, per dimension */
static void mode_extent(int d, long long K, const int* modes, int* M) {
  for (int a = 0; a < 3; ++a) M[a] = 0;
  for (long long q = 0; q < K; ++q)
    for (int a = 0; a < d; ++a) {
      int v = modes[q * d + a];
      if (v < 0) v = -v;
      if (v > M[a]) M[a] = v;
    }
}

/* table for one point: tab[a][m + M_a] = exp(i 2 pi m r_a / L_a), m in [-M_a, M_a]
 * layout: re/im interleaved; offsets off[a] into the point's table. */
static void point_table(int d, const double* L, const double* r, const int* M,
                        const long long* off, double* tab) {
  for (int a = 0; a < d; ++a) {
    double* t = tab + 2 * off[a];
    for (int m = -M[a]; m <= M[a]; ++m) {
      double ph = TWO_PI * (double)m * r[a] / L[a];
      t[2 * (m + M[a])] = cos(ph);
      t[2 * (m + M[a]) + 1] = sin(ph);
    }
  }
}

/* exp(i k.r) for mode n from the point's table: product over dimensions */
static inline void mode_exp(int d, const int* n, const int* M, const long long* off,
                            const double* tab, double* re, double* im) {
  double pr = 1.0, pi = 0.0;
  for (int a = 0; a < d; ++a) {
    const double* t = tab + 2 * (off[a] + n[a] + M[a]);
    double xr = pr * t[0] - pi * t[1];
    double xi = pr * t[1] + pi * t[0];
    pr = xr;
    pi = xi;
  }
  *re = pr;
  *im = pi;
}

#define BLOCK 512

/* rho(k) = sum_j c_j exp(+i k.r_j) over the listed modes (c NULL: c_j = 1);
 * rho is [K][2] (re, im). */
static int rho_impl(int d, long long N, const double* L, const double* pos, const double* c,
                    long long K, const int* modes, double* rho) {
  if (d < 1 || d > 3 || N < 0 || K < 0 || !L || (N && !pos) || (K && (!modes || !rho)))
    return OR_EINVAL;
  int M[3];
  mode_extent(d, K, modes, M);
  long long off[3], tlen = 0;
  for (int a = 0; a < d; ++a) { off[a] = tlen; tlen += 2 * M[a] + 1; }
  double* tabs = (double*)malloc(sizeof(double) * 2 * tlen * BLOCK);
  if (!tabs) return OR_ENOMEM;
  for (long long q = 0; q < 2 * K; ++q) rho[q] = 0.0;
  for (long long j0 = 0; j0 < N; j0 += BLOCK) {
    long long nb = (N - j0 < BLOCK) ? N - j0 : BLOCK;
#pragma omp parallel for schedule(static)
    for (long long b = 0; b < nb; ++b)
      point_table(d, L, pos + (j0 + b) * d, M, off, tabs + 2 * tlen * b);
#pragma omp parallel for schedule(static)
    for (long long q = 0; q < K; ++q) {
      double sr = 0.0, si = 0.0;
      for (long long b = 0; b < nb; ++b) {
        double er, ei;
        mode_exp(d, modes + q * d, M, off, tabs + 2 * tlen * b, &er, &ei);
        const double cj = c ? c[j0 + b] : 1.0;
        sr += cj * er;
        si += cj * ei;
      }
      rho[2 * q] += sr;
      rho[2 * q + 1] += si;
    }
  }
  free(tabs);
  return OR_OK;
}

int oracle_rho(int d, long long N, const double* L, const double* pos, long long K,
               const int* modes, double* rho) {
  return rho_impl(d, N, L, pos, NULL, K, modes, rho);
}

int oracle_rho_c(int d, long long N, const double* L, const double* pos, const double* c,
                 long long K, const int* modes, double* rho) {
  if (!c) return OR_EINVAL;
  return rho_impl(d, N, L, pos, c, K, modes, rho);
}

/*
 * Loss and gradient from the definitions.
 *   W, S0       : per listed mode (W already includes any 1/S0^2 normalisation)
 *   S_out       : [K] structure factor (may be NULL)
 *   rho_out     : [K][2] (may be NULL)
 *   loss_out    : scalar (may be NULL)
 *   G, gidx     : gradient wanted for points gidx[0..G) (gidx NULL: points 0..G-1)
 *   grad_out    : [G][d] (may be NULL)
 */
int oracle_loss_grad(int d, long long N, const double* L, const double* pos, long long K,
                     const int* modes, const double* W, const double* S0, double* S_out,
                     double* rho_out, double* loss_out, long long G, const long long* gidx,
                     double* grad_out) {
  if (d < 1 || d > 3 || N <= 0 || K < 0 || !L || !pos || (K && (!modes || !W || !S0)))
    return OR_EINVAL;
  if (G < 0 || (G && !grad_out)) return OR_EINVAL;
  double* rho = (double*)malloc(sizeof(double) * 2 * (K ? K : 1));
  double* C = (double*)malloc(sizeof(double) * 2 * d * (K ? K : 1));
  if (!rho || !C) { free(rho); free(C); return OR_ENOMEM; }
  int st = oracle_rho(d, N, L, pos, K, modes, rho);
  if (st) { free(rho); free(C); return st; }
  double loss = 0.0;
  for (long long q = 0; q < K; ++q) {
    double S = (rho[2 * q] * rho[2 * q] + rho[2 * q + 1] * rho[2 * q + 1]) / (double)N;
    double res = S - S0[q];
    loss += W[q] * res * res;
    if (S_out) S_out[q] = S;
    /* C_a = -4 i k_a W res rho / N  =  (4 k_a W res / N) * (-i rho) */
    for (int a = 0; a < d; ++a) {
      double ka = TWO_PI * (double)modes[q * d + a] / L[a];
      double f = 4.0 * ka * W[q] * res / (double)N;
      C[2 * (q * d + a)] = f * rho[2 * q + 1];      /* Re(-i rho) = Im rho */
      C[2 * (q * d + a) + 1] = -f * rho[2 * q];     /* Im(-i rho) = -Re rho */
    }
  }
  if (rho_out) memcpy(rho_out, rho, sizeof(double) * 2 * K);
  if (loss_out) *loss_out = loss;
  if (G && grad_out) {
    int M[3];
    mode_extent(d, K, modes, M);
    long long off[3], tlen = 0;
    for (int a = 0; a < d; ++a) { off[a] = tlen; tlen += 2 * M[a] + 1; }
    int fail = 0;
#pragma omp parallel
    {
      double* tab = (double*)malloc(sizeof(double) * 2 * tlen);
      if (!tab) {
#pragma omp atomic write
        fail = 1;
      } else {
#pragma omp for schedule(dynamic, 16)
        for (long long g = 0; g < G; ++g) {
          long long j = gidx ? gidx[g] : g;
          double acc[3] = {0.0, 0.0, 0.0};
          if (j >= 0 && j < N) {
            point_table(d, L, pos + j * d, M, off, tab);
            for (long long q = 0; q < K; ++q) {
              double er, ei; /* exp(+i k.r_j); exp(-i k.r_j) is its conjugate */
              mode_exp(d, modes + q * d, M, off, tab, &er, &ei);
              for (int a = 0; a < d; ++a) {
                const double* c = C + 2 * (q * d + a);
                /* Re[c * (er - i ei)] = c_re er + c_im ei */
                acc[a] += c[0] * er + c[1] * ei;
              }
            }
          }
          for (int a = 0; a < d; ++a) grad_out[g * d + a] = acc[a];
        }
        free(tab);
      }
    }
    if (fail) { free(rho); free(C); return OR_ENOMEM; }
  }
  free(rho);
  free(C);
  return OR_OK;
}

/*
 * Central finite differences of L along single coordinates, computed without
 * cancellation: moving r_ja by +-h changes rho(k) by
 *   delta_pm(k) = exp(i k.r_j) (exp(+-i k_a h) - 1),
 * with exp(i t) - 1 = -2 sin^2(t/2) + i sin t, so that
 *   S_pm - S   = [2 Re(conj(rho) delta_pm) + |delta_pm|^2] / N,
 *   L_+ - L_-  = sum_k W (S_+ - S_-) (S_+ + S_- - 2 S0).
 * out[c] = (L_+ - L_-) / (2h) for coordinate (cj[c], ca[c]).
 */
int oracle_fd(int d, long long N, const double* L, const double* pos, long long K,
              const int* modes, const double* W, const double* S0, long long nc,
              const long long* cj, const int* ca, double h, double* out) {
  if (d < 1 || d > 3 || N <= 0 || K < 0 || !L || !pos || nc < 0 || (nc && (!cj || !ca || !out)))
    return OR_EINVAL;
  double* rho = (double*)malloc(sizeof(double) * 2 * (K ? K : 1));
  if (!rho) return OR_ENOMEM;
  int st = oracle_rho(d, N, L, pos, K, modes, rho);
  if (st) { free(rho); return st; }
  int M[3];
  mode_extent(d, K, modes, M);
  long long off[3], tlen = 0;
  for (int a = 0; a < d; ++a) { off[a] = tlen; tlen += 2 * M[a] + 1; }
  int fail = 0;
#pragma omp parallel
  {
    double* tab = (double*)malloc(sizeof(double) * 2 * tlen);
    if (!tab) {
#pragma omp atomic write
      fail = 1;
    } else {
#pragma omp for schedule(dynamic, 1)
      for (long long c = 0; c < nc; ++c) {
        long long j = cj[c];
        int a = ca[c];
        double dl = 0.0;
        if (j >= 0 && j < N && a >= 0 && a < d) {
          point_table(d, L, pos + j * d, M, off, tab);
          for (long long q = 0; q < K; ++q) {
            double er, ei;
            mode_exp(d, modes + q * d, M, off, tab, &er, &ei);
            double ka = TWO_PI * (double)modes[q * d + a] / L[a];
            double t = ka * h;
            double s2 = sin(0.5 * t);
            double cm1 = -2.0 * s2 * s2; /* cos t - 1 */
            double sn = sin(t);
            /* delta_+ = e (cm1 + i sn), delta_- = e (cm1 - i sn) */
            double dpr = er * cm1 - ei * sn, dpi = er * sn + ei * cm1;
            double dmr = er * cm1 + ei * sn, dmi = -er * sn + ei * cm1;
            double rr = rho[2 * q], ri = rho[2 * q + 1];
            double Sp_minus_S = (2.0 * (rr * dpr + ri * dpi) + dpr * dpr + dpi * dpi) / (double)N;
            double Sm_minus_S = (2.0 * (rr * dmr + ri * dmi) + dmr * dmr + dmi * dmi) / (double)N;
            double S = (rr * rr + ri * ri) / (double)N;
            double dS = Sp_minus_S - Sm_minus_S;
            double sumS = 2.0 * S + Sp_minus_S + Sm_minus_S;
            dl += W[q] * dS * (sumS - 2.0 * S0[q]);
          }
        }
        out[c] = dl / (2.0 * h);
      }
      free(tab);
    }
  }
  free(rho);
  return fail ? OR_ENOMEM : OR_OK;
}

/*
 * Real point strengths c_j (Methods, "Analytical gradients": the density field
 * sum_j c_j delta(r - r_j); polydisperse packings weigh each particle by its
 * volume over the mean volume):
 *   rho(k)    = sum_j c_j exp(+i k.r_j),   rho0 = sum_j c_j^2,
 *   S(k)      = |rho(k)|^2 / rho0,         L = sum_K W (S - S0)^2,
 *   dS/dr_j   = (2 / rho0) Re[-i k c_j rho(k) exp(-i k.r_j)]
 *   dL/dr_j   = c_j Re sum_K C(k) exp(-i k.r_j),   C(k) = -4 i k W (S - S0) rho / rho0
 *   dS/dc_j   = (2 / rho0) Re[rho(k) exp(-i k.r_j)] - (2 c_j / rho0) S(k)   (Eq. weightgradient)
 *   dL/dc_j   = Re sum_K Cc(k) exp(-i k.r_j) - Fc_j,                        (Eq. lossweightgradient)
 *               Cc = 4 W (S - S0) rho / rho0,  Fc_j = (4 c_j / rho0) sum_K W S (S - S0).
 * With c_j = 1 everything reduces to the functions above (rho0 = N).  The
 * position gradient divides by rho0, the normalisation of S with strengths;
 * the paper writes N there, the two agreeing for unit strengths.
 *   grad_pos [G][d], grad_c [G] (either may be NULL) for the points gidx[0..G)
 *   (gidx NULL: 0..G-1).
 */
int oracle_loss_grad_c(int d, long long N, const double* L, const double* pos, const double* c,
                       long long K, const int* modes, const double* W, const double* S0,
                       double* S_out, double* loss_out, long long G, const long long* gidx,
                       double* grad_pos, double* grad_c) {
  if (d < 1 || d > 3 || N <= 0 || K < 0 || !L || !pos || !c || (K && (!modes || !W || !S0)))
    return OR_EINVAL;
  if (G < 0) return OR_EINVAL;
  double rho0 = 0.0;
  for (long long j = 0; j < N; ++j) rho0 += c[j] * c[j];
  if (!(rho0 > 0.0)) return OR_EINVAL;
  double* rho = (double*)malloc(sizeof(double) * 2 * (K ? K : 1));
  double* C = (double*)malloc(sizeof(double) * 2 * (d + 1) * (K ? K : 1));
  if (!rho || !C) { free(rho); free(C); return OR_ENOMEM; }
  int st = rho_impl(d, N, L, pos, c, K, modes, rho);
  if (st) { free(rho); free(C); return st; }
  double loss = 0.0, fsum = 0.0;
  for (long long q = 0; q < K; ++q) {
    double S = (rho[2 * q] * rho[2 * q] + rho[2 * q + 1] * rho[2 * q + 1]) / rho0;
    double res = S - S0[q];
    loss += W[q] * res * res;
    fsum += W[q] * S * res;
    if (S_out) S_out[q] = S;
    double* Cq = C + 2 * (d + 1) * q;
    /* C_a = -4 i k_a W res rho / rho0 = (4 k_a W res / rho0) (-i rho) */
    for (int a = 0; a < d; ++a) {
      double ka = TWO_PI * (double)modes[q * d + a] / L[a];
      double f = 4.0 * ka * W[q] * res / rho0;
      Cq[2 * a] = f * rho[2 * q + 1];
      Cq[2 * a + 1] = -f * rho[2 * q];
    }
    /* Cc = 4 W res rho / rho0 */
    Cq[2 * d] = 4.0 * W[q] * res / rho0 * rho[2 * q];
    Cq[2 * d + 1] = 4.0 * W[q] * res / rho0 * rho[2 * q + 1];
  }
  if (loss_out) *loss_out = loss;
  if (G && (grad_pos || grad_c)) {
    int M[3];
    mode_extent(d, K, modes, M);
    long long off[3], tlen = 0;
    for (int a = 0; a < d; ++a) { off[a] = tlen; tlen += 2 * M[a] + 1; }
    int fail = 0;
#pragma omp parallel
    {
      double* tab = (double*)malloc(sizeof(double) * 2 * tlen);
      if (!tab) {
#pragma omp atomic write
        fail = 1;
      } else {
#pragma omp for schedule(dynamic, 16)
        for (long long g = 0; g < G; ++g) {
          long long j = gidx ? gidx[g] : g;
          double acc[4] = {0.0, 0.0, 0.0, 0.0};
          if (j >= 0 && j < N) {
            point_table(d, L, pos + j * d, M, off, tab);
            for (long long q = 0; q < K; ++q) {
              double er, ei;
              mode_exp(d, modes + q * d, M, off, tab, &er, &ei);
              const double* Cq = C + 2 * (d + 1) * q;
              /* Re[x (er - i ei)] = x_re er + x_im ei */
              for (int a = 0; a <= d; ++a) acc[a] += Cq[2 * a] * er + Cq[2 * a + 1] * ei;
            }
          }
          const double cj = (j >= 0 && j < N) ? c[j] : 0.0;
          if (grad_pos)
            for (int a = 0; a < d; ++a) grad_pos[g * d + a] = cj * acc[a];
          if (grad_c) grad_c[g] = acc[d] - 4.0 * cj / rho0 * fsum;
        }
        free(tab);
      }
    }
    if (fail) { free(rho); free(C); return OR_ENOMEM; }
  }
  free(rho);
  free(C);
  return OR_OK;
}

/*
 * Cancellation-free central differences with strengths.  Coordinate entries
 * ca[c] in 0..d-1 move position r_{j,a} by +-h:
 *   delta_pm = c_j exp(i k.r_j) (exp(+-i k_a h) - 1),  S_pm - S = [2 Re(conj(rho) delta_pm) + |delta_pm|^2] / rho0;
 * ca[c] = d moves the strength c_j by +-h, which also changes rho0:
 *   rho_pm = rho +- h e,  rho0_pm = rho0 +- 2 h c_j + h^2,
 *   S_pm - S = [rho0 (+-2 h Re(conj(rho) e) + h^2) - |rho|^2 (+-2 h c_j + h^2)] / (rho0 rho0_pm).
 * Then L_+ - L_- = sum_K W (S_+ - S_-) (S_+ + S_- - 2 S0); out[c] = (L_+ - L_-) / 2h.
 */
int oracle_fd_c(int d, long long N, const double* L, const double* pos, const double* c,
                long long K, const int* modes, const double* W, const double* S0, long long nc,
                const long long* cj, const int* ca, double h, double* out) {
  if (d < 1 || d > 3 || N <= 0 || K < 0 || !L || !pos || !c || nc < 0 ||
      (nc && (!cj || !ca || !out)))
    return OR_EINVAL;
  double rho0 = 0.0;
  for (long long j = 0; j < N; ++j) rho0 += c[j] * c[j];
  if (!(rho0 > 0.0)) return OR_EINVAL;
  double* rho = (double*)malloc(sizeof(double) * 2 * (K ? K : 1));
  if (!rho) return OR_ENOMEM;
  int st = rho_impl(d, N, L, pos, c, K, modes, rho);
  if (st) { free(rho); return st; }
  int M[3];
  mode_extent(d, K, modes, M);
  long long off[3], tlen = 0;
  for (int a = 0; a < d; ++a) { off[a] = tlen; tlen += 2 * M[a] + 1; }
  int fail = 0;
#pragma omp parallel
  {
    double* tab = (double*)malloc(sizeof(double) * 2 * tlen);
    if (!tab) {
#pragma omp atomic write
      fail = 1;
    } else {
#pragma omp for schedule(dynamic, 1)
      for (long long q0 = 0; q0 < nc; ++q0) {
        long long j = cj[q0];
        int a = ca[q0];
        double dl = 0.0;
        if (j >= 0 && j < N && a >= 0 && a <= d) {
          point_table(d, L, pos + j * d, M, off, tab);
          for (long long q = 0; q < K; ++q) {
            double er, ei;
            mode_exp(d, modes + q * d, M, off, tab, &er, &ei);
            double rr = rho[2 * q], ri = rho[2 * q + 1];
            double r2 = rr * rr + ri * ri;
            double S = r2 / rho0, dSp, dSm;
            if (a < d) {
              double ka = TWO_PI * (double)modes[q * d + a] / L[a];
              double t = ka * h;
              double s2 = sin(0.5 * t);
              double cm1 = -2.0 * s2 * s2;
              double sn = sin(t);
              double ecr = c[j] * er, eci = c[j] * ei;
              double dpr = ecr * cm1 - eci * sn, dpi = ecr * sn + eci * cm1;
              double dmr = ecr * cm1 + eci * sn, dmi = -ecr * sn + eci * cm1;
              dSp = (2.0 * (rr * dpr + ri * dpi) + dpr * dpr + dpi * dpi) / rho0;
              dSm = (2.0 * (rr * dmr + ri * dmi) + dmr * dmr + dmi * dmi) / rho0;
            } else {
              double re = rr * er + ri * ei; /* Re(conj(rho) e) */
              double r0p = rho0 + 2.0 * h * c[j] + h * h, r0m = rho0 - 2.0 * h * c[j] + h * h;
              dSp = (rho0 * (2.0 * h * re + h * h) - r2 * (2.0 * h * c[j] + h * h)) / (rho0 * r0p);
              dSm = (rho0 * (-2.0 * h * re + h * h) - r2 * (-2.0 * h * c[j] + h * h)) / (rho0 * r0m);
            }
            dl += W[q] * (dSp - dSm) * (2.0 * S + dSp + dSm - 2.0 * S0[q]);
          }
        }
        out[q0] = dl / (2.0 * h);
      }
      free(tab);
    }
  }
  free(rho);
  return fail ? OR_ENOMEM : OR_OK;
}

/*
 * Non-uniform wave vectors (Methods, the NUwNU variant and the Ewald
 * construction: free boundary conditions, constraints at any continuous q):
 *   rho(q) = sum_j c_j exp(+i q.r_j) at the listed q [K][d] (c NULL: c_j = 1),
 * by direct sums with libm cos/sin of the FP64 phase q.r_j (positions as given,
 * no wrapping).  rho [K][2].
 */
int oracle_rho_q(int d, long long N, const double* pos, const double* c, long long K,
                 const double* q, double* rho) {
  if (d < 1 || d > 3 || N < 0 || K < 0 || (N && !pos) || (K && (!q || !rho))) return OR_EINVAL;
#pragma omp parallel for schedule(dynamic, 1)
  for (long long k = 0; k < K; ++k) {
    double sr = 0.0, si = 0.0;
    for (long long j = 0; j < N; ++j) {
      double ph = 0.0;
      for (int a = 0; a < d; ++a) ph += q[k * d + a] * pos[j * d + a];
      const double cj = c ? c[j] : 1.0;
      sr += cj * cos(ph);
      si += cj * sin(ph);
    }
    rho[2 * k] = sr;
    rho[2 * k + 1] = si;
  }
  return OR_OK;
}

/*
 * Loss over non-uniform wave vectors and its position gradient:
 *   S_k = |rho(q_k)|^2 / rho0 (rho0 = sum c^2, N for unit strengths),
 *   L = sum_k W_k (S_k - S0_k)^2,
 *   dL/dr_j = c_j sum_k (4 W_k (S_k - S0_k) / rho0) q_k Re[i conj(rho_k) exp(i q_k.r_j)].
 * S_out [K], grad [N][d] (either may be NULL).
 */
int oracle_loss_grad_q(int d, long long N, const double* pos, const double* c, long long K,
                       const double* q, const double* W, const double* S0, double* S_out,
                       double* loss_out, double* grad) {
  if (d < 1 || d > 3 || N <= 0 || K < 0 || !pos || (K && (!q || !W || !S0))) return OR_EINVAL;
  double rho0 = 0.0;
  for (long long j = 0; j < N; ++j) rho0 += c ? c[j] * c[j] : 1.0;
  if (!(rho0 > 0.0)) return OR_EINVAL;
  double* rho = (double*)malloc(sizeof(double) * 2 * (K ? K : 1));
  double* A = (double*)malloc(sizeof(double) * 2 * (K ? K : 1));
  if (!rho || !A) { free(rho); free(A); return OR_ENOMEM; }
  int st = oracle_rho_q(d, N, pos, c, K, q, rho);
  if (st) { free(rho); free(A); return st; }
  double loss = 0.0;
  for (long long k = 0; k < K; ++k) {
    const double S = (rho[2 * k] * rho[2 * k] + rho[2 * k + 1] * rho[2 * k + 1]) / rho0;
    const double res = S - S0[k];
    loss += W[k] * res * res;
    if (S_out) S_out[k] = S;
    const double f = 4.0 * W[k] * res / rho0;
    A[2 * k] = f * rho[2 * k];       /* f conj(rho): re */
    A[2 * k + 1] = -f * rho[2 * k + 1]; /* im */
  }
  if (loss_out) *loss_out = loss;
  if (grad) {
#pragma omp parallel for schedule(static)
    for (long long j = 0; j < N; ++j) {
      double acc[3] = {0.0, 0.0, 0.0};
      for (long long k = 0; k < K; ++k) {
        double ph = 0.0;
        for (int a = 0; a < d; ++a) ph += q[k * d + a] * pos[j * d + a];
        const double er = cos(ph), ei = sin(ph);
        /* Re[i A e] = -Im[A e] = -(A_re ei + A_im er) */
        const double v = -(A[2 * k] * ei + A[2 * k + 1] * er);
        for (int a = 0; a < d; ++a) acc[a] += q[k * d + a] * v;
      }
      const double cj = c ? c[j] : 1.0;
      for (int a = 0; a < d; ++a) grad[j * d + a] = cj * acc[a];
    }
  }
  free(rho);
  free(A);
  return OR_OK;
}

/*
 * Gradient of the loss over arbitrary wave vectors with respect to real
 * strengths (Methods, Eq. lossweightgradient; the UwU / UwNU variants optimise
 * the weights of fixed points, e.g. the pixels of a uniform grid):
 *   dL/dc_j = Re sum_k Cc_k exp(-i q_k.r_j) - (4 c_j / rho0) sum_k W_k S_k (S_k - S0_k),
 *   Cc_k = 4 W_k (S_k - S0_k) rho_k / rho0.      grad_c [N].
 */
int oracle_grad_c_q(int d, long long N, const double* pos, const double* c, long long K,
                    const double* q, const double* W, const double* S0, double* grad_c) {
  if (d < 1 || d > 3 || N <= 0 || K < 0 || !pos || !c || !grad_c || (K && (!q || !W || !S0)))
    return OR_EINVAL;
  double rho0 = 0.0;
  for (long long j = 0; j < N; ++j) rho0 += c[j] * c[j];
  if (!(rho0 > 0.0)) return OR_EINVAL;
  double* rho = (double*)malloc(sizeof(double) * 2 * (K ? K : 1));
  if (!rho) return OR_ENOMEM;
  int st = oracle_rho_q(d, N, pos, c, K, q, rho);
  if (st) { free(rho); return st; }
  double fsum = 0.0;
  for (long long k = 0; k < K; ++k) {
    const double S = (rho[2 * k] * rho[2 * k] + rho[2 * k + 1] * rho[2 * k + 1]) / rho0;
    const double res = S - S0[k];
    fsum += W[k] * S * res;
    const double f = 4.0 * W[k] * res / rho0;
    rho[2 * k] *= f; /* Cc_k */
    rho[2 * k + 1] *= f;
  }
#pragma omp parallel for schedule(static)
  for (long long j = 0; j < N; ++j) {
    double acc = 0.0;
    for (long long k = 0; k < K; ++k) {
      double ph = 0.0;
      for (int a = 0; a < d; ++a) ph += q[k * d + a] * pos[j * d + a];
      /* Re[Cc (cos - i sin)] = Cc_re cos + Cc_im sin */
      acc += rho[2 * k] * cos(ph) + rho[2 * k + 1] * sin(ph);
    }
    grad_c[j] = acc - 4.0 * c[j] / rho0 * fsum;
  }
  free(rho);
  return OR_OK;
}

/*
 * Vector-Jacobian product of the structure factor (the derivative of S with
 * respect to a position, Methods, "Analytical gradients"):
 *   dS(k)/dr_ja = (2/N) Re[conj(rho(k)) i k_a exp(i k.r_j)]
 *               = (2 k_a / N) (Im rho Re e - Re rho Im e),   e = exp(i k.r_j),
 *   grad_ja     = sum_{listed k} gS(k) dS(k)/dr_ja.
 *   gS          : [K] weights of the listed modes
 *   G, gidx     : points wanted (gidx NULL: points 0..G-1); grad_out [G][d]
 */
int oracle_sf_vjp(int d, long long N, const double* L, const double* pos, long long K,
                  const int* modes, const double* gS, long long G, const long long* gidx,
                  double* grad_out) {
  if (d < 1 || d > 3 || N <= 0 || K < 0 || !L || !pos || (K && (!modes || !gS)))
    return OR_EINVAL;
  if (G < 0 || (G && !grad_out)) return OR_EINVAL;
  double* rho = (double*)malloc(sizeof(double) * 2 * (K ? K : 1));
  if (!rho) return OR_ENOMEM;
  int st = oracle_rho(d, N, L, pos, K, modes, rho);
  if (st) { free(rho); return st; }
  int M[3];
  mode_extent(d, K, modes, M);
  long long off[3], tlen = 0;
  for (int a = 0; a < d; ++a) { off[a] = tlen; tlen += 2 * M[a] + 1; }
  int fail = 0;
#pragma omp parallel
  {
    double* tab = (double*)malloc(sizeof(double) * 2 * tlen);
    if (!tab) {
#pragma omp atomic write
      fail = 1;
    } else {
#pragma omp for schedule(dynamic, 16)
      for (long long g = 0; g < G; ++g) {
        long long j = gidx ? gidx[g] : g;
        double acc[3] = {0.0, 0.0, 0.0};
        if (j >= 0 && j < N) {
          point_table(d, L, pos + j * d, M, off, tab);
          for (long long q = 0; q < K; ++q) {
            double er, ei;
            mode_exp(d, modes + q * d, M, off, tab, &er, &ei);
            const double im = rho[2 * q + 1] * er - rho[2 * q] * ei;
            for (int a = 0; a < d; ++a) {
              double ka = TWO_PI * (double)modes[q * d + a] / L[a];
              acc[a] += gS[q] * 2.0 * ka / (double)N * im;
            }
          }
        }
        for (int a = 0; a < d; ++a) grad_out[g * d + a] = acc[a];
      }
      free(tab);
    }
  }
  free(rho);
  return fail ? OR_ENOMEM : OR_OK;
}

/*
 * Soft-core pair repulsion (the short-range term added to the spectral loss
 * for packings, Results, "Stealthy hyperuniform packings"):
 *   U(r) = (eps / alpha) (1 - r / sigma)^alpha  for r < sigma, else 0,
 *   E    = sum_{i<j} U(|r_i - r_j|),  distances under the minimum image
 *          convention of the periodic box (requires sigma < L_a / 2),
 *   dE/dr_i = sum_{j != i} U'(r_ij) (r_i - r_j) / r_ij,
 *   U'(r) = -(eps / sigma) (1 - r / sigma)^(alpha - 1).
 * Coincident points (r = 0) have no direction and contribute energy only.
 *
 * oracle_pair        : brute force over all pairs, O(N^2).
 * oracle_pair_cells  : the same sums over a cell list (cells of side >= sigma),
 *                      for large N; checked against the brute force in tests.
 * Both write energy (scalar) and grad [N][d]; each point's sum runs over its
 * partners in increasing index order.
 */
static inline double min_image(double x, double L) { return x - L * nearbyint(x / L); }

static inline void pair_term(int d, const double* L, const double* ri, const double* rj,
                             double sigma, double eps, double alpha, double* u, double* g) {
  double dx[3], r2 = 0.0;
  for (int a = 0; a < d; ++a) {
    dx[a] = min_image(ri[a] - rj[a], L[a]);
    r2 += dx[a] * dx[a];
  }
  *u = 0.0;
  for (int a = 0; a < d; ++a) g[a] = 0.0;
  if (r2 >= sigma * sigma) return;
  double r = sqrt(r2);
  double x = 1.0 - r / sigma;
  *u = eps / alpha * pow(x, alpha);
  if (r > 0.0) {
    double du = -eps / sigma * pow(x, alpha - 1.0);
    for (int a = 0; a < d; ++a) g[a] = du * dx[a] / r;
  }
}

static int pair_check(int d, long long N, const double* L, const double* pos, double sigma,
                      double alpha) {
  if (d < 1 || d > 3 || N < 0 || !L || (N && !pos) || !(sigma > 0.0) || !(alpha >= 1.0))
    return OR_EINVAL;
  for (int a = 0; a < d; ++a)
    if (!(L[a] > 2.0 * sigma)) return OR_EINVAL;
  return OR_OK;
}

int oracle_pair(int d, long long N, const double* L, const double* pos, double sigma, double eps,
                double alpha, double* energy, double* grad) {
  int st = pair_check(d, N, L, pos, sigma, alpha);
  if (st) return st;
  double e = 0.0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : e)
  for (long long i = 0; i < N; ++i) {
    double acc[3] = {0.0, 0.0, 0.0}, ei = 0.0;
    for (long long j = 0; j < N; ++j) {
      if (j == i) continue;
      double u, g[3];
      pair_term(d, L, pos + i * d, pos + j * d, sigma, eps, alpha, &u, g);
      ei += u;
      for (int a = 0; a < d; ++a) acc[a] += g[a];
    }
    e += 0.5 * ei;
    if (grad)
      for (int a = 0; a < d; ++a) grad[i * d + a] = acc[a];
  }
  if (energy) *energy = e;
  return OR_OK;
}

/*
 * Central difference of the pair energy in single coordinates, by brute force:
 * moving point j along axis a changes only the pairs (i, j), so
 *   (E(r_ja + h) - E(r_ja - h)) / 2h = sum_{i != j} (U(r+_ij) - U(r-_ij)) / 2h,
 * each pair's difference taken directly (no difference of two large totals).
 * O(N) per coordinate.  cj, ca: the nc coordinates (point, axis); out [nc].
 */
int oracle_pair_fd(int d, long long N, const double* L, const double* pos, double sigma,
                   double eps, double alpha, long long nc, const long long* cj, const int* ca,
                   double h, double* out) {
  int st = pair_check(d, N, L, pos, sigma, alpha);
  if (st) return st;
  if (nc < 0 || (nc && (!cj || !ca || !out))) return OR_EINVAL;
  for (long long c = 0; c < nc; ++c) {
    const long long j = cj[c];
    const int a = ca[c];
    if (j < 0 || j >= N || a < 0 || a >= d) return OR_EINVAL;
    double rp[3], rm[3];
    for (int b = 0; b < d; ++b) rp[b] = rm[b] = pos[j * d + b];
    rp[a] += h;
    rm[a] -= h;
    double du = 0.0;
#pragma omp parallel for schedule(static) reduction(+ : du)
    for (long long i = 0; i < N; ++i) {
      if (i == j) continue;
      double up, um, g[3];
      pair_term(d, L, rp, pos + i * d, sigma, eps, alpha, &up, g);
      pair_term(d, L, rm, pos + i * d, sigma, eps, alpha, &um, g);
      du += up - um;
    }
    out[c] = du / (2.0 * h);
  }
  return OR_OK;
}

static int cmp_ll(const void* a, const void* b) {
  long long x = *(const long long*)a, y = *(const long long*)b;
  return (x > y) - (x < y);
}

int oracle_pair_cells(int d, long long N, const double* L, const double* pos, double sigma,
                      double eps, double alpha, double* energy, double* grad) {
  int st = pair_check(d, N, L, pos, sigma, alpha);
  if (st) return st;
  long long nc[3] = {1, 1, 1}, ncell = 1;
  for (int a = 0; a < d; ++a) {
    nc[a] = (long long)floor(L[a] / sigma);
    if (nc[a] < 1) nc[a] = 1;
    ncell *= nc[a];
  }
  long long* cell = (long long*)malloc(sizeof(long long) * (N ? N : 1));
  long long* head = (long long*)calloc((size_t)ncell + 1, sizeof(long long));
  long long* list = (long long*)malloc(sizeof(long long) * (N ? N : 1));
  if (!cell || !head || !list) { free(cell); free(head); free(list); return OR_ENOMEM; }
  for (long long i = 0; i < N; ++i) {
    long long c = 0;
    for (int a = d - 1; a >= 0; --a) {
      double u = pos[i * d + a] - L[a] * floor(pos[i * d + a] / L[a]);
      long long k = (long long)floor(u / L[a] * (double)nc[a]);
      if (k < 0) k = 0;
      if (k >= nc[a]) k = nc[a] - 1;
      c = c * nc[a] + k;
    }
    cell[i] = c;
    head[c + 1]++;
  }
  for (long long c = 0; c < ncell; ++c) head[c + 1] += head[c];
  {
    long long* fill = (long long*)malloc(sizeof(long long) * (size_t)ncell);
    if (!fill) { free(cell); free(head); free(list); return OR_ENOMEM; }
    memcpy(fill, head, sizeof(long long) * (size_t)ncell);
    for (long long i = 0; i < N; ++i) list[fill[cell[i]]++] = i;  /* increasing i per cell */
    free(fill);
  }
  double e = 0.0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : e)
  for (long long i = 0; i < N; ++i) {
    long long ci[3] = {0, 0, 0}, c = cell[i];
    for (int a = 0; a < d; ++a) { ci[a] = c % nc[a]; c /= nc[a]; }
    /* distinct neighbour cells (fewer than 3 per axis when the box is narrow) */
    long long nbr[27];
    int nn = 0;
    int lo[3], hi[3];
    for (int a = 0; a < 3; ++a) {
      lo[a] = (a < d) ? -1 : 0;
      hi[a] = (a < d) ? 1 : 0;
      if (a < d && nc[a] == 1) lo[a] = hi[a] = 0;
      if (a < d && nc[a] == 2) { lo[a] = 0; hi[a] = 1; }
    }
    for (int oz = lo[2]; oz <= hi[2]; ++oz)
      for (int oy = lo[1]; oy <= hi[1]; ++oy)
        for (int ox = lo[0]; ox <= hi[0]; ++ox) {
          int o[3] = {ox, oy, oz};
          long long q = 0;
          for (int a = d - 1; a >= 0; --a) q = q * nc[a] + (ci[a] + o[a] + nc[a]) % nc[a];
          nbr[nn++] = q;
        }
    /* partners in increasing index order, as the brute force visits them */
    long long cand_n = 0;
    for (int t = 0; t < nn; ++t) cand_n += head[nbr[t] + 1] - head[nbr[t]];
    long long* cand = (long long*)malloc(sizeof(long long) * (cand_n ? cand_n : 1));
    long long m = 0;
    for (int t = 0; t < nn; ++t)
      for (long long s = head[nbr[t]]; s < head[nbr[t] + 1]; ++s) cand[m++] = list[s];
    qsort(cand, (size_t)m, sizeof(long long), cmp_ll);
    double acc[3] = {0.0, 0.0, 0.0}, ei = 0.0;
    for (long long s = 0; s < m; ++s) {
      long long j = cand[s];
      if (j == i) continue;
      double u, g[3];
      pair_term(d, L, pos + i * d, pos + j * d, sigma, eps, alpha, &u, g);
      ei += u;
      for (int a = 0; a < d; ++a) acc[a] += g[a];
    }
    free(cand);
    e += 0.5 * ei;
    if (grad)
      for (int a = 0; a < d; ++a) grad[i * d + a] = acc[a];
  }
  free(cell);
  free(head);
  free(list);
  if (energy) *energy = e;
  return OR_OK;
}

/*
 * rho(k) = sum_j exp(+i k.r_j) for a few listed modes over very many points, by
 * direct evaluation of cos and sin of k.r_j (no per-point tables, whose cost
 * grows with the largest |n|).  Points are taken in fixed blocks of 65536; each
 * block's partial sums are formed in point order and the blocks are added in
 * order, so the result does not depend on the thread count.
 */
#define DBLOCK 65536
int oracle_rho_direct(int d, long long N, const double* L, const double* pos, long long K,
                      const int* modes, double* rho) {
  if (d < 1 || d > 3 || N < 0 || K < 0 || !L || (N && !pos) || (K && (!modes || !rho)))
    return OR_EINVAL;
  long long nblk = (N + DBLOCK - 1) / DBLOCK;
  double* part = (double*)malloc(sizeof(double) * 2 * (K ? K : 1) * (nblk ? nblk : 1));
  if (!part) return OR_ENOMEM;
#pragma omp parallel for schedule(dynamic, 4)
  for (long long b = 0; b < nblk; ++b) {
    double* pb = part + 2 * K * b;
    for (long long q = 0; q < 2 * K; ++q) pb[q] = 0.0;
    long long j1 = (b + 1) * DBLOCK < N ? (b + 1) * DBLOCK : N;
    for (long long j = b * DBLOCK; j < j1; ++j)
      for (long long q = 0; q < K; ++q) {
        double ph = 0.0;
        for (int a = 0; a < d; ++a) ph += TWO_PI * (double)modes[q * d + a] * pos[j * d + a] / L[a];
        pb[2 * q] += cos(ph);
        pb[2 * q + 1] += sin(ph);
      }
  }
  for (long long q = 0; q < 2 * K; ++q) rho[q] = 0.0;
  for (long long b = 0; b < nblk; ++b)
    for (long long q = 0; q < 2 * K; ++q) rho[q] += part[2 * K * b + q];
  free(part);
  return OR_OK;
}

/*
 * Loss and gradient from a given rho(k) over the listed modes (for problems too
 * large for oracle_rho; rho from oracle_rho_direct).  N is the number of points
 * rho was summed over; the gradient is evaluated for the G points `gpos` [G][d]:
 *   S = |rho|^2 / N, loss = sum W (S - S0)^2,
 *   grad_a = Re sum_k C_a(k) exp(-i k.r),  C_a = -4 i k_a W (S - S0) rho / N.
 * exp(-i k.r) by direct cos/sin (no tables).
 */
int oracle_loss_grad_rho(int d, long long N, const double* L, long long K, const int* modes,
                         const double* W, const double* S0, const double* rho, double* S_out,
                         double* loss_out, long long G, const double* gpos, double* grad_out) {
  if (d < 1 || d > 3 || N <= 0 || K < 0 || !L || (K && (!modes || !W || !S0 || !rho)))
    return OR_EINVAL;
  if (G < 0 || (G && (!gpos || !grad_out))) return OR_EINVAL;
  double* C = (double*)malloc(sizeof(double) * 2 * d * (K ? K : 1));
  if (!C) return OR_ENOMEM;
  double loss = 0.0;
  for (long long q = 0; q < K; ++q) {
    double S = (rho[2 * q] * rho[2 * q] + rho[2 * q + 1] * rho[2 * q + 1]) / (double)N;
    double res = S - S0[q];
    loss += W[q] * res * res;
    if (S_out) S_out[q] = S;
    for (int a = 0; a < d; ++a) {
      double ka = TWO_PI * (double)modes[q * d + a] / L[a];
      double f = 4.0 * ka * W[q] * res / (double)N;
      C[2 * (q * d + a)] = f * rho[2 * q + 1];
      C[2 * (q * d + a) + 1] = -f * rho[2 * q];
    }
  }
  if (loss_out) *loss_out = loss;
#pragma omp parallel for schedule(static)
  for (long long g = 0; g < G; ++g) {
    double acc[3] = {0.0, 0.0, 0.0};
    for (long long q = 0; q < K; ++q) {
      double ph = 0.0;
      for (int a = 0; a < d; ++a) ph += TWO_PI * (double)modes[q * d + a] * gpos[g * d + a] / L[a];
      double er = cos(ph), ei = sin(ph);
      for (int a = 0; a < d; ++a) {
        const double* c = C + 2 * (q * d + a);
        acc[a] += c[0] * er + c[1] * ei;
      }
    }
    for (int a = 0; a < d; ++a) grad_out[g * d + a] = acc[a];
  }
  free(C);
  return OR_OK;
}
