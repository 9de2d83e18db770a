// Structure factor at arbitrary wave vectors (free boundary conditions): the
// NUwNU variant of the Methods (constraints at any continuous q, e.g. Bragg
// peaks with rotational symmetries no lattice has) and the Ewald construction
// of the main text (S on circles or spheres of scattered directions).
//
//   rho(q_k) = sum_j c_j exp(+i q_k . r_j)        positions as given, no wrapping
//   S_k      = |rho(q_k)|^2 / rho0,  rho0 = sum_j c_j^2 (N for unit strengths)
//
// Evaluated by direct sums, O(N K): the constraint sets of NUwNU are a few
// dozen peaks and the Ewald quadratures a few hundred to a few thousand
// directions per incidence, where a direct sum on the GPU is both exact and
// cheap; a rescaled type-3 nonuniform FFT pays off only for much larger K.
//
// rho_q_kernel: a block owns 64 wave vectors (one per lane) and a chunk of the
//   points, staged 256 at a time in LDS (every lane of a wavefront reads the
//   same point: a broadcast); four wavefronts split the chunk; the phase q.r is
//   formed and reduced to [-1/2, 1/2) revolutions in FP64, sin and cos of the
//   reduced angle taken in the working precision, products summed in FP64;
//   block partials per chunk, summed over the chunks in a fixed order.
// nuwnu_grad_kernel: one thread per point, the coefficients
//   A_k = 4 W_k (S_k - S0_k) conj(rho_k) / rho0 staged in LDS;
//   dL/dr_j = c_j sum_k q_k Re[i A_k exp(i q_k . r_j)].
// Ewald: the scattered directions of each incidence are built on the device,
//   S at q = k (e_s - e_inc) by the same kernels, and T = forward sum / total
//   sum per incidence in one block.
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "common.h"

struct fresco_q_ctx {
  int d = 0;
  int dtype = 0;
  long long n = 0;
  long long max_q = 0;
  hipStream_t st = nullptr;
  std::vector<void*> allocs;
  double* q = nullptr;     // [max_q][d]
  double* W = nullptr;     // [max_q]
  double* S0 = nullptr;    // [max_q]
  long long K = 0;         // wave vectors set by fresco_q_set
  double2* part = nullptr; // chunk partials
  long long part_cap = 0;
  double2* rho = nullptr;  // [max_q]
  double* S = nullptr;     // [max_q]
  double2* A = nullptr;    // [max_q] gradient coefficients
  double* red = nullptr;   // [kRed + 3] strength partials, rho0, loss, sum W S (S - S0)
  double* T = nullptr;     // [max incidences per batch]
  double* host = nullptr;  // pinned scratch
  long long host_cap = 0;
  int last_hip = 0;
};

namespace fresco {
namespace {

constexpr int kQTile = 64;       // wave vectors per block
constexpr int kQBlocks = 2048;   // blocks the point chunks aim at
constexpr int kRed = 256;        // blocks of the strength reduction

long long q_chunks(long long n, long long K) {
  const long long tq = (K + kQTile - 1) / kQTile;
  long long nc = (kQBlocks + tq - 1) / tq;
  const long long maxc = (n + 255) / 256;
  if (nc > maxc) nc = maxc;
  if (nc > 1024) nc = 1024;
  if (nc < 1) nc = 1;
  return nc;
}

template <class R>
__device__ __forceinline__ void sincos_rev(double ph, R* s, R* c) {
  // ph radians -> reduced revolutions in [-1/2, 1/2], then sin/cos of 2 pi x
  double rv = ph * 0.15915494309189533577;  // 1 / (2 pi)
  rv -= rint(rv);
  if constexpr (sizeof(R) == 4) {
    sincospif((float)(2.0 * rv), s, c);
  } else {
    sincospi(2.0 * rv, s, c);
  }
}

template <class R>
__global__ __launch_bounds__(256) void rho_q_kernel(int d, long long n, const R* __restrict__ pos,
                                                    const R* __restrict__ c,
                                                    const double* __restrict__ q, long long K,
                                                    long long chunk, double2* __restrict__ part) {
  __shared__ double sp[256 * 3];
  __shared__ double sc[256];
  __shared__ double2 red[256];
  const int lane = threadIdx.x & 63, sub = threadIdx.x >> 6;
  const long long k = (long long)blockIdx.y * kQTile + lane;
  const bool act = k < K;
  double q0 = 0.0, q1 = 0.0, q2 = 0.0;
  if (act) {
    q0 = q[k * d];
    q1 = d > 1 ? q[k * d + 1] : 0.0;
    q2 = d > 2 ? q[k * d + 2] : 0.0;
  }
  const long long p0 = (long long)blockIdx.x * chunk;
  const long long p1 = (p0 + chunk < n) ? p0 + chunk : n;
  double sr = 0.0, si = 0.0;
  for (long long base = p0; base < p1; base += 256) {
    __syncthreads();
    const long long j = base + threadIdx.x;
    if (j < p1) {
      for (int a = 0; a < 3; ++a) sp[threadIdx.x * 3 + a] = a < d ? (double)pos[j * d + a] : 0.0;
      sc[threadIdx.x] = c ? (double)c[j] : 1.0;
    }
    __syncthreads();
    const int cnt = (p1 - base < 256) ? (int)(p1 - base) : 256;
    for (int t = sub; t < cnt; t += 4) {
      const double ph = q0 * sp[t * 3] + q1 * sp[t * 3 + 1] + q2 * sp[t * 3 + 2];
      R s, co;
      sincos_rev<R>(ph, &s, &co);
      sr += sc[t] * (double)co;
      si += sc[t] * (double)s;
    }
  }
  red[threadIdx.x] = make_double2(sr, si);
  __syncthreads();
  if (sub == 0 && act) {
    double2 t = red[lane];
    for (int u = 1; u < 4; ++u) {
      t.x += red[lane + 64 * u].x;
      t.y += red[lane + 64 * u].y;
    }
    part[(long long)blockIdx.x * K + k] = t;
  }
}

// rho_k = sum over chunks (fixed order); S_k = |rho_k|^2 / rho0 (rho0 at red[kRed])
__global__ void rho_q_reduce_kernel(const double2* __restrict__ part, long long nchunk, long long K,
                                    const double* __restrict__ red, double2* __restrict__ rho,
                                    double* __restrict__ S) {
  const long long k = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= K) return;
  double2 t = make_double2(0.0, 0.0);
  for (long long c = 0; c < nchunk; ++c) {
    const double2 v = part[c * K + k];
    t.x += v.x;
    t.y += v.y;
  }
  rho[k] = t;
  S[k] = (t.x * t.x + t.y * t.y) / red[kRed];
}

// rho0 = sum c^2 (FP64, fixed order) into red[kRed]; unit strengths: N
template <class R>
__global__ void rho0_partials_kernel(const R* __restrict__ c, long long n, double* __restrict__ red) {
  __shared__ double sh[256];
  double a = 0.0;
  for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (long long)gridDim.x * blockDim.x) {
    const double v = (double)c[i];
    a += v * v;
  }
  sh[threadIdx.x] = a;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
    __syncthreads();
  }
  if (threadIdx.x == 0) red[blockIdx.x] = sh[0];
}
__global__ void rho0_final_kernel(double* red, int nb, double unit_n) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  if (nb == 0) {
    red[kRed] = unit_n;
    return;
  }
  double t = 0.0;
  for (int b = 0; b < nb; ++b) t += red[b];
  red[kRed] = t;
}

// loss = sum W (S - S0)^2 (fixed order) into red[kRed + 1]; A_k = 4 W (S - S0) conj(rho) / rho0
__global__ void nuwnu_coef_kernel(const double* __restrict__ S, const double2* __restrict__ rho,
                                  const double* __restrict__ W, const double* __restrict__ S0,
                                  long long K, double* __restrict__ red, double2* __restrict__ A) {
  __shared__ double sh[1024], sf[1024];
  const double r0 = red[kRed];
  double l = 0.0, fs = 0.0;
  for (long long k = threadIdx.x; k < K; k += blockDim.x) {
    const double res = S[k] - S0[k];
    l += W[k] * res * res;
    fs += W[k] * S[k] * res;
    const double f = 4.0 * W[k] * res / r0;
    A[k] = make_double2(f * rho[k].x, -f * rho[k].y);
  }
  sh[threadIdx.x] = l;
  sf[threadIdx.x] = fs;
  __syncthreads();
  for (int off = blockDim.x / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      sh[threadIdx.x] += sh[threadIdx.x + off];
      sf[threadIdx.x] += sf[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    red[kRed + 1] = sh[0];
    red[kRed + 2] = sf[0];  // sum W S (S - S0), for the strength gradient
  }
}

// dL/dc_j = Re sum_k conj(A_k) exp(-i q_k . r_j) - (4 c_j / rho0) sum_k W S (S - S0)
// (Eq. lossweightgradient at arbitrary q; conj(A_k) = 4 W (S - S0) rho_k / rho0)
template <class R>
__global__ __launch_bounds__(256) void q_grad_c_kernel(int d, long long n,
                                                       const R* __restrict__ pos,
                                                       const R* __restrict__ c,
                                                       const double* __restrict__ q,
                                                       const double2* __restrict__ A, long long K,
                                                       const double* __restrict__ red,
                                                       R* __restrict__ gc) {
  __shared__ double sq[256 * 3];
  __shared__ double2 sa[256];
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double r[3] = {0.0, 0.0, 0.0};
  if (j < n)
    for (int a = 0; a < d; ++a) r[a] = (double)pos[j * d + a];
  double acc = 0.0;
  for (long long base = 0; base < K; base += 256) {
    __syncthreads();
    const long long k = base + threadIdx.x;
    if (k < K) {
      for (int a = 0; a < 3; ++a) sq[threadIdx.x * 3 + a] = a < d ? q[k * d + a] : 0.0;
      sa[threadIdx.x] = A[k];
    }
    __syncthreads();
    const int cnt = (K - base < 256) ? (int)(K - base) : 256;
    for (int t = 0; t < cnt; ++t) {
      const double ph = sq[t * 3] * r[0] + sq[t * 3 + 1] * r[1] + sq[t * 3 + 2] * r[2];
      R s, co;
      sincos_rev<R>(ph, &s, &co);
      acc += sa[t].x * (double)co - sa[t].y * (double)s;
    }
  }
  if (j < n) gc[j] = (R)(acc - 4.0 * (double)c[j] / red[kRed] * red[kRed + 2]);
}

template <class R>
__global__ __launch_bounds__(256) void nuwnu_grad_kernel(int d, long long n,
                                                         const R* __restrict__ pos,
                                                         const R* __restrict__ c,
                                                         const double* __restrict__ q,
                                                         const double2* __restrict__ A, long long K,
                                                         R* __restrict__ grad) {
  __shared__ double sq[256 * 3];
  __shared__ double2 sa[256];
  const long long j = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  double r[3] = {0.0, 0.0, 0.0};
  if (j < n)
    for (int a = 0; a < d; ++a) r[a] = (double)pos[j * d + a];
  double acc[3] = {0.0, 0.0, 0.0};
  for (long long base = 0; base < K; base += 256) {
    __syncthreads();
    const long long k = base + threadIdx.x;
    if (k < K) {
      for (int a = 0; a < 3; ++a) sq[threadIdx.x * 3 + a] = a < d ? q[k * d + a] : 0.0;
      sa[threadIdx.x] = A[k];
    }
    __syncthreads();
    const int cnt = (K - base < 256) ? (int)(K - base) : 256;
    for (int t = 0; t < cnt; ++t) {
      const double ph = sq[t * 3] * r[0] + sq[t * 3 + 1] * r[1] + sq[t * 3 + 2] * r[2];
      R s, co;
      sincos_rev<R>(ph, &s, &co);
      // Re[i A e] = -(A_re sin + A_im cos)
      const double v = -(sa[t].x * (double)s + sa[t].y * (double)co);
      acc[0] += sq[t * 3] * v;
      acc[1] += sq[t * 3 + 1] * v;
      acc[2] += sq[t * 3 + 2] * v;
    }
  }
  if (j < n) {
    const double cj = c ? (double)c[j] : 1.0;
    for (int a = 0; a < d; ++a) grad[j * d + a] = (R)(cj * acc[a]);
  }
}

// scattered directions of incidence i = ik * ndir + id (see the Ewald
// construction in fresco.h): q = k (e_s - e_inc), nsp per incidence
__global__ void ewald_q_kernel(int d, const double* __restrict__ kv, const double* __restrict__ dirs,
                               int ndir, int ns, long long inc0, long long ninc,
                               double* __restrict__ q) {
  const int nsp = d == 2 ? ns - 1 : ns;
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= ninc * nsp) return;
  const long long i = inc0 + t / nsp;
  const int m = (int)(t % nsp);
  const double k = kv[i / ndir];
  const double* e = dirs + (i % ndir) * d;
  double* out = q + t * d;
  if (d == 2) {
    const double th = atan2(e[1], e[0]) + 2.0 * M_PI * (double)(m + 1) / (double)ns;
    out[0] = k * (cos(th) - e[0]);
    out[1] = k * (sin(th) - e[1]);
  } else {
    const double z = 1.0 - (2.0 * m + 1.0) / (double)ns;
    const double ph = (double)m * M_PI * (3.0 - sqrt(5.0));
    const double rr = sqrt(1.0 - z * z);
    const double ux = rr * cos(ph), uy = rr * sin(ph);
    double a[3] = {0.0, 0.0, 1.0};
    if (fabs(e[2]) > 0.9) {
      a[0] = 1.0;
      a[2] = 0.0;
    }
    double e1[3] = {a[1] * e[2] - a[2] * e[1], a[2] * e[0] - a[0] * e[2], a[0] * e[1] - a[1] * e[0]};
    const double nn = sqrt(e1[0] * e1[0] + e1[1] * e1[1] + e1[2] * e1[2]);
    for (int b = 0; b < 3; ++b) e1[b] /= nn;
    const double e2[3] = {e[1] * e1[2] - e[2] * e1[1], e[2] * e1[0] - e[0] * e1[2],
                          e[0] * e1[1] - e[1] * e1[0]};
    for (int b = 0; b < 3; ++b) out[b] = k * (ux * e1[b] + uy * e2[b] + z * e[b] - e[b]);
  }
}

// T of each incidence: forward sum over total sum of its S (fixed tree order)
__global__ void ewald_t_kernel(int d, int ns, const double* __restrict__ S, double* __restrict__ T) {
  __shared__ double sf[256], sa[256];
  const int nsp = d == 2 ? ns - 1 : ns;
  const double* s = S + (long long)blockIdx.x * nsp;
  double f = 0.0, a = 0.0;
  for (int m = threadIdx.x; m < nsp; m += blockDim.x) {
    // forward: strictly less than 90 degrees from the incident direction,
    // decided on integers (2D: 4 m' < ns or 4 m' > 3 ns with m' = m + 1; 3D: z > 0)
    bool fwd;
    if (d == 2) fwd = 4 * (m + 1) < ns || 4 * (m + 1) > 3 * ns;
    else fwd = 2 * m + 1 < ns;
    a += s[m];
    if (fwd) f += s[m];
  }
  sf[threadIdx.x] = f;
  sa[threadIdx.x] = a;
  __syncthreads();
  for (int off = 128; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off) {
      sf[threadIdx.x] += sf[threadIdx.x + off];
      sa[threadIdx.x] += sa[threadIdx.x + off];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) T[blockIdx.x] = sf[0] / sa[0];
}

template <class T>
int qalloc(fresco_q_ctx* c, T** p, size_t count) {
  void* v = nullptr;
  if (hipMalloc(&v, sizeof(T) * (count ? count : 1)) != hipSuccess) {
    (void)hipGetLastError();
    return FRESCO_ENOMEM;
  }
  c->allocs.push_back(v);
  *p = (T*)v;
  return FRESCO_OK;
}

#define QCHK(x)                  \
  do {                           \
    hipError_t e_ = (x);         \
    if (e_ != hipSuccess) {      \
      qc->last_hip = (int)e_;    \
      return FRESCO_EHIP;        \
    }                            \
  } while (0)

// rho0 of the strengths (or N) into red[kRed]
int enqueue_rho0(fresco_q_ctx* qc, const void* c) {
  if (c) {
    if (qc->dtype == FRESCO_F32)
      rho0_partials_kernel<float><<<kRed, 256, 0, qc->st>>>((const float*)c, qc->n, qc->red);
    else
      rho0_partials_kernel<double><<<kRed, 256, 0, qc->st>>>((const double*)c, qc->n, qc->red);
  }
  rho0_final_kernel<<<1, 64, 0, qc->st>>>(qc->red, c ? kRed : 0, (double)qc->n);
  QCHK(hipGetLastError());
  return FRESCO_OK;
}

// rho and S at the K wave vectors q (device, [K][d]) into rho, S
int enqueue_rho_q(fresco_q_ctx* qc, const void* pos, const void* c, const double* q, long long K,
                  double2* rho, double* S) {
  if (K == 0) return FRESCO_OK;
  const long long nchunk = q_chunks(qc->n, K);
  if (nchunk * K > qc->part_cap) return FRESCO_ENOTSUP;
  const long long chunk = (qc->n + nchunk - 1) / nchunk;
  dim3 grid((unsigned)nchunk, (unsigned)((K + kQTile - 1) / kQTile));
  if (qc->dtype == FRESCO_F32)
    rho_q_kernel<float><<<grid, 256, 0, qc->st>>>(qc->d, qc->n, (const float*)pos,
                                                  (const float*)c, q, K, chunk, qc->part);
  else
    rho_q_kernel<double><<<grid, 256, 0, qc->st>>>(qc->d, qc->n, (const double*)pos,
                                                   (const double*)c, q, K, chunk, qc->part);
  rho_q_reduce_kernel<<<(unsigned)((K + 255) / 256), 256, 0, qc->st>>>(qc->part, nchunk, K,
                                                                      qc->red, rho, S);
  QCHK(hipGetLastError());
  return FRESCO_OK;
}

int host_space(fresco_q_ctx* qc, long long doubles) {
  if (qc->host_cap >= doubles) return FRESCO_OK;
  if (qc->host) (void)hipHostFree(qc->host);
  qc->host = nullptr;
  qc->host_cap = 0;
  if (hipHostMalloc((void**)&qc->host, sizeof(double) * (size_t)doubles) != hipSuccess)
    return FRESCO_ENOMEM;
  qc->host_cap = doubles;
  return FRESCO_OK;
}

}  // namespace
}  // namespace fresco

using namespace fresco;

extern "C" {

int fresco_q_destroy(fresco_q_ctx* qc) {
  if (!qc) return FRESCO_OK;
  (void)hipStreamSynchronize(qc->st);
  for (void* p : qc->allocs) (void)hipFree(p);
  if (qc->host) (void)hipHostFree(qc->host);
  delete qc;
  return FRESCO_OK;
}

int fresco_q_create(fresco_q_ctx** out, int32_t dim, int32_t dtype, int64_t n, int64_t max_q,
                    void* stream) {
  if (!out) return FRESCO_EINVAL;
  *out = nullptr;
  if ((dim != 2 && dim != 3) || (dtype != FRESCO_F32 && dtype != FRESCO_F64) || n < 1 ||
      max_q < 1)
    return FRESCO_EINVAL;
  if (n > 2147483647LL || max_q > (1LL << 26)) return FRESCO_ENOTSUP;
  fresco_q_ctx* qc = new (std::nothrow) fresco_q_ctx();
  if (!qc) return FRESCO_ENOMEM;
  qc->d = dim;
  qc->dtype = dtype;
  qc->n = n;
  qc->max_q = max_q;
  qc->st = (hipStream_t)stream;
  // chunk partials: nchunk K <= kQBlocks kQTile + K + kQTile over every K
  qc->part_cap = (long long)kQBlocks * kQTile + max_q + kQTile;
  int st = FRESCO_OK;
  if (!st) st = qalloc(qc, &qc->q, (size_t)max_q * dim);
  if (!st) st = qalloc(qc, &qc->W, (size_t)max_q);
  if (!st) st = qalloc(qc, &qc->S0, (size_t)max_q);
  if (!st) st = qalloc(qc, &qc->part, (size_t)qc->part_cap);
  if (!st) st = qalloc(qc, &qc->rho, (size_t)max_q);
  if (!st) st = qalloc(qc, &qc->S, (size_t)max_q);
  if (!st) st = qalloc(qc, &qc->A, (size_t)max_q);
  if (!st) st = qalloc(qc, &qc->red, (size_t)kRed + 3);
  if (!st) st = qalloc(qc, &qc->T, (size_t)max_q);
  if (st) {
    fresco_q_destroy(qc);
    return st;
  }
  *out = qc;
  return FRESCO_OK;
}

int fresco_q_set(fresco_q_ctx* qc, int64_t K, const double* q, const double* W, const double* S0) {
  if (!qc || K < 0 || K > qc->max_q || (K > 0 && !q)) return FRESCO_EINVAL;
  std::vector<double> w((size_t)K), s((size_t)K);
  for (long long k = 0; k < K; ++k) {
    w[k] = W ? W[k] : 1.0;
    s[k] = S0 ? S0[k] : 0.0;
    if (!(w[k] >= 0.0) || !std::isfinite(w[k]) || !std::isfinite(s[k])) return FRESCO_EINVAL;
  }
  for (long long i = 0; i < K * qc->d; ++i)
    if (!std::isfinite(q[i])) return FRESCO_EINVAL;
  QCHK(hipStreamSynchronize(qc->st));
  if (K > 0) {
    QCHK(hipMemcpy(qc->q, q, sizeof(double) * K * qc->d, hipMemcpyHostToDevice));
    QCHK(hipMemcpy(qc->W, w.data(), sizeof(double) * K, hipMemcpyHostToDevice));
    QCHK(hipMemcpy(qc->S0, s.data(), sizeof(double) * K, hipMemcpyHostToDevice));
  }
  qc->K = K;
  return FRESCO_OK;
}

int fresco_q_structure_factor(fresco_q_ctx* qc, const void* pos, const void* c, double* S,
                              double* rho) {
  if (!qc || !pos || !S) return FRESCO_EINVAL;
  int st;
  if ((st = enqueue_rho0(qc, c))) return st;
  if ((st = enqueue_rho_q(qc, pos, c, qc->q, qc->K, rho ? (double2*)rho : qc->rho, S))) return st;
  return FRESCO_OK;
}

int fresco_q_loss_grad(fresco_q_ctx* qc, const void* pos, const void* c, double* loss,
                       void* grad) {
  if (!qc || !pos || !loss || !grad) return FRESCO_EINVAL;
  int st;
  if ((st = enqueue_rho0(qc, c))) return st;
  if ((st = enqueue_rho_q(qc, pos, c, qc->q, qc->K, qc->rho, qc->S))) return st;
  if ((st = host_space(qc, 1))) return st;
  nuwnu_coef_kernel<<<1, 1024, 0, qc->st>>>(qc->S, qc->rho, qc->W, qc->S0, qc->K, qc->red, qc->A);
  const unsigned nb = (unsigned)((qc->n + 255) / 256);
  if (qc->dtype == FRESCO_F32)
    nuwnu_grad_kernel<float><<<nb, 256, 0, qc->st>>>(qc->d, qc->n, (const float*)pos,
                                                    (const float*)c, qc->q, qc->A, qc->K,
                                                    (float*)grad);
  else
    nuwnu_grad_kernel<double><<<nb, 256, 0, qc->st>>>(qc->d, qc->n, (const double*)pos,
                                                     (const double*)c, qc->q, qc->A, qc->K,
                                                     (double*)grad);
  QCHK(hipGetLastError());
  QCHK(hipMemcpyAsync(qc->host, qc->red + kRed + 1, sizeof(double), hipMemcpyDeviceToHost, qc->st));
  QCHK(hipStreamSynchronize(qc->st));
  *loss = qc->host[0];
  return FRESCO_OK;
}

int fresco_q_loss_grad_strengths(fresco_q_ctx* qc, const void* pos, const void* c, double* loss,
                                 void* grad_c) {
  if (!qc || !pos || !c || !loss || !grad_c) return FRESCO_EINVAL;
  int st;
  if ((st = enqueue_rho0(qc, c))) return st;
  if ((st = enqueue_rho_q(qc, pos, c, qc->q, qc->K, qc->rho, qc->S))) return st;
  if ((st = host_space(qc, 1))) return st;
  nuwnu_coef_kernel<<<1, 1024, 0, qc->st>>>(qc->S, qc->rho, qc->W, qc->S0, qc->K, qc->red, qc->A);
  const unsigned nb = (unsigned)((qc->n + 255) / 256);
  if (qc->dtype == FRESCO_F32)
    q_grad_c_kernel<float><<<nb, 256, 0, qc->st>>>(qc->d, qc->n, (const float*)pos,
                                                  (const float*)c, qc->q, qc->A, qc->K, qc->red,
                                                  (float*)grad_c);
  else
    q_grad_c_kernel<double><<<nb, 256, 0, qc->st>>>(qc->d, qc->n, (const double*)pos,
                                                   (const double*)c, qc->q, qc->A, qc->K, qc->red,
                                                   (double*)grad_c);
  QCHK(hipGetLastError());
  QCHK(hipMemcpyAsync(qc->host, qc->red + kRed + 1, sizeof(double), hipMemcpyDeviceToHost, qc->st));
  QCHK(hipStreamSynchronize(qc->st));
  *loss = qc->host[0];
  return FRESCO_OK;
}

int fresco_ewald_transmission(fresco_q_ctx* qc, const void* pos, const void* c, int32_t n_k,
                              const double* k, int32_t n_dir, const double* dirs, int32_t ns,
                              double* T) {
  if (!qc || !pos || !k || !dirs || !T || n_k < 1 || n_dir < 1) return FRESCO_EINVAL;
  if (ns < (qc->d == 2 ? 4 : 2)) return FRESCO_EINVAL;
  const int d = qc->d;
  const int nsp = d == 2 ? ns - 1 : ns;
  if (nsp > qc->max_q) return FRESCO_ENOTSUP;
  for (int i = 0; i < n_k; ++i)
    if (!(k[i] > 0.0) || !std::isfinite(k[i])) return FRESCO_EINVAL;
  for (int i = 0; i < n_dir; ++i) {
    double nn = 0.0;
    for (int a = 0; a < d; ++a) nn += dirs[i * d + a] * dirs[i * d + a];
    if (!(std::fabs(nn - 1.0) < 1e-9)) return FRESCO_EINVAL;  // unit incident directions
  }
  const long long ninc = (long long)n_k * n_dir;
  int st;
  if ((st = host_space(qc, ninc))) return st;
  // the incidences' k values and directions, on the device for the q builder
  double* kv = nullptr;
  double* dv = nullptr;
  if (hipMalloc(&kv, sizeof(double) * n_k) != hipSuccess) return FRESCO_ENOMEM;
  if (hipMalloc(&dv, sizeof(double) * n_dir * d) != hipSuccess) {
    (void)hipFree(kv);
    return FRESCO_ENOMEM;
  }
  auto fail = [&](int code) {
    (void)hipStreamSynchronize(qc->st);
    (void)hipFree(kv);
    (void)hipFree(dv);
    return code;
  };
  if (hipMemcpy(kv, k, sizeof(double) * n_k, hipMemcpyHostToDevice) != hipSuccess ||
      hipMemcpy(dv, dirs, sizeof(double) * n_dir * d, hipMemcpyHostToDevice) != hipSuccess)
    return fail(FRESCO_EHIP);
  // the wave vectors of up to max_q / nsp incidences at a time go to the
  // context's q buffer (the constraint set of fresco_q_set is dropped)
  const long long per = qc->max_q / nsp;  // incidences per batch
  if ((st = enqueue_rho0(qc, c))) return fail(st);
  for (long long i0 = 0; i0 < ninc; i0 += per) {
    const long long nb = (ninc - i0 < per) ? ninc - i0 : per;
    const long long K = nb * nsp;
    ewald_q_kernel<<<(unsigned)((K + 255) / 256), 256, 0, qc->st>>>(d, kv, dv, n_dir, ns, i0, nb,
                                                                   qc->q);
    if ((st = enqueue_rho_q(qc, pos, c, qc->q, K, qc->rho, qc->S))) return fail(st);
    ewald_t_kernel<<<(unsigned)nb, 256, 0, qc->st>>>(d, ns, qc->S, qc->T);
    if (hipGetLastError() != hipSuccess) return fail(FRESCO_EHIP);
    if (hipMemcpyAsync(qc->host + i0, qc->T, sizeof(double) * nb, hipMemcpyDeviceToHost,
                       qc->st) != hipSuccess)
      return fail(FRESCO_EHIP);
  }
  if (hipStreamSynchronize(qc->st) != hipSuccess) return fail(FRESCO_EHIP);
  std::memcpy(T, qc->host, sizeof(double) * ninc);
  qc->K = 0;  // the wave vectors set by fresco_q_set were overwritten
  (void)hipFree(kv);
  (void)hipFree(dv);
  return FRESCO_OK;
}

int fresco_q_last_hip_error(const fresco_q_ctx* qc) { return qc ? qc->last_hip : 0; }

}  // extern "C"
