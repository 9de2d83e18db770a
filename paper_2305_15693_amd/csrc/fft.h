// Parameter blocks of the FFT passes (see fft.hip).
#pragma once

#include "common.h"

namespace fresco {

// Device twiddles and stage plan of one transform length.
template <class R>
struct AxisFft {
  FftFactors F;         // stages of the complex FFT of length F.n
  int rmin;             // smallest radix used
  cpx<R>* tw = nullptr;   // exp(+2 pi i q / F.n), q in [0, F.n)
  cpx<R>* twN = nullptr;  // rows only: exp(+2 pi i q / (2 F.n)), q in [0, F.n)
};

// Forward rows read straight from the padded spreading tiles (the fold fused
// into the row pass): cover lists as in FoldTables, at most two entries per
// grid coordinate on every axis; the first axis's lists are staged in LDS.
template <class R>
struct RowFold {
  const R* tiles;        // null: rows read rin
  const int* off[3];
  const int2* ent[3];
  int nent0;             // entries of the first-axis lists
  int d, nf0, nf1;
  int E0, E1, nt0, nt1;
  long long ncell;       // cells of one padded tile
};

template <class R>
struct RowParams {
  long long nrows;
  bool tw_lds;           // twiddles staged in LDS (false for lines too long for it)
  int lines_per_block;
  int threads;
  int M0;
  const R* rin;          // forward input rows (real, length 2H)
  cpx<R>* cout;          // forward output rows (M0+1 complex)
  // half-spectrum layout: mode k of row r at r * rstride + k * kstride
  // (row-major: M0 + 1, 1; column-major: 1, nrows)
  long long rstride, kstride;
  // one row per workgroup, each group of 16 consecutive rows on one XCD
  // (workgroups go to the 8 XCDs round-robin), so that a column-major
  // half spectrum's lines fill in one L2
  int xcd16;
  const cpx<R>* cin[3];  // inverse inputs per component
  R* rout[3];            // inverse outputs per component
  RowFold<R> fold;       // forward only
};

template <class R>
struct ColParams {
  long long ncols;
  int bc;        // columns per block (power of two)
  bool tw_lds;   // twiddles staged in LDS (false for lines too long for it)
  int threads;   // block size
  int M;         // mode half-width along this axis
  FastDiv cdiv;  // columns per outer group
  long long in_outer, in_line, out_outer, out_line;  // strides in complex elements
  const cpx<R>* in[3];
  cpx<R>* out[3];
  // mode stage (last forward axis)
  int d;
  int M0, M1, M2;
  int P1, P2;        // 2 M_1 + 1, 2 M_2 + 1 (cube indexing)
  FastDiv h0div;     // M0 + 1
  const R* dec[3];   // spreading kernel: h_a / psihat_a(|n_a|), n_a in [0, M_a]
  const R* deci[3];  // interpolation kernel: h_a / psihat_i,a(|n_a|)
  R invN;
  R g_scale;         // GFIELD / GBACK: 1 / N, the factor of the pair correlation function
  bool mcol;         // mode-stage arrays below column-major [c][m] (else [m][c])
  const R* Wp;       // half spectrum: W(n), S0(n), W(-n), S0(-n)
  const R* S0p;
  const R* Wm;
  const R* S0m;
  double* loss_part; // one partial per block (FUSED)
  double* fsum_part; // optional (FUSED): one partial of sum_K W S (S - S0) per block
  R* S_cube;         // optional full-cube S
  cpx<R>* rho_save;  // optional half-spectrum rho (written by FUSED / SF, read by BWD)
  const R* g_cube;   // BWD: dL/dS on the full cube
};

template <class R>
size_t rows_lds_bytes(const RowParams<R>& p, const AxisFft<R>& ax);
template <class R>
size_t cols_lds_bytes(int mode, const ColParams<R>& p, const AxisFft<R>& ax);
// one-time kernel attributes for the launch shapes in p
template <class R>
hipError_t prepare_rows(const RowParams<R>& p, const AxisFft<R>& ax);
template <class R>
hipError_t prepare_cols(int mode, const ColParams<R>& p, const AxisFft<R>& ax);
template <class R>
hipError_t launch_rows(bool inverse, const RowParams<R>& p, const AxisFft<R>& ax, int ncomp,
                       hipStream_t st);
template <class R>
hipError_t launch_cols(int mode, const ColParams<R>& p, const AxisFft<R>& ax, int ncomp,
                       hipStream_t st);
// 2D columns of length n = 2m too long for LDS: recombination of the two
// length-m sub-transforms Y (= [Y0][Y1], each [2M+1][M0+1]), the mode stage
// `mode` (COL_FUSED, COL_SF or COL_BWD) and the two pre-twiddled coefficient
// sets Q (same layout) for the inverse sub-transforms; twn = exp(+2 pi i q / n).
// FUSED writes one loss partial per block (`blocks` of 256 threads).
template <class R>
hipError_t launch_long_modes(int mode, const ColParams<R>& p, const cpx<R>* Y, cpx<R>* Q,
                             const cpx<R>* twn, int n, int blocks, hipStream_t st);

}  // namespace fresco
