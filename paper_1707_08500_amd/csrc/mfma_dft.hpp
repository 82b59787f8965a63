// Split-BF16 DFT-GEMM stage on the matrix cores (the precision forms
// F32_BF16X3 / F32_BF16X6 of the local FFTs, Sec. 3.2).
//
// The first stage of a length-N transform with radix 16 (stride S = N/16) is
// a complex 16x16 DFT applied to S*M columns: column (j, m) holds the inputs
// x_q = buf[m*ms + (j + q*S)*es], q = 0..15.  As a real product the 16x16
// complex matrix F becomes a 32-deep contraction: for output t
//   Re y_t = sum_q (Re F_tq Re x_q - Im F_tq Im x_q),
//   Im y_t = sum_q (Im F_tq Re x_q + Re F_tq Im x_q),
// i.e. two 16x32 by 32x16 products per 16 columns, one per output component,
// with the contraction index K = 2q + c (c = 0 real, 1 imaginary part).  Each
// product runs as one v_mfma_f32_16x16x32_bf16 (FP32 accumulation).
//
// FP32 operands are split into BF16 terms: v = v0 + v1 (+ v2), v0 = bf16(v),
// v1 = bf16(v - v0), v2 = bf16(v - v0 - v1).  SPL = 2 keeps the 3 products
// F0 x0 + F0 x1 + F1 x0; SPL = 3 keeps the 6 products with term indices
// summing to <= 2.  The constant F is split from its FP64 value.  The
// remaining stages of the transform run as VALU radix stages.
//
// Operand layout of the 16x16x32 BF16 instruction (64 lanes): lane l holds
// A[l % 16][8 (l / 16) + v] and B[8 (l / 16) + v][l % 16], v = 0..7, and
// receives C[4 (l / 16) + r][l % 16], r = 0..3.  So lane l serves column
// l % 16 of its 16-column chunk with inputs q = 4 (l / 16) .. +3 and outputs
// t = 4 (l / 16) .. +3.
#pragma once

#include "fft_engine.hpp"

namespace psatd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// BF16 terms of an FP32 value (each difference is exact in FP32).
template <int SPL>
PSATD_HD void split_bf16(float v, __bf16* out) {
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    const __bf16 h = (__bf16)v;
    out[s] = h;
    v -= (float)h;
  }
}

// BF16 terms of an FP64 constant.
template <int SPL>
PSATD_HD void split_bf16_f64(double v, __bf16* out) {
#pragma unroll
  for (int s = 0; s < SPL; ++s) {
    const __bf16 h = (__bf16)(float)v;
    out[s] = h;
    v -= (double)(float)h;
  }
}

// This lane's slice of the real 16x32 DFT operands (output real and
// imaginary rows), split into SPL BF16 terms.
template <int SPL>
struct Dft16Operand {
  bf16x8 re[SPL];
  bf16x8 im[SPL];
};

template <int DIR, int SPL>
PSATD_HD Dft16Operand<SPL> dft16_operand(int lane) {
  Dft16Operand<SPL> A;
  const int t = lane & 15, quad = lane >> 4;
#pragma unroll
  for (int v = 0; v < 8; ++v) {
    const int q = 4 * quad + (v >> 1);
    const int e = (q * t) & 15;
    // F_tq = exp(DIR 2 pi i q t / 16): real cos, imaginary DIR sin
    const double fr = DftConst<16>::c[e];
    const double fi = DIR < 0 ? -DftConst<16>::s[e] : DftConst<16>::s[e];
    __bf16 ar[SPL], ai[SPL];
    split_bf16_f64<SPL>((v & 1) ? -fi : fr, ar);
    split_bf16_f64<SPL>((v & 1) ? fr : fi, ai);
#pragma unroll
    for (int s = 0; s < SPL; ++s) {
      A.re[s][v] = ar[s];
      A.im[s][v] = ai[s];
    }
  }
  return A;
}

// One radix-16 stage (the first of the transform) on the matrix cores.
// DIF: DFT then twiddle W_N^{j t}; DIT: twiddle W_N^{j q} then DFT, with
// W_N^{j u} at tw[15 j + u - 1] (the first stage's part of the table).  In place;
// every wave takes whole 16-column chunks, all waves run the same number of
// chunk iterations (idle lanes load zeros and store nothing), so a model of
// the instruction that synchronises the work-group sees uniform calls.
template <int DIR, bool DIF, int SPL, class Mma>
PSATD_HD void dft16_mfma(cx<float>* buf, int M, FastDiv dM, int ms, int es, int N,
                         const cx<float>* tw, int tid, int nt, const Mma& mma) {
  const int lane = tid & 63, wave = tid >> 6, nwave = nt >> 6;
  const int S = N >> 4;
  const int ncol = S * M;
  const int nchunk = (ncol + 15) >> 4;
  const int niter = (nchunk + nwave - 1) / nwave;
  const int quad = lane >> 4;
  const int step = S * es;
  const Dft16Operand<SPL> A = dft16_operand<DIR, SPL>(lane);
  for (int it = 0; it < niter; ++it) {
    const int col = ((it * nwave + wave) << 4) + (lane & 15);
    const bool act = col < ncol;
    int j = 0, m = 0;
    if (act) {
      j = (int)fdiv((uint32_t)col, dM);
      m = col - j * M;
    }
    cx<float>* p = buf + m * ms + j * es;
    bf16x8 b[SPL];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int q = 4 * quad + r;
      cx<float> x = act ? p[q * step] : cx<float>{0.f, 0.f};
      if (!DIF && j && q) x = cmul(x, twid<DIR>(tw, 15 * j + q - 1));
      __bf16 hr[SPL], hi[SPL];
      split_bf16<SPL>(x.x, hr);
      split_bf16<SPL>(x.y, hi);
#pragma unroll
      for (int s = 0; s < SPL; ++s) {
        b[s][2 * r] = hr[s];
        b[s][2 * r + 1] = hi[s];
      }
    }
    f32x4 yr = {0.f, 0.f, 0.f, 0.f}, yi = {0.f, 0.f, 0.f, 0.f};
    // smallest products first
    if (SPL == 3) {
      yr = mma(A.re[SPL - 1], b[0], yr);
      yi = mma(A.im[SPL - 1], b[0], yi);
      yr = mma(A.re[1], b[1], yr);
      yi = mma(A.im[1], b[1], yi);
      yr = mma(A.re[0], b[SPL - 1], yr);
      yi = mma(A.im[0], b[SPL - 1], yi);
    }
    yr = mma(A.re[1], b[0], yr);
    yi = mma(A.im[1], b[0], yi);
    yr = mma(A.re[0], b[1], yr);
    yi = mma(A.im[0], b[1], yi);
    yr = mma(A.re[0], b[0], yr);
    yi = mma(A.im[0], b[0], yi);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int t = 4 * quad + r;
      cx<float> y{yr[r], yi[r]};
      if (DIF && j && t) y = cmul(y, twid<DIR>(tw, 15 * j + t - 1));
      if (act) p[t * step] = y;
    }
  }
}

// Transforms whose first stage has radix 16 run it on the matrix cores; the
// other stages (and plans without a radix-16 first stage) as VALU stages.
template <int DIR, int MAXR, int SPL, class Bar, class Mma>
PSATD_HD void fft_dif_mfma(cx<float>* buf, int M, int ms, int es, const FftPlanD* pl,
                           const cx<float>* tw, int tid, int nt, Bar bar, const Mma& mma) {
  const int N = pl->N;
  const int ns = pl->nstages;
  const FastDiv dM = make_fastdiv((uint32_t)M);
  int L = N;
  int s = 0;
  if (ns > 0 && pl->radix[0] == 16) {
    dft16_mfma<DIR, true, SPL>(buf, M, dM, ms, es, N, tw, tid, nt, mma);
    bar();
    L = N >> 4;
    s = 1;
  }
  for (; s < ns; ++s) {
    const int R = pl->radix[s];
    fft_stage_dispatch<DIR, true, MAXR, float>(R, buf, M, dM, ms, es, N, L, pl->sdiv[s], tw + pl->twoff[s],
                                               tid, nt);
    bar();
    L /= R;
  }
}

template <int DIR, int MAXR, int SPL, class Bar, class Mma>
PSATD_HD void fft_dit_mfma(cx<float>* buf, int M, int ms, int es, const FftPlanD* pl,
                           const cx<float>* tw, int tid, int nt, Bar bar, const Mma& mma) {
  const int N = pl->N;
  const int ns = pl->nstages;
  const FastDiv dM = make_fastdiv((uint32_t)M);
  const bool gemm = ns > 0 && pl->radix[0] == 16;
  for (int s = ns - 1; s >= (gemm ? 1 : 0); --s) {
    const int L = pl->stride[s] * pl->radix[s];
    fft_stage_dispatch<DIR, false, MAXR, float>(pl->radix[s], buf, M, dM, ms, es, N, L, pl->sdiv[s],
                                                tw + pl->twoff[s], tid, nt);
    bar();
  }
  if (gemm) {
    dft16_mfma<DIR, false, SPL>(buf, M, dM, ms, es, N, tw, tid, nt, mma);
    bar();
  }
}

// FFT engine of the bodies: split-BF16 matrix-core first stage (FP32 data).
template <int SPL, class Mma>
struct FftMfma {
  Mma mma;
  template <int DIR, int MAXR, typename T, class Bar>
  PSATD_HD void dif(cx<T>* buf, int M, int ms, int es, const FftPlanD* pl, const cx<T>* tw, int tid,
                    int nt, Bar bar) const {
    fft_dif_mfma<DIR, MAXR, SPL>(buf, M, ms, es, pl, tw, tid, nt, bar, mma);
  }
  template <int DIR, int MAXR, typename T, class Bar>
  PSATD_HD void dit(cx<T>* buf, int M, int ms, int es, const FftPlanD* pl, const cx<T>* tw, int tid,
                    int nt, Bar bar) const {
    fft_dit_mfma<DIR, MAXR, SPL>(buf, M, ms, es, pl, tw, tid, nt, bar, mma);
  }
};

}  // namespace psatd
