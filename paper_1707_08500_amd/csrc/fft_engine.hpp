// Mixed-radix FFT engine for padded-subdomain local FFTs (Sec. 3.2: each padded
// subdomain takes its own local 3D FFT).
//
// Radix codelets (2, 3, 4, 5, 6, 7, 8, 10, 11, 12, 16) run in registers; a
// length-N transform is one to four in-place stages over a work-group's LDS
// buffer, with a barrier between stages.  Two in-place orders are provided:
//   dif: natural-order input  -> output in "stage-digit" order
//   dit: stage-digit input    -> natural-order output
// For a plan N = r_0 r_1 ... r_{S-1}, frequency (or time) index
//   k = t_0 + r_0 t_1 + r_0 r_1 t_2 + ...     sits at position
//   pos(k) = t_0 N/r_0 + t_1 N/(r_0 r_1) + ...
// so a forward dif followed by a backward dit is N times the identity with no
// permutation pass.  DIR = -1 is exp(-i...) (forward), +1 backward; no scaling.
//
// Everything here is __host__ __device__: the barrier is a callable passed in
// by the kernel, and (tid, nthreads) distribute butterflies over the threads.
#pragma once
#include <stdint.h>

#include "dft_consts.h"

#define PSATD_HD __host__ __device__ __forceinline__

namespace psatd {

template <typename T>
struct alignas(2 * sizeof(T)) cx {
  T x, y;
};

template <typename T> PSATD_HD cx<T> operator+(cx<T> a, cx<T> b) { return {a.x + b.x, a.y + b.y}; }
template <typename T> PSATD_HD cx<T> operator-(cx<T> a, cx<T> b) { return {a.x - b.x, a.y - b.y}; }
template <typename T> PSATD_HD cx<T> cmul(cx<T> a, cx<T> b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
template <typename T> PSATD_HD cx<T> conj(cx<T> a) { return {a.x, -a.y}; }
template <typename T> PSATD_HD cx<T> scale(cx<T> a, T s) { return {a.x * s, a.y * s}; }
// i * a
template <typename T> PSATD_HD cx<T> mul_i(cx<T> a) { return {-a.y, a.x}; }

// a * exp(DIR * i * 2 pi e / R), e a compile-time constant after unrolling
template <int R, int DIR, typename T>
PSATD_HD cx<T> rot(cx<T> a, int e) {
  const T c = (T)DftConst<R>::c[e % R];
  const T s = (T)(DIR * DftConst<R>::s[e % R]);
  return {a.x * c - a.y * s, a.x * s + a.y * c};
}

// ----------------------------------------------------------------- codelets
template <int R, int DIR, typename T> struct Dft;

template <int DIR, typename T> struct Dft<2, DIR, T> {
  static PSATD_HD void run(cx<T>* a) {
    cx<T> t = a[0];
    a[0] = t + a[1];
    a[1] = t - a[1];
  }
};

template <int DIR, typename T> struct Dft<4, DIR, T> {
  static PSATD_HD void run(cx<T>* a) {
    cx<T> s02 = a[0] + a[2], d02 = a[0] - a[2];
    cx<T> s13 = a[1] + a[3], d13 = a[1] - a[3];
    // DIR * i * d13
    cx<T> r = (DIR < 0) ? cx<T>{d13.y, -d13.x} : cx<T>{-d13.y, d13.x};
    a[0] = s02 + s13;
    a[2] = s02 - s13;
    a[1] = d02 + r;
    a[3] = d02 - r;
  }
};

// odd prime R: pair q with R-q; X[t] = A_t + DIR i B_t, X[R-t] = A_t - DIR i B_t
template <int R, int DIR, typename T> struct DftOdd {
  static PSATD_HD void run(cx<T>* a) {
    constexpr int h = (R - 1) / 2;
    cx<T> sp[h], sm[h];
    cx<T> x0 = a[0];
    cx<T> X0 = x0;
#pragma unroll
    for (int q = 1; q <= h; ++q) {
      sp[q - 1] = a[q] + a[R - q];
      sm[q - 1] = a[q] - a[R - q];
      X0 = X0 + sp[q - 1];
    }
#pragma unroll
    for (int t = 1; t <= h; ++t) {
      cx<T> A = x0, B = {T(0), T(0)};
#pragma unroll
      for (int q = 1; q <= h; ++q) {
        const int e = (q * t) % R;
        const T cq = (T)DftConst<R>::c[e];
        const T sq = (T)DftConst<R>::s[e];
        A.x += sp[q - 1].x * cq;
        A.y += sp[q - 1].y * cq;
        B.x += sm[q - 1].x * sq;
        B.y += sm[q - 1].y * sq;
      }
      a[t] = cx<T>{A.x - DIR * B.y, A.y + DIR * B.x};
      a[R - t] = cx<T>{A.x + DIR * B.y, A.y - DIR * B.x};
    }
    a[0] = X0;
  }
};
template <int DIR, typename T> struct Dft<3, DIR, T> : DftOdd<3, DIR, T> {};
template <int DIR, typename T> struct Dft<5, DIR, T> : DftOdd<5, DIR, T> {};
template <int DIR, typename T> struct Dft<7, DIR, T> : DftOdd<7, DIR, T> {};
template <int DIR, typename T> struct Dft<11, DIR, T> : DftOdd<11, DIR, T> {};

// composite R = A B: n = j + q B, k = t0 + A t1
//   X[t0 + A t1] = sum_j W_B^{j t1} W_R^{j t0} sum_q x[j + q B] W_A^{q t0}
template <int A, int B, int DIR, typename T> struct DftSplit {
  static PSATD_HD void run(cx<T>* a) {
    constexpr int R = A * B;
    cx<T> v[R];
#pragma unroll
    for (int j = 0; j < B; ++j) {
      cx<T> u[A];
#pragma unroll
      for (int q = 0; q < A; ++q) u[q] = a[j + q * B];
      Dft<A, DIR, T>::run(u);
#pragma unroll
      for (int t0 = 0; t0 < A; ++t0) v[j * A + t0] = (j * t0) ? rot<R, DIR, T>(u[t0], j * t0) : u[t0];
    }
#pragma unroll
    for (int t0 = 0; t0 < A; ++t0) {
      cx<T> w[B];
#pragma unroll
      for (int j = 0; j < B; ++j) w[j] = v[j * A + t0];
      Dft<B, DIR, T>::run(w);
#pragma unroll
      for (int t1 = 0; t1 < B; ++t1) a[t0 + A * t1] = w[t1];
    }
  }
};
template <int DIR, typename T> struct Dft<6, DIR, T> : DftSplit<2, 3, DIR, T> {};
template <int DIR, typename T> struct Dft<8, DIR, T> : DftSplit<2, 4, DIR, T> {};
template <int DIR, typename T> struct Dft<10, DIR, T> : DftSplit<2, 5, DIR, T> {};
template <int DIR, typename T> struct Dft<12, DIR, T> : DftSplit<4, 3, DIR, T> {};
template <int DIR, typename T> struct Dft<16, DIR, T> : DftSplit<4, 4, DIR, T> {};

// ------------------------------------------------------------------ plans
constexpr int kMaxStages = 4;

// n / d by a multiply-high: m = ceil(2^32 / d) makes floor(n m / 2^32) equal
// to n/d or n/d + 1 for every 32-bit n, so one correction gives the exact
// quotient (valid while n + d < 2^32).  d == 1 is the identity.
struct FastDiv {
  uint32_t d, m;
};
PSATD_HD FastDiv make_fastdiv(uint32_t d) {
  FastDiv f;
  f.d = d;
  f.m = d > 1 ? 0xFFFFFFFFu / d + 1u : 0u;
  return f;
}
PSATD_HD uint32_t fdiv(uint32_t n, FastDiv f) {
  if (f.d == 1u) return n;
  const uint32_t q = (uint32_t)(((uint64_t)n * f.m) >> 32);
  return (q * f.d > n) ? q - 1u : q;
}

// One FFT length's schedule.  Stage s has radix r_s and stride
// ms_s = N / (r_0 ... r_s).  The plan's twiddle table (offset tw, N entries,
// forward sign) is laid out by stage and butterfly: stage s, butterfly offset
// j < ms_s, output t = 1..r_s-1 holds W_N^{j t r_0...r_{s-1}} at
//   twoff[s] + j (r_s - 1) + t - 1,
// so one butterfly reads r_s - 1 consecutive entries (one base address); the
// stages take sum_s ms_s (r_s - 1) = N - 1 entries, the last one is 1.
struct FftPlanD {
  int32_t N;
  int32_t nstages;
  int32_t radix[kMaxStages];
  int32_t stride[kMaxStages];   // ms_s
  int32_t prod[kMaxStages];     // r_0 ... r_{s-1}
  int32_t twoff[kMaxStages];    // start of stage s in the plan's twiddle table
  FastDiv rdiv[kMaxStages];     // division by r_s
  FastDiv sdiv[kMaxStages];     // division by ms_s
  int32_t tw;    // offset of the plan's twiddle table
  int32_t pad_;
};

// Position of index k in stage-digit order: k = t_0 + r_0 t_1 + ..., pos = sum t_s ms_s.
PSATD_HD int plan_pos(const FftPlanD* pl, int k) {
  int pos = 0;
  uint32_t rem = (uint32_t)k;
  for (int s = 0; s < pl->nstages; ++s) {
    const uint32_t q = fdiv(rem, pl->rdiv[s]);
    pos += (int)(rem - q * (uint32_t)pl->radix[s]) * pl->stride[s];
    rem = q;
  }
  return pos;
}

// Inverse of plan_pos: the index held at position p.
PSATD_HD int plan_index(const FftPlanD* pl, int p) {
  int k = 0;
  uint32_t rem = (uint32_t)p;
  for (int s = 0; s < pl->nstages; ++s) {
    const uint32_t t = fdiv(rem, pl->sdiv[s]);
    rem -= t * (uint32_t)pl->stride[s];
    k += (int)t * pl->prod[s];
  }
  return k;
}

// twiddle W_N^e for direction DIR from the forward table
template <int DIR, typename T>
PSATD_HD cx<T> twid(const cx<T>* tw, int e) {
  cx<T> w = tw[e];
  if (DIR > 0) w.y = -w.y;
  return w;
}

// One stage over M transforms; element e of transform m at buf[m*ms + e*es].
// Sub-transform length L, stride L/R.  Butterflies are distributed with the
// transform index fastest across threads.  tws: this stage's twiddles (R - 1
// per butterfly offset j, see FftPlanD).
template <int R, int DIR, bool DIF, typename T>
PSATD_HD void fft_stage(cx<T>* buf, int M, FastDiv dM, int ms, int es, int N, int L, FastDiv dS,
                        const cx<T>* tws, int tid, int nt) {
  const int mstride = L / R;
  const int nb = N / R;
  const int total = M * nb;
  if (tid >= total) return;
  // butterfly b = w M + m, advanced incrementally by nt per iteration
  int w = (int)fdiv((uint32_t)tid, dM);
  int m = tid - w * M;
  const int dw = (int)fdiv((uint32_t)nt, dM);
  const int dm = nt - dw * M;
  const int step = mstride * es;
  for (int b = tid; b < total; b += nt) {
    const int blk = (int)fdiv((uint32_t)w, dS);
    const int j = w - blk * mstride;
    cx<T>* p = buf + m * ms + (blk * L + j) * es;
    const cx<T>* tb = tws + j * (R - 1) - 1;  // tb[t] = W^{j t ...}, t = 1..R-1
    cx<T> a[R];
#pragma unroll
    for (int q = 0; q < R; ++q) a[q] = p[q * step];
    if (DIF) {
      Dft<R, DIR, T>::run(a);
      if (j) {
#pragma unroll
        for (int t = 1; t < R; ++t) a[t] = cmul(a[t], twid<DIR>(tb, t));
      }
    } else {
      if (j) {
#pragma unroll
        for (int t = 1; t < R; ++t) a[t] = cmul(a[t], twid<DIR>(tb, t));
      }
      Dft<R, DIR, T>::run(a);
    }
#pragma unroll
    for (int q = 0; q < R; ++q) p[q * step] = a[q];
    m += dm;
    w += dw;
    if (m >= M) {
      m -= M;
      ++w;
    }
  }
}

// MAXR bounds the codelets compiled into a kernel (registers scale with the
// largest one); radices 2..8 and 11 are always present.
template <int DIR, bool DIF, int MAXR, typename T>
PSATD_HD void fft_stage_dispatch(int R, cx<T>* buf, int M, FastDiv dM, int ms, int es, int N, int L,
                                 FastDiv dS, const cx<T>* tw, int tid, int nt) {
  switch (R) {
    case 2: fft_stage<2, DIR, DIF>(buf, M, dM, ms, es, N, L, dS, tw, tid, nt); break;
    case 3: fft_stage<3, DIR, DIF>(buf, M, dM, ms, es, N, L, dS, tw, tid, nt); break;
    case 4: fft_stage<4, DIR, DIF>(buf, M, dM, ms, es, N, L, dS, tw, tid, nt); break;
    case 5: fft_stage<5, DIR, DIF>(buf, M, dM, ms, es, N, L, dS, tw, tid, nt); break;
    case 6: fft_stage<6, DIR, DIF>(buf, M, dM, ms, es, N, L, dS, tw, tid, nt); break;
    case 7: fft_stage<7, DIR, DIF>(buf, M, dM, ms, es, N, L, dS, tw, tid, nt); break;
    case 8: fft_stage<8, DIR, DIF>(buf, M, dM, ms, es, N, L, dS, tw, tid, nt); break;
    case 10: if (MAXR >= 10) fft_stage<10, DIR, DIF>(buf, M, dM, ms, es, N, L, dS, tw, tid, nt); break;
    case 11: fft_stage<11, DIR, DIF>(buf, M, dM, ms, es, N, L, dS, tw, tid, nt); break;
    case 12: if (MAXR >= 12) fft_stage<12, DIR, DIF>(buf, M, dM, ms, es, N, L, dS, tw, tid, nt); break;
    case 16: if (MAXR >= 16) fft_stage<16, DIR, DIF>(buf, M, dM, ms, es, N, L, dS, tw, tid, nt); break;
    default: break;  // plans only hold the radices above (checked at plan time)
  }
}

// natural -> stage-digit order; ends with a barrier.  tw: this plan's twiddle
// table (global or LDS).  The plan is read from uniform memory.
template <int DIR, int MAXR, typename T, class Bar>
PSATD_HD void fft_dif(cx<T>* buf, int M, int ms, int es, const FftPlanD* pl, const cx<T>* tw,
                      int tid, int nt, Bar bar) {
  const int N = pl->N;
  const int ns = pl->nstages;
  const FastDiv dM = make_fastdiv((uint32_t)M);
  int L = N;
  for (int s = 0; s < ns; ++s) {
    const int R = pl->radix[s];
    fft_stage_dispatch<DIR, true, MAXR, T>(R, buf, M, dM, ms, es, N, L, pl->sdiv[s], tw + pl->twoff[s], tid,
                                           nt);
    bar();
    L /= R;
  }
}

// stage-digit -> natural order; ends with a barrier
template <int DIR, int MAXR, typename T, class Bar>
PSATD_HD void fft_dit(cx<T>* buf, int M, int ms, int es, const FftPlanD* pl, const cx<T>* tw,
                      int tid, int nt, Bar bar) {
  const int N = pl->N;
  const int ns = pl->nstages;
  const FastDiv dM = make_fastdiv((uint32_t)M);
  for (int s = ns - 1; s >= 0; --s) {
    const int L = pl->stride[s] * pl->radix[s];
    fft_stage_dispatch<DIR, false, MAXR, T>(pl->radix[s], buf, M, dM, ms, es, N, L, pl->sdiv[s],
                                            tw + pl->twoff[s], tid, nt);
    bar();
  }
}

// FFT engine of the kernel bodies: every stage as a VALU radix stage.
struct FftValu {
  template <int DIR, int MAXR, typename T, class Bar>
  PSATD_HD void dif(cx<T>* buf, int M, int ms, int es, const FftPlanD* pl, const cx<T>* tw, int tid,
                    int nt, Bar bar) const {
    fft_dif<DIR, MAXR>(buf, M, ms, es, pl, tw, tid, nt, bar);
  }
  template <int DIR, int MAXR, typename T, class Bar>
  PSATD_HD void dit(cx<T>* buf, int M, int ms, int es, const FftPlanD* pl, const cx<T>* tw, int tid,
                    int nt, Bar bar) const {
    fft_dit<DIR, MAXR>(buf, M, ms, es, pl, tw, tid, nt, bar);
  }
};

// ------------------------------------------- real <-> half-spectrum helpers
// A real row a[0..N) (N = 2 Nh) is packed as z[n] = a[2n] + i a[2n+1].  With
// Z = FFT_Nh(z) in natural order in row[0..Nh), r2c_post turns the pair
// (k, Nh-k) into the half spectrum A[k], A[Nh-k] of a (and A[Nh] from k = 0):
//   E = (Z[k] + conj Z[Nh-k]) / 2,  O = (Z[k] - conj Z[Nh-k]) / (2i),
//   A[k] = E + W_N^k O,  A[Nh-k] = conj(E) + W_N^{Nh-k} conj(O).
// twr: W_N^e table, N = 2 Nh.  k in [0, Nh/2].
template <typename T>
PSATD_HD void r2c_post_w(cx<T>* row, int k, int Nh, cx<T> wk, cx<T> wp) {  // wk = W_N^k, wp = W_N^{Nh-k}
  if (k == 0) {
    const cx<T> z = row[0];
    row[0] = cx<T>{z.x + z.y, T(0)};
    row[Nh] = cx<T>{z.x - z.y, T(0)};
    return;
  }
  const int kp = Nh - k;
  const cx<T> zk = row[k], zp = row[kp];
  const cx<T> cz = conj(zp);
  const cx<T> E = scale(zk + cz, T(0.5));
  const cx<T> D = zk - cz;
  const cx<T> O = cx<T>{T(0.5) * D.y, T(-0.5) * D.x};
  row[k] = E + cmul(wk, O);
  if (kp != k) row[kp] = conj(E) + cmul(wp, conj(O));
}
template <typename T>
PSATD_HD void r2c_post(cx<T>* row, int k, int Nh, const cx<T>* twr) {
  r2c_post_w(row, k, Nh, twr[k], twr[Nh - k]);
}

// Inverse of r2c_post up to a factor 2: from A[0..Nh] builds
//   Z[k] = (A[k] + conj A[Nh-k]) + i (A[k] - conj A[Nh-k]) W_N^{-k}
// so that the unnormalised backward FFT_Nh of Z gives N (a[2n] + i a[2n+1]).
template <typename T>
PSATD_HD cx<T> c2r_pair(cx<T> ak, cx<T> ap, cx<T> wk) {
  const cx<T> cap = conj(ap);
  return (ak + cap) + mul_i(cmul(ak - cap, conj(wk)));
}

template <typename T>
PSATD_HD void c2r_pre_w(cx<T>* row, int k, int Nh, cx<T> wk, cx<T> wp) {  // wk = W_N^k, wp = W_N^{Nh-k}
  const int kp = Nh - k;
  const cx<T> ak = row[k], ap = row[kp];
  const cx<T> zk = c2r_pair(ak, ap, wk);
  if (k != 0 && kp != k) row[kp] = c2r_pair(ap, ak, wp);
  row[k] = zk;
}
template <typename T>
PSATD_HD void c2r_pre(cx<T>* row, int k, int Nh, const cx<T>* twr) {
  c2r_pre_w(row, k, Nh, twr[k], twr[Nh - k]);
}

// The pair pass (r2c_post if FWD, else c2r_pre) over R rows (row r at
// rows + r ld) of a work-group's plane: each thread keeps one k of the Nh/2 + 1
// pairs with its two twiddles in registers and walks rows r0, r0 + per, ...
template <bool FWD, typename T>
PSATD_HD void pair_pass_rows(cx<T>* rows, int R, int ld, int Nh, const cx<T>* twr, int tid, int nt) {
  const int np = Nh / 2 + 1;
  if (np <= nt) {
    const int per = nt / np;
    const int r0 = tid / np;
    if (r0 >= per) return;
    const int k = tid - r0 * np;
    const cx<T> wk = twr[k], wp = twr[Nh - k];
    for (int r = r0; r < R; r += per) {
      if (FWD) r2c_post_w(rows + r * ld, k, Nh, wk, wp);
      else c2r_pre_w(rows + r * ld, k, Nh, wk, wp);
    }
    return;
  }
  const FastDiv dnp = make_fastdiv((uint32_t)np);
  for (int i = tid; i < R * np; i += nt) {
    const int r = (int)fdiv((uint32_t)i, dnp);
    if (FWD) r2c_post(rows + r * ld, i - r * np, Nh, twr);
    else c2r_pre(rows + r * ld, i - r * np, Nh, twr);
  }
}

}  // namespace psatd
