// Register-resident FFTs of compile-time length (the z transforms of the
// local 3D FFT of Sec. 3.2, FP32 forms).
//
// RegFft<N, DIR, T>::run(a) transforms a[0..N) in place, natural order in
// and out, unnormalised, DIR = -1 forward (exp(-i...)), +1 backward.  Every
// index is a compile-time constant after unrolling, so the array lives in
// registers and the transform costs only its arithmetic: no address
// arithmetic, no LDS traffic and no barrier between stages.
//
// A length is either a codelet radix (fft_engine.hpp) or split N = A B with
// A the largest codelet radix that leaves a realisable cofactor:
//   n = b + B q (q < A, b < B),  k = t + A s (t < A, s < B),
//   X[t + A s] = sum_b W_B^{b s} W_N^{b t} sum_q x[b + B q] W_A^{q t}.
//
// xlane: the radix-2 steps of the length-L DFT (L = 2 or 4) across the L
// neighbouring lanes that share one length-N transform, through DPP lane
// moves (no LDS); buffer loads and stores address a tile with one 32-bit
// offset register and a wave-uniform offset per element.
#pragma once

#include "fft_engine.hpp"

namespace psatd {

constexpr bool is_codelet(int r) {
  return r == 2 || r == 3 || r == 4 || r == 5 || r == 6 || r == 7 || r == 8 || r == 10 || r == 11 || r == 12 ||
         r == 16;
}

constexpr bool realisable(int n);

// The first radix of a length-n split (0: n is 1 or not realisable).
constexpr int first_radix(int n) {
  constexpr int R[] = {16, 12, 11, 10, 8, 7, 6, 5, 4, 3, 2};
  for (int i = 0; i < 11; ++i)
    if (n % R[i] == 0 && n / R[i] > 1 && realisable(n / R[i])) return R[i];
  return 0;
}

constexpr bool realisable(int n) { return n == 1 || is_codelet(n) || first_radix(n) != 0; }

// a * W_R^e for DIR, with e a constant after unrolling: quarter turns are
// swaps and sign flips, eighth turns use one constant, the rest the table.
template <int R, int DIR, typename T>
PSATD_HD cx<T> rot_k(cx<T> a, int e) {
  e %= R;
  if (e == 0) return a;
  if (4 * e == R) return DIR < 0 ? cx<T>{a.y, -a.x} : cx<T>{-a.y, a.x};
  if (2 * e == R) return cx<T>{-a.x, -a.y};
  if (4 * e == 3 * R) return DIR < 0 ? cx<T>{-a.y, a.x} : cx<T>{a.y, -a.x};
  const T c = (T)DftConst<R>::c[e];
  const T s = (T)(DIR * DftConst<R>::s[e]);
  return {a.x * c - a.y * s, a.x * s + a.y * c};
}

template <int N, int DIR, typename T, bool CODELET = is_codelet(N)>
struct RegFft {
  static PSATD_HD void run(cx<T>* a) { Dft<N, DIR, T>::run(a); }
};

template <int DIR, typename T>
struct RegFft<1, DIR, T, false> {
  static PSATD_HD void run(cx<T>*) {}
};

template <int N, int DIR, typename T>
struct RegFft<N, DIR, T, false> {
  static constexpr int A = first_radix(N);
  static constexpr int B = N / A;
  static_assert(A > 0, "length without a register FFT schedule");
  static PSATD_HD void run(cx<T>* a) {
    cx<T> v[N];
#pragma unroll
    for (int b = 0; b < B; ++b) {
      cx<T> u[A];
#pragma unroll
      for (int q = 0; q < A; ++q) u[q] = a[b + B * q];
      Dft<A, DIR, T>::run(u);
#pragma unroll
      for (int t = 0; t < A; ++t) v[t * B + b] = rot_k<N, DIR, T>(u[t], b * t);
    }
#pragma unroll
    for (int t = 0; t < A; ++t) {
      RegFft<B, DIR, T>::run(v + t * B);
#pragma unroll
      for (int s = 0; s < B; ++s) a[t + A * s] = v[t * B + s];
    }
  }
};

// Value of the neighbouring lane l ^ 1 (DPP quad permutation 1, 0, 3, 2).
__device__ __forceinline__ float lane_xor1(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0xB1, 0xF, 0xF, true));
}

// Value of lane l ^ 2 (DPP quad permutation 2, 3, 0, 1).
__device__ __forceinline__ float lane_xor2(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), 0x4E, 0xF, 0xF, true));
}

// Radix-2 step across the lane pair (l, l ^ M), M = 1 or 2, one complex value
// per lane: the lower lane gets v_lo + v_hi, the upper v_lo - v_hi (the same
// for either direction).  sgn: +1 on the lower lane, -1 on the upper.
template <int M>
__device__ __forceinline__ cx<float> xlane(cx<float> v, float sgn) {
  const float wr = M == 1 ? lane_xor1(v.x) : lane_xor2(v.x);
  const float wi = M == 1 ? lane_xor1(v.y) : lane_xor2(v.y);
  return {fmaf(sgn, v.x, wr), fmaf(sgn, v.y, wi)};
}

// Buffer resource over `bytes` bytes at base (raw, untyped; the third word
// selects 32-bit elements on this GPU family).  Accesses at or beyond `bytes`
// read zeros and write nothing.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(void* base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(base, (short)0, (int)bytes, 0x00020000);
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

// One complex FP32 value at byte offset voff + soff (soff wave-uniform).
__device__ __forceinline__ cx<float> buf_load(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff) {
  const u32x2 w = __builtin_amdgcn_raw_buffer_load_b64(rs, (int)voff, (int)soff, 0);
  return {__uint_as_float(w.x), __uint_as_float(w.y)};
}
__device__ __forceinline__ void buf_store(__amdgpu_buffer_rsrc_t rs, uint32_t voff, uint32_t soff, cx<float> v) {
  const u32x2 w = {__float_as_uint(v.x), __float_as_uint(v.y)};
  __builtin_amdgcn_raw_buffer_store_b64(w, rs, (int)voff, (int)soff, 0);
}

}  // namespace psatd
