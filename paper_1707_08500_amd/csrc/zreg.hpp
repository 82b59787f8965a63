// Z pass of the FP32 forms with the z transforms held in registers: forward
// C2C along z of the 9 fields, the Eq. PSATD update at every k-point (Sec.
// 3.1, increments), inverse C2C along z of the 6 results (Sec. 3.2: each
// padded box's local 3D FFT), for boxes whose padded z length is the
// compile-time N.
//
// A work-group of NT = 64 W threads takes P consecutive (ky, kx) pencils of
// one box.  L neighbouring lanes share one (field, pencil) transform, lane l
// holding z = l + L e, e < E = N / L, in registers (reg_fft.hpp).  Forward:
// the length-E transform per lane, the twiddle W_N^{l k_e}, then the length-L
// DFT across the lanes (radix-2 steps, decimation in frequency), after which
// lane l holds frequency k_e + E brev(l) (brev: bit reversal over log2 L
// bits).  The
// update couples the 9 fields of one k-point, which sit in 9 lane groups: it
// runs over chunks of CH consecutive k_e through LDS laid out
// [k_e in chunk][lane l][field][pencil], with the FP32 coefficients of every
// chunk evaluated beforehand into a second LDS table.  The inverse mirrors the
// forward.
// Only the interior z-planes are stored (all the inverse x/y pass reads).
#pragma once

#include "psatd_device.hpp"
#include "reg_fft.hpp"

namespace psatd {

template <int N, int L, int W>
struct ZReg {
  static constexpr int NT = 64 * W;
  static constexpr int E = N / L;
  static constexpr int S = NT / L;   // transform slots
  static constexpr int P = S / 9;    // pencils per work-group
  static constexpr int CH = NT / (L * P) < E ? NT / (L * P) : E;  // k_e per update chunk
  static constexpr int NCH = (E + CH - 1) / CH;  // update chunks
  static constexpr int XCH_ELEMS = CH * L * 9 * P;  // exchange buffer (complex)
  static constexpr int COEF_FLOATS = 7 * NCH * NT;  // per-thread coefficient table
  static constexpr int LDS_BYTES = XCH_ELEMS * 8 + COEF_FLOATS * 4;
  static_assert(L == 1 || L == 2 || L == 4, "one, two or four lanes per transform");
  static_assert(N % L == 0 && P >= 1 && CH >= 1, "bad register z tile");
};

template <int N, int L, int W>
__device__ __forceinline__ void body_z_reg(const UpdArgs<float>& a, const int32_t* items, int item, int tid,
                                           cx<float>* lds) {
  using Z = ZReg<N, L, W>;
  constexpr int E = Z::E, P = Z::P, CH = Z::CH, NCH = Z::NCH, NT = Z::NT;
  float* const coef = reinterpret_cast<float*>(lds + Z::XCH_ELEMS);  // [chunk][7][thread]
  const int s = find_box(items, a.t.nsub, item);
  const BoxD& bx = a.t.box[s];
  const int blk = item - items[s];
  const int H = bx.H;
  const int nq = bx.P[1] * H;
  const int q0 = blk * P;
  const int np = (nq - q0) < P ? (nq - q0) : P;
  const int slot = tid / L, l = tid % L;
  const int f = slot / P, p = slot - (slot / P) * P;
  const bool inslot = slot < 9 * P;
  const bool live = inslot && p < np;
  // Buffer accesses over the tile's window of the box's 9 fields (less than
  // 2^31 bytes, checked at plan time): one 32-bit offset register per lane and
  // a wave-uniform offset per z element.  Offsets of idle lanes are clamped
  // into the tile (their data is never used).
  cx<float>* const wbase = spec_at(a.spec, bx, a.sbias, 0) + q0;
  const auto rs = buffer_rsrc(wbase, (uint32_t)((9 * bx.svol - q0) * sizeof(cx<float>)));
  const uint32_t lane_off =
      (uint32_t)(((live ? p : 0) + (inslot ? f : 0) * bx.svol + (int64_t)l * nq) * sizeof(cx<float>));
  const uint32_t zstep = (uint32_t)(L * nq * sizeof(cx<float>));  // bytes from e to e + 1

  // Thread tid updates the same (k_e offset j, lane ll, pencil pp) slot of
  // every chunk.  Its coefficients for every chunk are evaluated first, in
  // FP64, into its column of an LDS table (the barrier keeps the FP64
  // temporaries apart from the register-resident transforms).
  const int uj = tid / (L * P);
  const int ur = tid - uj * (L * P);
  const int ull = ur / P;
  const int upp = ur - ull * P;
  const bool upd = tid < CH * L * P && upp < np;
  const int ukl = L == 4 ? ((ull & 1) << 1) | (ull >> 1) : ull;  // frequency block of lane ull
  if (upd) {
    const double c = a.k.c, dt = a.k.dt, rc = 1.0 / c;
    const int q = q0 + upp;
    const int ky = q / H;
    const double kxv = a.t.kmod[bx.kx + q - ky * H], kyv = a.t.kmod[bx.ky + ky];
    // one chunk at a time: unrolled, the independent FP64 evaluations would be
    // interleaved and hold several chunks' temporaries at once
#pragma unroll 1
    for (int ch = 0; ch < NCH; ++ch) {
      const int ke = ch * CH + uj;
      if (ke >= E) break;
      const UpdCoef<float> u = update_coef<float, true>(kxv, kyv, a.t.kmod[bx.kz + ke + E * ukl], c, rc, dt);
      float* col = coef + ch * 7 * NT + tid;
      col[0 * NT] = u.C;
      col[1 * NT] = u.S;
      col[2 * NT] = u.X1;
      col[3 * NT] = u.X2;
      col[4 * NT] = u.a1;
      col[5 * NT] = u.x1c;
      col[6 * NT] = u.kz;
    }
  }
  __syncthreads();
  float ukx = 0.f, uky = 0.f;
  if (upd) {
    const int q = q0 + upp;
    const int ky = q / H;
    ukx = (float)a.t.kmod[bx.kx + q - ky * H];
    uky = (float)a.t.kmod[bx.ky + ky];
  }

  cx<float> v[E];
#pragma unroll
  for (int e = 0; e < E; ++e) v[e] = buf_load(rs, lane_off, e * zstep);

  // forward transform along z
  RegFft<E, -1, float>::run(v);
  const float sg1 = (l & 1) ? -1.f : 1.f, sg2 = (l & 2) ? -1.f : 1.f;
  if constexpr (L == 2) {
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const cx<float> w = rot_k<N, -1, float>(v[k], k);
      v[k] = xlane<1>(l ? w : v[k], sg1);
    }
  } else if constexpr (L == 4) {
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const cx<float> w1 = rot_k<N, -1, float>(v[k], k);
      const cx<float> w2 = rot_k<N, -1, float>(v[k], 2 * k);
      const cx<float> w3 = rot_k<N, -1, float>(v[k], 3 * k);
      const cx<float> u = l == 0 ? v[k] : (l == 1 ? w1 : (l == 2 ? w2 : w3));
      const cx<float> d = xlane<2>(u, sg2);
      v[k] = xlane<1>(l == 3 ? rot_k<4, -1, float>(d, 1) : d, sg1);
    }
  }

  // the update, chunk by chunk of k_e
#pragma unroll
  for (int ch = 0; ch < NCH; ++ch) {
    const int c0 = ch * CH;
    const int cn = (E - c0) < CH ? (E - c0) : CH;
    if (inslot) {
#pragma unroll
      for (int j = 0; j < cn; ++j) lds[((j * L + l) * 9 + f) * P + p] = v[c0 + j];
    }
    __syncthreads();
    if (upd && uj < cn) {
      cx<float>* row = lds + (uj * L + ull) * 9 * P + upp;
      float vr[9], vi[9];
#pragma unroll
      for (int g = 0; g < 9; ++g) {
        const cx<float> x = row[g * P];
        vr[g] = x.x;
        vi[g] = x.y;
      }
      const float* col = coef + ch * 7 * NT + tid;
      const UpdCoef<float> u{col[0 * NT], col[1 * NT], col[2 * NT], col[3 * NT], col[4 * NT], col[5 * NT],
                             ukx, uky, col[6 * NT]};
      update_apply<float>(vr, vi, u);
#pragma unroll
      for (int g = 0; g < 6; ++g) row[g * P] = cx<float>{vr[g], vi[g]};
    }
    __syncthreads();
    if (inslot && f < 6) {
#pragma unroll
      for (int j = 0; j < cn; ++j) v[c0 + j] = lds[((j * L + l) * 9 + f) * P + p];
    }
    __syncthreads();
  }

  // inverse transform along z (the 6 output fields; the J lanes idle along)
  if constexpr (L == 2) {
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const cx<float> x = xlane<1>(v[k], sg1);
      const cx<float> w = rot_k<N, +1, float>(x, k);
      v[k] = l ? w : x;
    }
  } else if constexpr (L == 4) {
#pragma unroll
    for (int k = 0; k < E; ++k) {
      const cx<float> d = xlane<1>(v[k], sg1);
      const cx<float> x = xlane<2>(l == 3 ? rot_k<4, +1, float>(d, 1) : d, sg2);
      const cx<float> w1 = rot_k<N, +1, float>(x, k);
      const cx<float> w2 = rot_k<N, +1, float>(x, 2 * k);
      const cx<float> w3 = rot_k<N, +1, float>(x, 3 * k);
      v[k] = l == 0 ? x : (l == 1 ? w1 : (l == 2 ? w2 : w3));
    }
  }
  RegFft<E, +1, float>::run(v);

  if (live && f < 6) {
    const int gz = bx.g[2], nz = bx.n[2];
#pragma unroll
    for (int e = 0; e < E; ++e) {
      const int z = l + L * e;
      if (z >= gz && z < gz + nz) buf_store(rs, lane_off, e * zstep, v[e]);
    }
  }
}

}  // namespace psatd
