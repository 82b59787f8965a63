// Device data structures and kernel bodies of the local-FFT PSATD step.
//
// Bodies are __host__ __device__ templates taking (work item, thread id,
// thread count, LDS pointer, barrier) so that the same code runs in the
// __global__ wrappers of psatd_kernels.hip.
#pragma once
#include <math.h>
#include <stdint.h>

#include "fft_engine.hpp"

namespace psatd {

// Launch shapes (gfx950: 64-wide waves, 160 KiB LDS per compute unit).
constexpr int kThreadsXY = 256;   // x/y plane passes, exchange, scatter/gather
constexpr int kThreadsU32 = 512;  // z-update, FP32
constexpr int kThreadsU64 = 256;  // z-update, FP64
constexpr int kPB32 = 16;         // z-pencils per z-update work-group (128 B rows), FP32
constexpr int kPB64 = 8;          // same, FP64
constexpr int kMaxPPT = 6;        // k-points per thread held in registers by the z-update
constexpr int kMaxDynLds = 160 * 1024;

// One padded subdomain (Sec. 3.2, Fig. 2a).  Axes (x, y, z).
struct BoxD {
  int32_t lo[3];   // first owned global cell
  int32_t n[3];    // owned cells
  int32_t g[3];    // guard cells per side
  int32_t P[3];    // padded extents n + 2 g
  int32_t H;       // P[0]/2 + 1 (half-spectrum length along x)
  int32_t ld;      // LDS row stride (complex elements) of an (x, y) plane
  int32_t planx;   // FFT plan of length P[0]/2 (packed real rows)
  int32_t plany;   // FFT plan of length P[1]
  int32_t planz;   // FFT plan of length P[2]
  int32_t twr;     // offset of the W_{P[0]}^e table (real <-> half spectrum)
  int32_t kx, ky, kz;  // offsets of the FP64 modified-wavenumber tables
  int32_t pad_;
  int64_t foff;    // element offset of the box in a field buffer
  int64_t soff;    // complex-element offset of the box in one spectral field slab
};

// Work list: item -> box by binary search in a prefix array (size nsub + 1).
PSATD_HD int find_box(const int32_t* prefix, int nsub, int item) {
  int lo = 0, hi = nsub;  // prefix[lo] <= item < prefix[hi]
  while (hi - lo > 1) {
    const int mid = (lo + hi) >> 1;
    if (prefix[mid] <= item) lo = mid; else hi = mid;
  }
  return lo;
}

PSATD_HD int pmod(int v, int N) {
  int r = v % N;
  return r < 0 ? r + N : r;
}

// Tables shared by all passes.
template <typename T>
struct Tables {
  const BoxD* box;
  int32_t nsub;
  const FftPlanD* plans;
  const cx<T>* tw;        // twiddle tables (forward sign)
  const int32_t* idx;     // pos / ipos tables
  const double* kmod;     // modified wavenumbers (FP64)
};

// ------------------------------------------------------------------ pass F
// Forward R2C along x and C2C along y of one z-plane of one field of one box.
// Output: half spectrum plane [ky][kx] (kx = 0..H-1) in natural order.
template <typename T>
struct FwdArgs {
  Tables<T> t;
  const int32_t* items;    // prefix over boxes of P[2] * nfield
  int32_t nfield;
  const T* in[9];
  cx<T>* spec;             // spectral slabs, field f at spec + f * slab
  int64_t slab;
};

template <typename T, class Bar>
PSATD_HD void body_fwd_xy(const FwdArgs<T>& a, int item, int tid, int nt, cx<T>* lds, Bar bar) {
  const int s = find_box(a.items, a.t.nsub, item);
  const BoxD& bx = a.t.box[s];
  const int local = item - a.items[s];
  const int Px = bx.P[0], Py = bx.P[1], Pz = bx.P[2];
  const int f = local / Pz;
  const int z = local - f * Pz;
  const int Nh = Px >> 1, H = bx.H, ld = bx.ld;
  const FftPlanD* plx = a.t.plans + bx.planx;
  const FftPlanD* ply = a.t.plans + bx.plany;
  const int32_t* posx = a.t.idx + plx->pos;
  const int32_t* posy = a.t.idx + ply->pos;

  // packed real rows -> LDS rows in stage-digit order (for the dit transform)
  const cx<T>* src = reinterpret_cast<const cx<T>*>(a.in[f] + bx.foff + (int64_t)z * Py * Px);
  for (int i = tid; i < Py * Nh; i += nt) {
    const int y = i / Nh;
    const int nn = i - y * Nh;
    lds[y * ld + posx[nn]] = src[i];
  }
  bar();
  fft_dit<-1>(lds, Py, ld, 1, plx, a.t.tw, tid, nt, bar);
  const cx<T>* twr = a.t.tw + bx.twr;
  const int np = Nh / 2 + 1;
  for (int i = tid; i < Py * np; i += nt) {
    const int y = i / np;
    r2c_post(lds + y * ld, i - y * np, Nh, twr);
  }
  bar();
  fft_dif<-1>(lds, H, 1, ld, ply, a.t.tw, tid, nt, bar);
  cx<T>* dst = a.spec + f * a.slab + bx.soff + (int64_t)z * Py * H;
  for (int i = tid; i < Py * H; i += nt) {
    const int ky = i / H;
    const int kx = i - ky * H;
    dst[i] = lds[posy[ky] * ld + kx];
  }
}

// ------------------------------------------------------------------ pass U
// Along z: forward C2C of 9 fields for a block of PB consecutive (ky, kx)
// pencils, the Eq. PSATD update at every k, backward C2C of the 6 results.
struct UpdConst {
  double c, dt;
};

// Eqs. PSATD_1 / PSATD_2 (general c) at one k-point, FP64 arithmetic.
//   E' = C E + i c^2 (S/ck) [k]xB - (S/ck) J + X1 [k]([k].E) + X2 [k]([k].J)
//   B' = C B - i (S/ck) [k]xE + i (X1/c^2) [k]xJ
// C = cos th, S = sin th, th = c|[k]|dt, X1 = (1-C)/|[k]|^2 = 2 sin^2(th/2)/|[k]|^2,
// X2 = (S/ck - dt)/|[k]|^2 (series below th = 0.1); k -> 0 limits at |[k]| = 0.
template <typename T>
PSATD_HD void psatd_point(T* vr, T* vi /* E0 E1 E2 B0 B1 B2 J0 J1 J2 */, double kx, double ky,
                          double kz, double c, double dt) {
  const double k2 = kx * kx + ky * ky + kz * kz;
  double C, Sck, X1, X2;
  const double c2 = c * c;
  if (k2 == 0.0) {
    C = 1.0;
    Sck = dt;
    X1 = 0.5 * c2 * dt * dt;
    X2 = -c2 * dt * dt * dt / 6.0;
  } else {
    const double k = sqrt(k2);
    const double th = c * k * dt;
    const double sh = sin(0.5 * th), ch = cos(0.5 * th);
    C = 1.0 - 2.0 * sh * sh;
    Sck = (2.0 * sh * ch) / (c * k);
    X1 = 2.0 * sh * sh / k2;
    const double t2 = th * th;
    if (t2 < 1e-2) {
      X2 = -c2 * dt * dt * dt *
           (1.0 / 6.0 - t2 * (1.0 / 120.0 - t2 * (1.0 / 5040.0 - t2 * (1.0 / 362880.0 - t2 / 39916800.0))));
    } else {
      X2 = (Sck - dt) / k2;
    }
  }
  double er[3], ei[3], br[3], bi[3], jr[3], ji[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    er[a] = (double)vr[a]; ei[a] = (double)vi[a];
    br[a] = (double)vr[3 + a]; bi[a] = (double)vi[3 + a];
    jr[a] = (double)vr[6 + a]; ji[a] = (double)vi[6 + a];
  }
  const double K[3] = {kx, ky, kz};
  const double kEr = kx * er[0] + ky * er[1] + kz * er[2];
  const double kEi = kx * ei[0] + ky * ei[1] + kz * ei[2];
  const double kJr = kx * jr[0] + ky * jr[1] + kz * jr[2];
  const double kJi = kx * ji[0] + ky * ji[1] + kz * ji[2];
  // cross products [k] x F, real and imaginary parts
  const double kxBr[3] = {ky * br[2] - kz * br[1], kz * br[0] - kx * br[2], kx * br[1] - ky * br[0]};
  const double kxBi[3] = {ky * bi[2] - kz * bi[1], kz * bi[0] - kx * bi[2], kx * bi[1] - ky * bi[0]};
  const double kxEr[3] = {ky * er[2] - kz * er[1], kz * er[0] - kx * er[2], kx * er[1] - ky * er[0]};
  const double kxEi[3] = {ky * ei[2] - kz * ei[1], kz * ei[0] - kx * ei[2], kx * ei[1] - ky * ei[0]};
  const double kxJr[3] = {ky * jr[2] - kz * jr[1], kz * jr[0] - kx * jr[2], kx * jr[1] - ky * jr[0]};
  const double kxJi[3] = {ky * ji[2] - kz * ji[1], kz * ji[0] - kx * ji[2], kx * ji[1] - ky * ji[0]};
  const double a1 = c2 * Sck;
  const double x1c = X1 / c2;
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    // i * z = (-z.i, z.r)
    const double Er = C * er[a] - a1 * kxBi[a] - Sck * jr[a] + X1 * K[a] * kEr + X2 * K[a] * kJr;
    const double Ei = C * ei[a] + a1 * kxBr[a] - Sck * ji[a] + X1 * K[a] * kEi + X2 * K[a] * kJi;
    const double Br = C * br[a] + Sck * kxEi[a] - x1c * kxJi[a];
    const double Bi = C * bi[a] - Sck * kxEr[a] + x1c * kxJr[a];
    vr[a] = (T)Er; vi[a] = (T)Ei;
    vr[3 + a] = (T)Br; vi[3 + a] = (T)Bi;
  }
}

template <typename T>
struct UpdArgs {
  Tables<T> t;
  const int32_t* items;  // prefix over boxes of ceil(P[1] H / PB)
  cx<T>* spec;
  int64_t slab;
  UpdConst k;
};

template <typename T, int PB, int PPT, class Bar>
PSATD_HD void body_z_update(const UpdArgs<T>& a, int item, int tid, int nt, cx<T>* lds, Bar bar) {
  const int s = find_box(a.items, a.t.nsub, item);
  const BoxD& bx = a.t.box[s];
  const int blk = item - a.items[s];
  const int Py = bx.P[1], Pz = bx.P[2], H = bx.H;
  const int nq = Py * H;
  const int q0 = blk * PB;
  const int np = (nq - q0) < PB ? (nq - q0) : PB;
  const FftPlanD* plz = a.t.plans + bx.planz;
  const int32_t* iposz = a.t.idx + plz->ipos;
  const int tot = Pz * PB;

  // 9 field values of each owned k-point, split re/im so they stay in VGPRs
  T rr[PPT][9], ri[PPT][9];
  for (int f = 0; f < 9; ++f) {
    const cx<T>* src = a.spec + f * a.slab + bx.soff + q0;
    for (int i = tid; i < tot; i += nt) {
      const int z = i / PB;
      const int p = i - z * PB;
      if (p < np) lds[i] = src[(int64_t)z * nq + p];
    }
    bar();
    fft_dif<-1>(lds, np, 1, PB, plz, a.t.tw, tid, nt, bar);
#pragma unroll
    for (int r = 0; r < PPT; ++r) {
      const int i = tid + r * nt;
      if (i < tot) {
        const cx<T> v = lds[i];
        // f is uniform: a select chain keeps every register slot static
#pragma unroll
        for (int k = 0; k < 9; ++k) {
          rr[r][k] = (f == k) ? v.x : rr[r][k];
          ri[r][k] = (f == k) ? v.y : ri[r][k];
        }
      }
    }
    bar();
  }
  const double* kxt = a.t.kmod + bx.kx;
  const double* kyt = a.t.kmod + bx.ky;
  const double* kzt = a.t.kmod + bx.kz;
#pragma unroll
  for (int r = 0; r < PPT; ++r) {
    const int i = tid + r * nt;
    if (i < tot) {
      const int slot = i / PB;
      const int p = i - slot * PB;
      if (p < np) {
        const int q = q0 + p;
        const int ky = q / H;
        const int kx = q - ky * H;
        psatd_point(rr[r], ri[r], kxt[kx], kyt[ky], kzt[iposz[slot]], a.k.c, a.k.dt);
      }
    }
  }
  for (int f = 0; f < 6; ++f) {
#pragma unroll
    for (int r = 0; r < PPT; ++r) {
      const int i = tid + r * nt;
      if (i < tot) {
        cx<T> v = {rr[r][0], ri[r][0]};
#pragma unroll
        for (int k = 1; k < 6; ++k) {
          v.x = (f == k) ? rr[r][k] : v.x;
          v.y = (f == k) ? ri[r][k] : v.y;
        }
        lds[i] = v;
      }
    }
    bar();
    fft_dit<+1>(lds, np, 1, PB, plz, a.t.tw, tid, nt, bar);
    cx<T>* dst = a.spec + f * a.slab + bx.soff + q0;
    for (int i = tid; i < tot; i += nt) {
      const int z = i / PB;
      const int p = i - z * PB;
      if (p < np) dst[(int64_t)z * nq + p] = lds[i];
    }
    bar();
  }
}

// ------------------------------------------------------------------ pass I
// Backward C2C along y and C2R along x of one interior z-plane of one of the 6
// output fields; writes the interior cells of the plane, scaled by 1/V.
template <typename T>
struct InvArgs {
  Tables<T> t;
  const int32_t* items;  // prefix over boxes of n[2] * 6
  const cx<T>* spec;
  int64_t slab;
  T* out[6];
};

template <typename T, class Bar>
PSATD_HD void body_inv_xy(const InvArgs<T>& a, int item, int tid, int nt, cx<T>* lds, Bar bar) {
  const int s = find_box(a.items, a.t.nsub, item);
  const BoxD& bx = a.t.box[s];
  const int local = item - a.items[s];
  const int nz = bx.n[2];
  const int f = local / nz;
  const int z = bx.g[2] + (local - f * nz);
  const int Px = bx.P[0], Py = bx.P[1], Pz = bx.P[2];
  const int Nh = Px >> 1, H = bx.H, ld = bx.ld;
  const FftPlanD* plx = a.t.plans + bx.planx;
  const FftPlanD* ply = a.t.plans + bx.plany;
  const int32_t* posx = a.t.idx + plx->pos;
  const int32_t* posy = a.t.idx + ply->pos;

  const cx<T>* src = a.spec + f * a.slab + bx.soff + (int64_t)z * Py * H;
  for (int i = tid; i < Py * H; i += nt) {
    const int ky = i / H;
    const int kx = i - ky * H;
    lds[posy[ky] * ld + kx] = src[i];
  }
  bar();
  fft_dit<+1>(lds, H, 1, ld, ply, a.t.tw, tid, nt, bar);
  const int ny = bx.n[1], gy = bx.g[1];
  const cx<T>* twr = a.t.tw + bx.twr;
  const int np = Nh / 2 + 1;
  for (int i = tid; i < ny * np; i += nt) {
    const int y = i / np;
    c2r_pre(lds + (gy + y) * ld, i - y * np, Nh, twr);
  }
  bar();
  fft_dif<+1>(lds + gy * ld, ny, ld, 1, plx, a.t.tw, tid, nt, bar);
  const T sc = T(1.0 / ((double)Px * (double)Py * (double)Pz));
  const int nx = bx.n[0], gx = bx.g[0];
  T* dst = a.out[f] + bx.foff + (int64_t)z * Py * Px;
  for (int i = tid; i < ny * nx; i += nt) {
    const int yy = i / nx;
    const int x = gx + (i - yy * nx);
    const int y = gy + yy;
    const cx<T> v = lds[y * ld + posx[x >> 1]];
    dst[y * Px + x] = ((x & 1) ? v.y : v.x) * sc;
  }
}

// --------------------------------------------------------------- exchange
// Owner lookup for a global cell: per-axis cut index (tensor refinement of
// every box boundary), then a table over the refined cells.
struct OwnerD {
  const int32_t* cut[3];   // global index -> refined interval, per axis
  int32_t ncut[3];
  const int32_t* owner;    // [cz][cy][cx] -> box
  int32_t N[3];
};

PSATD_HD int owner_of(const OwnerD& o, int X, int Y, int Z) {
  return o.owner[(o.cut[2][Z] * o.ncut[1] + o.cut[1][Y]) * o.ncut[0] + o.cut[0][X]];
}

template <typename T>
struct FillArgs {
  const BoxD* box;
  int32_t nsub;
  const int32_t* items;  // prefix over boxes of P[2]
  OwnerD own;
  int32_t ncomp;
  T* comp[9];
};

// Fig. 3 step 3: every guard cell of box s takes the value of the owner of
// its global index (mod N).  One padded z-plane per item.
template <typename T>
PSATD_HD void body_fill(const FillArgs<T>& a, int item, int tid, int nt) {
  const int s = find_box(a.items, a.nsub, item);
  const BoxD& bx = a.box[s];
  const int z = item - a.items[s];
  const int Px = bx.P[0], Py = bx.P[1];
  const bool zg = z < bx.g[2] || z >= bx.g[2] + bx.n[2];
  const int Z = pmod(bx.lo[2] - bx.g[2] + z, a.own.N[2]);
  // interior rows only have guard cells at both x ends
  const int gx = bx.g[0], nx = bx.n[0];
  for (int i = tid; i < Py * Px; i += nt) {
    const int y = i / Px;
    const int x = i - y * Px;
    const bool yg = y < bx.g[1] || y >= bx.g[1] + bx.n[1];
    const bool xg = x < gx || x >= gx + nx;
    if (!(zg || yg || xg)) continue;
    const int Y = pmod(bx.lo[1] - bx.g[1] + y, a.own.N[1]);
    const int X = pmod(bx.lo[0] - gx + x, a.own.N[0]);
    const int o = owner_of(a.own, X, Y, Z);
    const BoxD& bo = a.box[o];
    const int64_t src = bo.foff + ((int64_t)(Z - bo.lo[2] + bo.g[2]) * bo.P[1] + (Y - bo.lo[1] + bo.g[1])) * bo.P[0] +
                        (X - bo.lo[0] + bo.g[0]);
    const int64_t dst = bx.foff + ((int64_t)z * Py + y) * Px + x;
    for (int c = 0; c < a.ncomp; ++c) a.comp[c][dst] = a.comp[c][src];
  }
}

template <typename T>
struct SumArgs {
  const BoxD* box;
  int32_t nsub;
  const int32_t* items;    // prefix over boxes of n[2]
  const int32_t* nbr_off;  // per box: boxes whose padded region meets its interior
  const int32_t* nbr;      // sorted ascending
  int32_t N[3];
  T* comp[3];
};

// Deposited currents: J_tot(X) = sum over every padded copy of X, in fixed
// order (neighbour boxes ascending, then z, y, x positions ascending), written
// to the owner's interior cell.  A fill pass then copies it to the guards.
template <typename T>
PSATD_HD void body_sum(const SumArgs<T>& a, int item, int tid, int nt) {
  const int s = find_box(a.items, a.nsub, item);
  const BoxD& bx = a.box[s];
  const int z = item - a.items[s];
  const int nx = bx.n[0], ny = bx.n[1];
  const int Z = bx.lo[2] + z;
  for (int i = tid; i < nx * ny; i += nt) {
    const int y = i / nx;
    const int x = i - y * nx;
    const int Y = bx.lo[1] + y, X = bx.lo[0] + x;
    T acc[3] = {T(0), T(0), T(0)};
    for (int e = a.nbr_off[s]; e < a.nbr_off[s + 1]; ++e) {
      const BoxD& b2 = a.box[a.nbr[e]];
      const int iz0 = pmod(Z - b2.lo[2] + b2.g[2], a.N[2]);
      const int iy0 = pmod(Y - b2.lo[1] + b2.g[1], a.N[1]);
      const int ix0 = pmod(X - b2.lo[0] + b2.g[0], a.N[0]);
      for (int iz = iz0; iz < b2.P[2]; iz += a.N[2])
        for (int iy = iy0; iy < b2.P[1]; iy += a.N[1])
          for (int ix = ix0; ix < b2.P[0]; ix += a.N[0]) {
            const int64_t idx = b2.foff + ((int64_t)iz * b2.P[1] + iy) * b2.P[0] + ix;
            acc[0] += a.comp[0][idx];
            acc[1] += a.comp[1][idx];
            acc[2] += a.comp[2][idx];
          }
    }
    const int64_t dst = bx.foff + ((int64_t)(z + bx.g[2]) * bx.P[1] + (y + bx.g[1])) * bx.P[0] + (x + bx.g[0]);
    a.comp[0][dst] = acc[0];
    a.comp[1][dst] = acc[1];
    a.comp[2][dst] = acc[2];
  }
}

// ------------------------------------------------------- scatter / gather
template <typename T>
struct ScatterArgs {
  const BoxD* box;
  int32_t nsub;
  const int32_t* items;  // scatter: prefix of P[2]; gather: prefix of n[2]
  int32_t N[3];
  const T* src[3];
  T* dst[3];
};

template <typename T>
PSATD_HD void body_scatter(const ScatterArgs<T>& a, int item, int tid, int nt) {
  const int s = find_box(a.items, a.nsub, item);
  const BoxD& bx = a.box[s];
  const int z = item - a.items[s];
  const int Px = bx.P[0], Py = bx.P[1];
  const int Z = pmod(bx.lo[2] - bx.g[2] + z, a.N[2]);
  for (int i = tid; i < Px * Py; i += nt) {
    const int y = i / Px;
    const int x = i - y * Px;
    const int Y = pmod(bx.lo[1] - bx.g[1] + y, a.N[1]);
    const int X = pmod(bx.lo[0] - bx.g[0] + x, a.N[0]);
    const int64_t gi = ((int64_t)Z * a.N[1] + Y) * a.N[0] + X;
    const int64_t pi = bx.foff + ((int64_t)z * Py + y) * Px + x;
    for (int c = 0; c < 3; ++c) a.dst[c][pi] = a.src[c][gi];
  }
}

template <typename T>
PSATD_HD void body_gather(const ScatterArgs<T>& a, int item, int tid, int nt) {
  const int s = find_box(a.items, a.nsub, item);
  const BoxD& bx = a.box[s];
  const int z = item - a.items[s];
  const int nx = bx.n[0], ny = bx.n[1];
  for (int i = tid; i < nx * ny; i += nt) {
    const int y = i / nx;
    const int x = i - y * nx;
    const int64_t gi = ((int64_t)(bx.lo[2] + z) * a.N[1] + (bx.lo[1] + y)) * a.N[0] + (bx.lo[0] + x);
    const int64_t pi = bx.foff + ((int64_t)(z + bx.g[2]) * bx.P[1] + (y + bx.g[1])) * bx.P[0] + (x + bx.g[0]);
    for (int c = 0; c < 3; ++c) a.dst[c][gi] = a.src[c][pi];
  }
}

// ------------------------------------------------ modified wavenumbers (a1)
// Sec. 3.1: [k](m) = sum_{j=1}^{p/2} w_j sin(j k_m du)/(du/2), k_m = 2 pi m~/(N du),
// w_1 = M/(M+1), w_{j+1} = -w_j j/(j+1) (M-j)/(M+j+1), M = p/2; p = 0: [k] = k_m.
// Even N: the Nyquist entry is exactly 0.
struct KEntry {
  int32_t N;
  int32_t off;
  double du;
};

PSATD_HD double modified_k_entry(int N, double du, int p, int m) {
  if ((N % 2 == 0) && 2 * m == N) return 0.0;
  const int mt = (m <= (N - 1) / 2) ? m : m - N;
  const double PI = 3.14159265358979323846;
  if (p == 0) return 2.0 * PI * (double)mt / ((double)N * du);
  const int M = p / 2;
  double w = (double)M / (double)(M + 1);
  double acc = 0.0;
  for (int j = 1; j <= M; ++j) {
    // sin(2 pi j m~ / N) with the integer argument reduced exactly
    const int64_t e = ((int64_t)j * mt) % N;
    acc += w * sin(2.0 * PI * (double)e / (double)N);
    w = -w * ((double)j / (double)(j + 1)) * ((double)(M - j) / (double)(M + j + 1));
  }
  return acc / (0.5 * du);
}

}  // namespace psatd
