// Device data structures and kernel bodies of the local-FFT PSATD step.
//
// Bodies are __host__ __device__ templates taking (work item, thread id,
// thread count, LDS pointer, barrier) so that the same code runs in the
// __global__ wrappers of psatd_kernels.hip.
#pragma once
#include <math.h>
#include <stdint.h>

#include <type_traits>

#include "fft_engine.hpp"

namespace psatd {

// Launch shapes (gfx950: 64-wide waves, 160 KiB LDS per compute unit).
constexpr int kThreadsXY = 256;   // x/y plane passes, exchange, scatter/gather
constexpr int kMaxR = 16;         // largest radix codelet (radix 11 is always available)
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
  int64_t soff;    // sum of the half-spectrum sizes of the boxes before it
  int64_t svol;    // half-spectrum size of one field of the box, P[2] P[1] H (complex)
};

// The spectral workspace is box-major: box s holds the half spectra of its 9
// fields back to back, field f at 9 soff + f svol (complex elements, relative
// to the first box of the batch the workspace holds), [z][ky][kx] each.  So
// every field of a box lies within 9 svol elements of the box's first one.
template <typename T>
PSATD_HD cx<T>* spec_at(cx<T>* spec, const BoxD& bx, int64_t sbias, int f) {
  return spec + 9 * (bx.soff - sbias) + f * bx.svol;
}
template <typename T>
PSATD_HD const cx<T>* spec_at(const cx<T>* spec, const BoxD& bx, int64_t sbias, int f) {
  return spec + 9 * (bx.soff - sbias) + f * bx.svol;
}

// A batch of boxes [b0, b1) for the FFT/update passes: its work-item ranges
// and the spectral offset of box b0 (the workspace holds the batch only).
struct Batch {
  int32_t b0, b1;
  int32_t F0, nF, U0, nU, I0, nI;
  int64_t sbias;
};

// One rectangular piece of a box interior that is also a guard region of a
// padded box (a neighbour's, or the box's own when its padding wraps the
// grid): interior cells [z0, z0+lz) x [y0, y0+ly) x [x0, x0+lx) of the source
// box are the padded cells starting at (qz, qy, qx) of box dst.  Every guard
// cell of every box lies in exactly one piece of exactly one source box.
struct PushBlk {
  int32_t src, dst;
  int32_t z0, lz, qz;
  int32_t y0, ly, qy;
  int32_t x0, lx, qx;
};

// Register z pass: the padded z lengths with a register schedule, as
// X(N, lanes per transform, waves per work-group, min waves per SIMD).
#define PSATD_ZREG_SHAPES(X) \
  X(96, 2, 4, 2)             \
  X(176, 4, 4, 2)

// A group of boxes sharing one padded z length: its work list is
// itemsZR[off .. off + nsub] (a prefix over all boxes, zero for the others).
struct ZGroup {
  int32_t N, off, n, pad_;
};
constexpr int kMaxZGroups = 8;

// A launch class of the x/y passes: the boxes whose padded planes fit the
// same number of times into a compute unit's LDS, run with their own group
// size and dynamic LDS.  Its work lists are prefixes over all boxes (zero for
// the boxes of other classes) at the given offsets of one table: planes of the
// 9 fields (F), of one field (P), interior planes of the 6 outputs (I) and of
// one output (N), with their totals.
struct XyClass {
  int32_t nt, lds;
  int32_t F, nF, P, nP, I, nI, N, nN;
};
constexpr int kMaxXyClasses = 3;

// A launch class of the z pass: the boxes whose z tile takes the same number
// of pencils (FP32: the widest of 10, 8, 6 of which two tiles fit a compute
// unit's LDS, else 4; FP64: 8 where one tile fits, else 4), launched with the
// LDS of the class's longest padded z.  Work list: a prefix over all boxes at
// offset U of one table.
struct ZClass {
  int32_t PB, lds, U, nU;
};
constexpr int kMaxZClasses = 4;

// Pencils per work-group of the register z pass (9 fields share its lanes).
constexpr int zreg_pencils(int L, int W) { return (64 * W / L) / 9; }

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
  const double* kmod;     // modified wavenumbers (FP64)
};

// Copies total elements i -> dst(i, src(i)) with U loads in flight per
// thread (all U loads are issued before the first store).
template <int U, typename V, class Src, class Dst>
PSATD_HD void copy_batched(int total, int tid, int nt, Src src, Dst dst) {
  for (int base = tid; base < total; base += U * nt) {
    V v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = base + u * nt;
      if (i < total) v[u] = src(i);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int i = base + u * nt;
      if (i < total) dst(i, v[u]);
    }
  }
}

// Two neighbouring values accessed as one vector (aligned to its size, at
// most 16 bytes: the widest single access).
template <typename V>
struct alignas(2 * sizeof(V) < 16 ? 2 * sizeof(V) : 16) Pair {
  V a, b;
};

// Row-major R x C walk shared by a work-group: element i = tid + k nt, with
// its (row, col) advanced incrementally (no per-element division), in
// batches of U whose U loads are all issued before the first store; full
// batches run without bounds checks.  The remainder (fewer than U per
// thread) runs one element at a time, or with TAILB as one more guarded
// batch (fewer round trips to memory, more registers live at once).
// get(i, r, c) -> V, put(i, r, c, v).
template <int U, class V, bool TAILB = false, class Get, class Put>
PSATD_HD void copy_grid(int R, int C, int tid, int nt, Get get, Put put) {
  const int total = R * C;
  const FastDiv dC = make_fastdiv((uint32_t)C);
  int r = (int)fdiv((uint32_t)tid, dC);
  int c = tid - r * C;
  const int dr = (int)fdiv((uint32_t)nt, dC);
  const int dc = nt - dr * C;
  auto advance = [&](int& rr, int& cc) {
    cc += dc;
    rr += dr;
    if (cc >= C) {
      cc -= C;
      ++rr;
    }
  };
  int i = tid;
  for (; i + (U - 1) * nt < total; i += U * nt) {
    V v[U];
    int rs[U], cs[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      rs[u] = r;
      cs[u] = c;
      v[u] = get(i + u * nt, r, c);
      advance(r, c);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) put(i + u * nt, rs[u], cs[u], v[u]);
  }
  if (!TAILB) {
    for (; i < total; i += nt) {
      put(i, r, c, get(i, r, c));
      advance(r, c);
    }
  } else if (i < total) {  // the last, partial batch, its loads in flight together
    V v[U];
    int rs[U], cs[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      rs[u] = r;
      cs[u] = c;
      if (i + u * nt < total) v[u] = get(i + u * nt, r, c);
      advance(r, c);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i + u * nt < total) put(i + u * nt, rs[u], cs[u], v[u]);
  }
}

// The same walk over the pairs (e, e+1), e = 2 j, of a row-major R x C grid
// with R C even (a pair may straddle two rows): get(j, r0, c0, r1, c1) -> V,
// put(j, r0, c0, r1, c1, v), with (r1, c1) the position of e + 1.
template <int U, class V, bool TAILB = false, class Get, class Put>
PSATD_HD void copy_grid_pairs(int R, int C, int tid, int nt, Get get, Put put) {
  const int total = (R * C) >> 1;
  const FastDiv dC = make_fastdiv((uint32_t)C);
  int r = (int)fdiv((uint32_t)(2 * tid), dC);
  int c = 2 * tid - r * C;
  const int dr = (int)fdiv((uint32_t)(2 * nt), dC);
  const int dc = 2 * nt - dr * C;
  auto advance = [&](int& rr, int& cc) {
    cc += dc;
    rr += dr;
    if (cc >= C) {
      cc -= C;
      ++rr;
    }
  };
  auto second = [&](int rr, int cc, int& r1, int& c1) {
    const bool wrap = cc + 1 == C;
    r1 = wrap ? rr + 1 : rr;
    c1 = wrap ? 0 : cc + 1;
  };
  int j = tid;
  for (; j + (U - 1) * nt < total; j += U * nt) {
    V v[U];
    int rs[U], cs[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      rs[u] = r;
      cs[u] = c;
      int r1, c1;
      second(r, c, r1, c1);
      v[u] = get(j + u * nt, r, c, r1, c1);
      advance(r, c);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      int r1, c1;
      second(rs[u], cs[u], r1, c1);
      put(j + u * nt, rs[u], cs[u], r1, c1, v[u]);
    }
  }
  if (!TAILB) {
    for (; j < total; j += nt) {
      int r1, c1;
      second(r, c, r1, c1);
      put(j, r, c, r1, c1, get(j, r, c, r1, c1));
      advance(r, c);
    }
  } else if (j < total) {  // the last, partial batch
    V v[U];
    int rs[U], cs[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      rs[u] = r;
      cs[u] = c;
      int r1, c1;
      second(r, c, r1, c1);
      if (j + u * nt < total) v[u] = get(j + u * nt, r, c, r1, c1);
      advance(r, c);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (j + u * nt < total) {
        int r1, c1;
        second(rs[u], cs[u], r1, c1);
        put(j + u * nt, rs[u], cs[u], r1, c1, v[u]);
      }
  }
}

// The same walk over an A x B x C box (C fastest), the remainder always as a
// guarded batch: get(i, a, b, c), put(i, a, b, c, v).
template <int U, class V, class Get, class Put>
PSATD_HD void copy_grid3(int A, int B, int C, int tid, int nt, Get get, Put put) {
  const int total = A * B * C;
  const FastDiv dC = make_fastdiv((uint32_t)C);
  const FastDiv dB = make_fastdiv((uint32_t)B);
  auto split = [&](int v, int& a, int& b, int& c) {
    const int q = (int)fdiv((uint32_t)v, dC);
    c = v - q * C;
    a = (int)fdiv((uint32_t)q, dB);
    b = q - a * B;
  };
  int a, b, c, da, db, dc;
  split(tid, a, b, c);
  split(nt, da, db, dc);
  auto advance = [&](int& aa, int& bb, int& cc) {
    cc += dc;
    bb += db;
    aa += da;
    if (cc >= C) {
      cc -= C;
      ++bb;
    }
    if (bb >= B) {
      bb -= B;
      ++aa;
    }
  };
  int i = tid;
  for (; i + (U - 1) * nt < total; i += U * nt) {
    V v[U];
    int as[U], bs[U], cs[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      as[u] = a;
      bs[u] = b;
      cs[u] = c;
      v[u] = get(i + u * nt, a, b, c);
      advance(a, b, c);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) put(i + u * nt, as[u], bs[u], cs[u], v[u]);
  }
  if (i < total) {  // the last, partial batch
    V v[U];
    int as[U], bs[U], cs[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      as[u] = a;
      bs[u] = b;
      cs[u] = c;
      if (i + u * nt < total) v[u] = get(i + u * nt, a, b, c);
      advance(a, b, c);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i + u * nt < total) put(i + u * nt, as[u], bs[u], cs[u], v[u]);
  }
}

// Fused E,B guard exchange: after the inverse pass of interior plane zi (rows
// [ya, yb) of it held by this work-group), write the new values into every
// guard copy of those cells.  val(y, x) returns the new value of interior cell
// (y, x).  The pieces of a source box are visited in a uniform loop; rows of a
// piece are contiguous in the destination.
template <typename T, class Val>
PSATD_HD void push_guards(const PushBlk* blk, int b0, int b1, const BoxD* boxes, T* out, int zi,
                          int ya, int yb, Val val, int tid, int nt) {
  for (int b = b0; b < b1; ++b) {
    const PushBlk k = blk[b];
    if (zi < k.z0 || zi >= k.z0 + k.lz) continue;
    const int y_lo = ya > k.y0 ? ya : k.y0;
    const int y_hi = yb < k.y0 + k.ly ? yb : k.y0 + k.ly;
    if (y_lo >= y_hi) continue;
    const BoxD& d = boxes[k.dst];
    T* base = out + d.foff + ((int64_t)(k.qz + zi - k.z0) * d.P[1] + (k.qy + y_lo - k.y0)) * d.P[0] + k.qx;
    const int n = (y_hi - y_lo) * k.lx;
    const FastDiv dl = make_fastdiv((uint32_t)k.lx);
    for (int i = tid; i < n; i += nt) {
      const int r = (int)fdiv((uint32_t)i, dl);
      const int c = i - r * k.lx;
      base[(int64_t)r * d.P[0] + c] = val(y_lo + r, k.x0 + c);
    }
  }
}

// ------------------------------------------------------------------ pass F
// Forward R2C along x and C2C along y of one z-plane of one field of one box.
// Output: half spectrum plane [ky][kx] (kx = 0..H-1) in natural order.
// A guard region of a destination box seen from the box that owns it: the
// padded cells [qz, qz+lz) x [qy, qy+ly) x [qx, qx+lx) of the destination are
// the source's interior cells starting at element `so` (plane 0, row 0,
// column 0) with the source's plane and row pitches.  Every guard cell of a
// box lies in exactly one of its pull pieces.
struct PullPiece {
  int64_t so;
  int32_t sPl, sP0;
  int32_t qz, lz, qy, ly, qx, lx;
};

template <typename T>
struct FwdArgs {
  Tables<T> t;
  const int32_t* items;    // prefix over boxes of P[2] * nfield
  int32_t nfield;
  const T* in[9];
  cx<T>* spec;             // spectral workspace (box-major, see spec_at)
  int64_t sbias;           // spectral offset of the first box held by spec
  // Fields f < npull read their guard cells from the owners (pull pieces of
  // box s: pull[pull_off[s] .. pull_off[s+1])) instead of the box's own,
  // possibly stale, guard copies; npull = 0 reads every padded cell in place.
  int32_t npull;
  const PullPiece* pull;
  const int32_t* pull_off;
};

// Copies a rectangle of real cells src[r * sP0 + c] (r < ly, c < lx) into the
// LDS plane whose x rows are packed as complex pairs in stage-digit order:
// cell (y0 + r, x0 + c) goes to float 2 posx[(x0 + c) / 2] + (x0 + c) % 2 of
// row y0 + r.  Four cells per access when the rectangle and the source are
// 16-byte aligned, two when 8-byte aligned, else one.
template <typename T>
PSATD_HD void copy_rect_to_plane(const T* src, int sP0, int ly, int lx, int y0, int x0, cx<T>* lds, int ld,
                                 const int32_t* posx, int tid, int nt) {
  T* ldsT = reinterpret_cast<T*>(lds);
  const uintptr_t sa = reinterpret_cast<uintptr_t>(src);
  if (sizeof(T) == 4 && ((x0 | lx | sP0) & 3) == 0 && (sa & 15) == 0) {
    using Q = Pair<Pair<T>>;
    copy_grid<4, Q>(ly, lx >> 2, tid, nt,
                    [&](int, int r, int c4) { return *reinterpret_cast<const Q*>(src + (int64_t)r * sP0 + 4 * c4); },
                    [&](int, int r, int c4, Q v) {
                      cx<T>* row = lds + (y0 + r) * ld;
                      const int h = (x0 >> 1) + 2 * c4;
                      row[posx[h]] = cx<T>{v.a.a, v.a.b};
                      row[posx[h + 1]] = cx<T>{v.b.a, v.b.b};
                    });
  } else if (((x0 | lx | sP0) & 1) == 0 && (sa % sizeof(Pair<T>)) == 0) {
    copy_grid<8, Pair<T>>(ly, lx >> 1, tid, nt,
                          [&](int, int r, int c2) {
                            return *reinterpret_cast<const Pair<T>*>(src + (int64_t)r * sP0 + 2 * c2);
                          },
                          [&](int, int r, int c2, Pair<T> v) {
                            lds[(y0 + r) * ld + posx[(x0 >> 1) + c2]] = cx<T>{v.a, v.b};
                          });
  } else {
    copy_grid<8, T>(ly, lx, tid, nt, [&](int, int r, int c) { return src[(int64_t)r * sP0 + c]; },
                    [&](int, int r, int c, T v) {
                      const int x = x0 + c;
                      ldsT[2 * ((y0 + r) * ld + posx[x >> 1]) + (x & 1)] = v;
                    });
  }
}

// LDS: the plane [y][x] with row stride ld, then the twiddles of the x plan
// (Nh), the y plan (Py) and W_Px (real <-> half spectrum).
template <typename T, int MAXR, class Bar, class Eng = FftValu>
PSATD_HD void body_fwd_xy(const FwdArgs<T>& a, int item, int tid, int nt, cx<T>* lds, Bar bar, Eng eng = Eng{}) {
  const int s = find_box(a.items, a.t.nsub, item);
  const BoxD& bx = a.t.box[s];
  const int local = item - a.items[s];
  const int Px = bx.P[0], Py = bx.P[1], Pz = bx.P[2];
  const int f = local / Pz;
  const int z = local - f * Pz;
  const int Nh = Px >> 1, H = bx.H, ld = bx.ld;
  const FftPlanD* plx = a.t.plans + bx.planx;
  const FftPlanD* ply = a.t.plans + bx.plany;
  cx<T>* twx = lds + Py * ld;
  cx<T>* twy = twx + Nh;
  cx<T>* twr = twy + Py;
  int32_t* posx = reinterpret_cast<int32_t*>(twr + Px);
  int32_t* posy = posx + Nh;
  const cx<T>* gtx = a.t.tw + plx->tw;
  const cx<T>* gty = a.t.tw + ply->tw;
  const cx<T>* gtr = a.t.tw + bx.twr;

  // stage-digit positions along x (input of the dit) and y (output of the dif)
  for (int i = tid; i < Nh + Py; i += nt) {
    if (i < Nh) posx[i] = plan_pos(plx, i);
    else posy[i - Nh] = plan_pos(ply, i - Nh);
  }
  bar();
  // packed real rows (x natural) -> LDS rows in stage-digit order along x,
  // together with the three twiddle tables
  const cx<T>* src = reinterpret_cast<const cx<T>*>(a.in[f] + bx.foff + (int64_t)z * Py * Px);
  for (int i = tid; i < Nh + Py + Px; i += nt)  // twx, twy, twr are contiguous
    twx[i] = i < Nh ? gtx[i] : (i < Nh + Py ? gty[i - Nh] : gtr[i - Nh - Py]);
  if (f < a.npull) {
    // The box's own interior cells, then every guard region of this plane
    // from the box that owns it (Fig. 3 step 3 fused into the next push).
    // The waves share the rectangles (the interior in one row band per wave,
    // the pieces that meet the plane dealt round-robin), each copying its own
    // with its 64 lanes, so their memory round trips overlap.
    const int lane = tid & 63, wave = tid >> 6, nw = nt >> 6;
    const int gx = bx.g[0], gy = bx.g[1], gz = bx.g[2];
    const T* inf = a.in[f];
    int dealt = 0;
    if (z >= gz && z < gz + bx.n[2]) {
      const int ny = bx.n[1];
      const int r0 = (int)(((int64_t)ny * wave) / nw), r1 = (int)(((int64_t)ny * (wave + 1)) / nw);
      if (r1 > r0)
        copy_rect_to_plane<T>(inf + bx.foff + ((int64_t)z * Py + gy + r0) * Px + gx, Px, r1 - r0, bx.n[0], gy + r0,
                              gx, lds, ld, posx, lane, 64);
      dealt = nw;
    }
    for (int b = a.pull_off[s]; b < a.pull_off[s + 1]; ++b) {
      const PullPiece k = a.pull[b];
      if (z < k.qz || z >= k.qz + k.lz) continue;
      if (dealt++ % nw != wave) continue;
      copy_rect_to_plane<T>(inf + k.so + (int64_t)(z - k.qz) * k.sPl, k.sP0, k.ly, k.lx, k.qy, k.qx, lds, ld, posx,
                            lane, 64);
    }
  } else if ((Nh & 1) == 0 && (reinterpret_cast<uintptr_t>(src) % sizeof(Pair<cx<T>>)) == 0) {
    // two neighbouring complex values per access (rows of even length)
    const Pair<cx<T>>* src2 = reinterpret_cast<const Pair<cx<T>>*>(src);
    copy_grid<4, Pair<cx<T>>>(Py, Nh >> 1, tid, nt, [&](int i, int, int) { return src2[i]; },
                              [&](int, int y, int x2, Pair<cx<T>> v) {
                                cx<T>* row = lds + y * ld;
                                row[posx[2 * x2]] = v.a;
                                row[posx[2 * x2 + 1]] = v.b;
                              });
  } else {
    copy_grid<8, cx<T>>(Py, Nh, tid, nt, [&](int i, int, int) { return src[i]; },
                        [&](int, int y, int x, cx<T> v) { lds[y * ld + posx[x]] = v; });
  }
  bar();
  eng.template dit<-1, MAXR>(lds, Py, ld, 1, plx, twx, tid, nt, bar);
  pair_pass_rows<true>(lds, Py, ld, Nh, twr, tid, nt);
  bar();
  eng.template dif<-1, MAXR>(lds, H, 1, ld, ply, twy, tid, nt, bar);
  cx<T>* dst = spec_at(a.spec, bx, a.sbias, f) + (int64_t)z * Py * H;
  copy_grid<8, cx<T>>(Py, H, tid, nt, [&](int, int ky, int kx) { return lds[posy[ky] * ld + kx]; },
                      [&](int i, int, int, cx<T> v) { dst[i] = v; });
}

// ------------------------------------------------------------------ pass U
// Along z: forward C2C of 9 fields for a block of PB consecutive (ky, kx)
// pencils, the Eq. PSATD update at every k, backward C2C of the 6 results.
struct UpdConst {
  double c, dt;
};

// sin h and cos h in FP64: Cody-Waite reduction of h by multiples of pi/2
// (the two-term pi/2 leaves r within about 1e-16 of its true value for any
// |h| below 2^30), then the Taylor series of sin and cos on |r| <= pi/4 to
// the r^19 and r^18 terms (truncation below 1e-19), then the quadrant.
PSATD_HD void sincos_cw(double h, double* sh, double* ch) {
  const double two_over_pi = 0.63661977236758134308;
  const double pio2_hi = 1.5707963267948966;      // nearest double to pi/2
  const double pio2_lo = 6.123233995736766036e-17;  // pi/2 - pio2_hi
  const double n = rint(h * two_over_pi);
  const double r = fma(-n, pio2_lo, fma(-n, pio2_hi, h));
  const double r2 = r * r;
  // sin r = r (1 - r^2/3! + r^4/5! - ...), cos r = 1 - r^2/2! + r^4/4! - ...
  double ps = -1.0 / 121645100408832000.0;         // -1/19!
  ps = fma(ps, r2, 1.0 / 355687428096000.0);       // 1/17!
  ps = fma(ps, r2, -1.0 / 1307674368000.0);        // -1/15!
  ps = fma(ps, r2, 1.0 / 6227020800.0);            // 1/13!
  ps = fma(ps, r2, -1.0 / 39916800.0);             // -1/11!
  ps = fma(ps, r2, 1.0 / 362880.0);                // 1/9!
  ps = fma(ps, r2, -1.0 / 5040.0);                 // -1/7!
  ps = fma(ps, r2, 1.0 / 120.0);                   // 1/5!
  ps = fma(ps, r2, -1.0 / 6.0);                    // -1/3!
  const double s = fma(ps * r2, r, r);
  double pc = 1.0 / 6402373705728000.0;            // 1/18!
  pc = fma(pc, r2, -1.0 / 20922789888000.0);       // -1/16!
  pc = fma(pc, r2, 1.0 / 87178291200.0);           // 1/14!
  pc = fma(pc, r2, -1.0 / 479001600.0);            // -1/12!
  pc = fma(pc, r2, 1.0 / 3628800.0);               // 1/10!
  pc = fma(pc, r2, -1.0 / 40320.0);                // -1/8!
  pc = fma(pc, r2, 1.0 / 720.0);                   // 1/6!
  pc = fma(pc, r2, -1.0 / 24.0);                   // -1/4!
  pc = fma(pc, r2, 0.5);
  const double c = fma(-pc, r2, 1.0);
  const int q = (int)((int64_t)n & 3);
  *sh = q == 0 ? s : (q == 1 ? c : (q == 2 ? -s : -c));
  *ch = q == 0 ? c : (q == 1 ? -s : (q == 2 ? -c : s));
}

// The FP64 coefficients of Eqs. PSATD_1 / PSATD_2 at |[k]|^2 = k2 (Sec. 3.1):
// th = c |[k]| dt, C - 1 = -2 sin^2(th/2) (no cancellation), S/(ck),
// X1 = (1 - C)/|[k]|^2 = 2 sin^2(th/2)/|[k]|^2, X2 = (S/(ck) - dt)/|[k]|^2 (by
// its series below th = 0.1, where the difference cancels); the k -> 0
// limits at |[k]| = 0.  rc = 1/c.
struct Coef64 {
  double cm1, sck, x1, x2;
};

PSATD_HD Coef64 psatd_coef(double k2, double c, double rc, double dt) {
  Coef64 r;
  const double c2 = c * c;
  if (k2 == 0.0) {
    r.cm1 = 0.0;
    r.sck = dt;
    r.x1 = 0.5 * c2 * dt * dt;
    r.x2 = -c2 * dt * dt * dt / 6.0;
    return r;
  }
  const double rk = rsqrt(k2);
  const double rk2 = rk * rk;
  const double k = k2 * rk;
  const double h = 0.5 * c * dt * k;  // th / 2
  double sh, ch;
  sincos_cw(h, &sh, &ch);
  const double sh2 = sh * sh;
  r.cm1 = -2.0 * sh2;
  r.sck = (2.0 * sh * ch) * rk * rc;
  r.x1 = 2.0 * sh2 * rk2;
  const double t2 = 4.0 * h * h;
  if (t2 < 1e-2) {
    r.x2 = -c2 * dt * dt * dt *
           (1.0 / 6.0 - t2 * (1.0 / 120.0 - t2 * (1.0 / 5040.0 - t2 * (1.0 / 362880.0 - t2 / 39916800.0))));
  } else {
    r.x2 = (r.sck - dt) * rk2;
  }
  return r;
}

// Eqs. PSATD_1 / PSATD_2 (general c) at one k-point; coefficients in FP64.
//   E' = C E + i c^2 (S/ck) [k]xB - (S/ck) J + X1 [k]([k].E) + X2 [k]([k].J)
//   B' = C B - i (S/ck) [k]xE + i (X1/c^2) [k]xJ
// with the coefficients of psatd_coef.
//
// INC: return the increments E' - E and B' - B instead (C replaced by
// C - 1 = -2 sin^2(th/2), exact without cancellation).  The FP32 path moves the
// increment through the FFTs: for resolved fields it is far smaller than E,
// so the FFT roundoff, relative to what is transformed, shrinks with it.
// The coefficients of one k-point in the state's type T, evaluated in FP64
// and rounded once: C (or C - 1 for increments), S/(ck), X1, X2, c^2 S/(ck),
// X1/c^2, and the modified wave vector.
template <typename T>
struct UpdCoef {
  T C, S, X1, X2, a1, x1c, kx, ky, kz;
};

template <typename T, bool INC>
PSATD_HD UpdCoef<T> update_coef(double kx, double ky, double kz, double c, double rc, double dt) {
  const Coef64 cf = psatd_coef(kx * kx + ky * ky + kz * kz, c, rc, dt);
  UpdCoef<T> u;
  u.C = (T)(INC ? cf.cm1 : 1.0 + cf.cm1);
  u.S = (T)cf.sck;
  u.X1 = (T)cf.x1;
  u.X2 = (T)cf.x2;
  u.a1 = (T)(c * c * cf.sck);
  u.x1c = (T)(cf.x1 * (rc * rc));
  u.kx = (T)kx;
  u.ky = (T)ky;
  u.kz = (T)kz;
  return u;
}

// The update's multiply-adds in the state's type T (FP64 path: double; FP32
// path: float, where they act on increments).
template <typename T>
PSATD_HD void update_apply(T* vr, T* vi /* E0 E1 E2 B0 B1 B2 J0 J1 J2 */, const UpdCoef<T>& u) {
  T er[3], ei[3], br[3], bi[3], jr[3], ji[3];
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    er[a] = vr[a]; ei[a] = vi[a];
    br[a] = vr[3 + a]; bi[a] = vi[3 + a];
    jr[a] = vr[6 + a]; ji[a] = vi[6 + a];
  }
  const T tkx = u.kx, tky = u.ky, tkz = u.kz;
  const T K[3] = {tkx, tky, tkz};
  const T tC = u.C, tS = u.S, tX1 = u.X1, tX2 = u.X2, a1 = u.a1, x1c = u.x1c;
  const T kEr = tkx * er[0] + tky * er[1] + tkz * er[2];
  const T kEi = tkx * ei[0] + tky * ei[1] + tkz * ei[2];
  const T kJr = tkx * jr[0] + tky * jr[1] + tkz * jr[2];
  const T kJi = tkx * ji[0] + tky * ji[1] + tkz * ji[2];
  // cross products [k] x F, real and imaginary parts
  const T kxBr[3] = {tky * br[2] - tkz * br[1], tkz * br[0] - tkx * br[2], tkx * br[1] - tky * br[0]};
  const T kxBi[3] = {tky * bi[2] - tkz * bi[1], tkz * bi[0] - tkx * bi[2], tkx * bi[1] - tky * bi[0]};
  const T kxEr[3] = {tky * er[2] - tkz * er[1], tkz * er[0] - tkx * er[2], tkx * er[1] - tky * er[0]};
  const T kxEi[3] = {tky * ei[2] - tkz * ei[1], tkz * ei[0] - tkx * ei[2], tkx * ei[1] - tky * ei[0]};
  const T kxJr[3] = {tky * jr[2] - tkz * jr[1], tkz * jr[0] - tkx * jr[2], tkx * jr[1] - tky * jr[0]};
  const T kxJi[3] = {tky * ji[2] - tkz * ji[1], tkz * ji[0] - tkx * ji[2], tkx * ji[1] - tky * ji[0]};
#pragma unroll
  for (int a = 0; a < 3; ++a) {
    // i * z = (-z.i, z.r)
    vr[a] = tC * er[a] - a1 * kxBi[a] - tS * jr[a] + tX1 * K[a] * kEr + tX2 * K[a] * kJr;
    vi[a] = tC * ei[a] + a1 * kxBr[a] - tS * ji[a] + tX1 * K[a] * kEi + tX2 * K[a] * kJi;
    vr[3 + a] = tC * br[a] + tS * kxEi[a] - x1c * kxJi[a];
    vi[3 + a] = tC * bi[a] - tS * kxEr[a] + x1c * kxJr[a];
  }
}

// Eqs. PSATD_1 / PSATD_2 at one k-point: the coefficients (FP64, rounded to T
// once), then the multiply-adds in T.
template <typename T, bool INC = false>
PSATD_HD void psatd_point(T* vr, T* vi /* E0 E1 E2 B0 B1 B2 J0 J1 J2 */, double kx, double ky,
                          double kz, double c, double dt) {
  const double rc = 1.0 / c;  // uniform: hoisted out of the k-point loop
  update_apply<T>(vr, vi, update_coef<T, INC>(kx, ky, kz, c, rc, dt));
}

template <typename T>
struct UpdArgs {
  Tables<T> t;
  const int32_t* items;  // prefix over boxes of ceil(P[1] H / PB)
  cx<T>* spec;
  int64_t sbias;
  UpdConst k;
};

// The 9 fields of PB consecutive (ky, kx) pencils are staged in LDS as
// [z][f * PB + p] (W = 9 PB complex per z row), so that all 9 (then the 6
// output) fields are transformed by one multi-transform pass with a uniform
// element stride W.  Pencils past the end of the box (last block) are zeros.
template <typename T, int PB, bool INC, int MAXR, class Bar, class Eng = FftValu>
PSATD_HD void body_z_update(const UpdArgs<T>& a, int item, int tid, int nt, cx<T>* lds, Bar bar, Eng eng = Eng{}) {
  const int s = find_box(a.items, a.t.nsub, item);
  const BoxD& bx = a.t.box[s];
  const int blk = item - a.items[s];
  const int Py = bx.P[1], Pz = bx.P[2], H = bx.H;
  const int nq = Py * H;
  const int q0 = blk * PB;
  const int np = (nq - q0) < PB ? (nq - q0) : PB;
  const FftPlanD* plz = a.t.plans + bx.planz;
  constexpr int W = 9 * PB;
  cx<T>* twz = lds + Pz * W;
  int32_t* kzi = reinterpret_cast<int32_t*>(twz + Pz);  // frequency at each z slot
  const cx<T>* gtz = a.t.tw + plz->tw;
  for (int i = tid; i < Pz; i += nt) kzi[i] = plan_index(plz, i);
  const cx<T>* src = spec_at(a.spec, bx, a.sbias, 0) + q0;
  const int64_t slab = bx.svol;  // field stride
  for (int i = tid; i < Pz; i += nt) twz[i] = gtz[i];
  // a full tile whose pencil runs start at even offsets moves two neighbouring
  // pencils per access
  const bool pairs = (PB % 2) == 0 && np == PB &&
                     (((int64_t)nq | slab | (int64_t)(9 * (bx.soff - a.sbias) + q0)) & 1) == 0;
  if (pairs) {
    // up to 8 loads in flight per thread (a 96-plane FP32 tile of 8 pencils is
    // 6.75 pairs per thread of 512: one batch)
    copy_grid3<8, Pair<cx<T>>>(9, Pz, PB / 2, tid, nt,
        [&](int, int f, int z, int p2) {
          return *reinterpret_cast<const Pair<cx<T>>*>(src + f * slab + (int64_t)z * nq + 2 * p2);
        },
        [&](int, int f, int z, int p2, Pair<cx<T>> v) {
          *reinterpret_cast<Pair<cx<T>>*>(lds + z * W + f * PB + 2 * p2) = v;
        });
  } else {
    copy_grid3<8, cx<T>>(9, Pz, PB, tid, nt,
        [&](int, int f, int z, int p) {
          return (p < np) ? src[f * slab + (int64_t)z * nq + p] : cx<T>{T(0), T(0)};
        },
        [&](int, int f, int z, int p, cx<T> v) { lds[z * W + f * PB + p] = v; });
  }
  bar();
  eng.template dif<-1, MAXR>(lds, 9 * PB, 1, W, plz, twz, tid, nt, bar);

  const double* kxt = a.t.kmod + bx.kx;
  const double* kyt = a.t.kmod + bx.ky;
  const double* kzt = a.t.kmod + bx.kz;
  const FastDiv dH = make_fastdiv((uint32_t)H);
  for (int i = tid; i < Pz * PB; i += nt) {
    const int slot = i / PB;
    const int p = i % PB;
    if (p >= np) continue;
    cx<T>* row = lds + slot * W + p;
    T vr[9], vi[9];
#pragma unroll
    for (int f = 0; f < 9; ++f) {
      const cx<T> v = row[f * PB];
      vr[f] = v.x;
      vi[f] = v.y;
    }
    const int q = q0 + p;
    const int ky = (int)fdiv((uint32_t)q, dH);
    const int kx = q - ky * H;
    psatd_point<T, INC>(vr, vi, kxt[kx], kyt[ky], kzt[kzi[slot]], a.k.c, a.k.dt);
#pragma unroll
    for (int f = 0; f < 6; ++f) row[f * PB] = cx<T>{vr[f], vi[f]};
  }
  bar();
  eng.template dit<+1, MAXR>(lds, 6 * PB, 1, W, plz, twz, tid, nt, bar);

  // only the interior z-planes: the inverse pass reads nothing else (the guard
  // planes of E and B are rewritten by the exchange)
  const int gz = bx.g[2];
  cx<T>* dst = spec_at(a.spec, bx, a.sbias, 0) + q0 + (int64_t)gz * nq;
  const cx<T>* res = lds + gz * W;
  if (pairs) {
    copy_grid3<4, Pair<cx<T>>>(6, bx.n[2], PB / 2, tid, nt,
        [&](int, int f, int z, int p2) {
          return *reinterpret_cast<const Pair<cx<T>>*>(res + z * W + f * PB + 2 * p2);
        },
        [&](int, int f, int z, int p2, Pair<cx<T>> v) {
          *reinterpret_cast<Pair<cx<T>>*>(dst + f * slab + (int64_t)z * nq + 2 * p2) = v;
        });
    return;
  }
  copy_grid3<8, cx<T>>(6, bx.n[2], PB, tid, nt,
                       [&](int, int f, int z, int p) { return res[z * W + f * PB + p]; },
                       [&](int, int f, int z, int p, cx<T> v) {
                         if (p < np) dst[f * slab + (int64_t)z * nq + p] = v;
                       });
}

// ------------------------------------------------------- heat equation
// Sec. 5 names the diffusion equation among the initial-value problems the
// local-FFT method applies to: du/dt = D lap u, Laplacian symbol -|[k]|^2 with
// the same order-p modified wavenumbers, exact propagator per step.  The x/y
// passes are the field passes with one field; this is its z pass.
template <typename T>
struct HeatArgs {
  Tables<T> t;
  const int32_t* items;  // prefix over boxes of ceil(P[1] H / PB)
  cx<T>* spec;           // the half spectrum of u
  double D, dt;
};

// PB consecutive (ky, kx) pencils staged as [z][p]: forward z transform,
// multiply by g = exp(-D |[k]|^2 dt) in FP64 (INC: by g - 1 = expm1(...), the
// increment's spectrum), inverse z transform.
template <typename T, int PB, bool INC, int MAXR, class Bar, class Eng = FftValu>
PSATD_HD void body_z_heat(const HeatArgs<T>& a, int item, int tid, int nt, cx<T>* lds, Bar bar,
                          Eng eng = Eng{}) {
  const int s = find_box(a.items, a.t.nsub, item);
  const BoxD& bx = a.t.box[s];
  const int blk = item - a.items[s];
  const int Py = bx.P[1], Pz = bx.P[2], H = bx.H;
  const int nq = Py * H;
  const int q0 = blk * PB;
  const int np = (nq - q0) < PB ? (nq - q0) : PB;
  const FftPlanD* plz = a.t.plans + bx.planz;
  cx<T>* twz = lds + Pz * PB;
  int32_t* kzi = reinterpret_cast<int32_t*>(twz + Pz);
  const cx<T>* gtz = a.t.tw + plz->tw;
  for (int i = tid; i < Pz; i += nt) kzi[i] = plan_index(plz, i);
  cx<T>* col = spec_at(a.spec, bx, 0, 0) + q0;
  const int ndata = Pz * PB;
  copy_batched<8, cx<T>>(ndata + Pz, tid, nt,
      [&](int i) {
        if (i >= ndata) return gtz[i - ndata];
        const int p = i % PB;
        return (p < np) ? col[(int64_t)(i / PB) * nq + p] : cx<T>{T(0), T(0)};
      },
      [&](int i, cx<T> v) {
        if (i >= ndata) twz[i - ndata] = v;
        else lds[i] = v;
      });
  bar();
  eng.template dif<-1, MAXR>(lds, PB, 1, PB, plz, twz, tid, nt, bar);
  const double* kxt = a.t.kmod + bx.kx;
  const double* kyt = a.t.kmod + bx.ky;
  const double* kzt = a.t.kmod + bx.kz;
  const FastDiv dH = make_fastdiv((uint32_t)H);
  for (int i = tid; i < ndata; i += nt) {
    const int p = i % PB;
    if (p >= np) continue;
    const int q = q0 + p;
    const int ky = (int)fdiv((uint32_t)q, dH);
    const int kx = q - ky * H;
    const double k1 = kxt[kx], k2 = kyt[ky], k3 = kzt[kzi[i / PB]];
    const double e = -a.D * (k1 * k1 + k2 * k2 + k3 * k3) * a.dt;
    const T g = (T)(INC ? expm1(e) : exp(e));
    lds[i] = cx<T>{lds[i].x * g, lds[i].y * g};
  }
  bar();
  eng.template dit<+1, MAXR>(lds, PB, 1, PB, plz, twz, tid, nt, bar);
  // interior z-planes only (all the inverse pass reads)
  const int gz = bx.g[2];
  copy_batched<8, cx<T>>(bx.n[2] * PB, tid, nt, [&](int i) { return lds[gz * PB + i]; },
                         [&](int i, cx<T> v) {
                           const int p = i % PB;
                           if (p < np) col[(int64_t)(gz + i / PB) * nq + p] = v;
                         });
}

// ------------------------------------------------------------------ pass I
// Backward C2C along y and C2R along x of one interior z-plane of one of the 6
// output fields; writes the interior cells of the plane, scaled by 1/V.
template <typename T>
struct InvArgs {
  Tables<T> t;
  const int32_t* items;  // prefix over boxes of n[2] * 6
  const cx<T>* spec;
  int64_t sbias;
  T* out[6];
  const PushBlk* push;       // fused E,B guard exchange (null: a separate fill pass)
  const int32_t* push_off;   // pieces of box s: [push_off[s], push_off[s+1])
};

// LDS: the plane with row stride ld, then the twiddles of the y plan (Py),
// the x plan (Nh) and W_Px.
template <typename T, bool INC, int MAXR, bool PUSH = false, class Bar, class Eng = FftValu>
PSATD_HD void body_inv_xy(const InvArgs<T>& a, int item, int tid, int nt, cx<T>* lds, Bar bar, Eng eng = Eng{}) {
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
  cx<T>* twy = lds + Py * ld;
  cx<T>* twx = twy + Py;
  cx<T>* twr = twx + Nh;
  int32_t* posy = reinterpret_cast<int32_t*>(twr + Px);
  int32_t* posx = posy + Py;
  const cx<T>* gty = a.t.tw + ply->tw;
  const cx<T>* gtx = a.t.tw + plx->tw;
  const cx<T>* gtr = a.t.tw + bx.twr;

  // stage-digit positions along y (input of the dit) and x (output of the dif)
  for (int i = tid; i < Py + Nh; i += nt) {
    if (i < Py) posy[i] = plan_pos(ply, i);
    else posx[i - Py] = plan_pos(plx, i - Py);
  }
  bar();

  // half-spectrum rows (ky natural) -> LDS rows in stage-digit order along y
  const cx<T>* src = spec_at(a.spec, bx, a.sbias, f) + (int64_t)z * Py * H;
  for (int i = tid; i < Py + Nh + Px; i += nt)  // twy, twx, twr are contiguous
    twy[i] = i < Py ? gty[i] : (i < Py + Nh ? gtx[i - Py] : gtr[i - Py - Nh]);
  // FP32: two spectrum entries per access (measured slower in FP64)
  if (sizeof(T) == 4 && ((Py * H) & 1) == 0 && (reinterpret_cast<uintptr_t>(src) % sizeof(Pair<cx<T>>)) == 0) {
    const Pair<cx<T>>* src2 = reinterpret_cast<const Pair<cx<T>>*>(src);
    copy_grid_pairs<4, Pair<cx<T>>, true>(Py, H, tid, nt, [&](int j, int, int, int, int) { return src2[j]; },
        [&](int, int r0, int c0, int r1, int c1, Pair<cx<T>> v) {
          lds[posy[r0] * ld + c0] = v.a;
          lds[posy[r1] * ld + c1] = v.b;
        });
  } else {
    copy_grid<8, cx<T>, true>(Py, H, tid, nt, [&](int i, int, int) { return src[i]; },
                        [&](int, int ky, int kx, cx<T> v) { lds[posy[ky] * ld + kx] = v; });
  }
  bar();
  eng.template dit<+1, MAXR>(lds, H, 1, ld, ply, twy, tid, nt, bar);
  const int ny = bx.n[1], gy = bx.g[1];
  pair_pass_rows<false>(lds + gy * ld, ny, ld, Nh, twr, tid, nt);
  bar();
  eng.template dif<+1, MAXR>(lds + gy * ld, ny, ld, 1, plx, twx, tid, nt, bar);
  // 1/V applied in FP64 and rounded once: an FP32 1/V (not a power of two for
  // most V) would bias every step by the same relative amount.
  const double sc = 1.0 / ((double)Px * (double)Py * (double)Pz);
  const int nx = bx.n[0], gx = bx.g[0];
  T* dst = a.out[f] + bx.foff + (int64_t)z * Py * Px;
  [[maybe_unused]] T* ldsT = reinterpret_cast<T*>(lds);
  constexpr bool push = PUSH;  // the fused E,B exchange (compiled only where used)
  T* dst0 = dst + (int64_t)gy * Px + gx;  // first interior cell of the plane
  if (!push && sizeof(T) == 4 && (gx & 1) == 0 && (nx & 3) == 0 && (Px & 3) == 0 &&
      (reinterpret_cast<uintptr_t>(dst0) % sizeof(Pair<Pair<T>>)) == 0) {
    // FP32: four cells (two complex LDS entries, 16 bytes) per access
    const int hx = gx >> 1;
    using Q = Pair<Pair<T>>;
    copy_grid<4, Q>(ny, nx >> 2, tid, nt,
                    [&](int, int yy, int x4) {
                      const cx<T>* row = lds + (gy + yy) * ld;
                      const cx<T> v0 = row[posx[hx + 2 * x4]], v1 = row[posx[hx + 2 * x4 + 1]];
                      return Q{{(T)((double)v0.x * sc), (T)((double)v0.y * sc)},
                               {(T)((double)v1.x * sc), (T)((double)v1.y * sc)}};
                    },
                    [&](int, int yy, int x4, Q v) {
                      Q* q = reinterpret_cast<Q*>(dst0 + (int64_t)yy * Px) + x4;
                      if (INC) {  // v is the increment
                        const Q o = *q;
                        v.a.a = o.a.a + v.a.a;
                        v.a.b = o.a.b + v.a.b;
                        v.b.a = o.b.a + v.b.a;
                        v.b.b = o.b.b + v.b.b;
                      }
                      *q = v;
                    });
    return;
  }
  if (!push && ((gx | nx) & 1) == 0 && (reinterpret_cast<uintptr_t>(dst0) % sizeof(Pair<T>)) == 0) {
    // cells x, x+1 (x even) are the two halves of one complex LDS entry: one
    // LDS read and one 2-wide access per pair
    const int hx = gx >> 1;
    copy_grid<8, Pair<T>>(ny, nx >> 1, tid, nt,
                          [&](int, int yy, int x2) {
                            const cx<T> v = lds[(gy + yy) * ld + posx[hx + x2]];
                            return Pair<T>{(T)((double)v.x * sc), (T)((double)v.y * sc)};
                          },
                          [&](int, int yy, int x2, Pair<T> v) {
                            Pair<T>* q = reinterpret_cast<Pair<T>*>(dst0 + (int64_t)yy * Px) + x2;
                            if (INC) {  // v is the increment
                              const Pair<T> o = *q;
                              v.a = o.a + v.a;
                              v.b = o.b + v.b;
                            }
                            *q = v;
                          });
    return;
  }
  copy_grid<8, T>(ny, nx, tid, nt,
                  [&](int, int yy, int xi) {
                    const int x = gx + xi;
                    const cx<T> v = lds[(gy + yy) * ld + posx[x >> 1]];
                    return (T)((double)((x & 1) ? v.y : v.x) * sc);
                  },
                  [&](int, int yy, int xi, T v) {
                    const int x = gx + xi;
                    T* q = dst + (gy + yy) * Px + x;
                    const T nv = INC ? *q + v : v;  // INC: v is the increment
                    *q = nv;
                    // the new value back into its own LDS slot for the guard copies
                    if constexpr (push) ldsT[2 * ((gy + yy) * ld + posx[x >> 1]) + (x & 1)] = nv;
                  });
  if constexpr (push) {
    bar();
    push_guards<T>(a.push, a.push_off[s], a.push_off[s + 1], a.t.box, a.out[f], z - bx.g[2], 0, ny,
                   [&](int yi, int xi) {
                     const int x = gx + xi;
                     return ldsT[2 * ((gy + yi) * ld + posx[x >> 1]) + (x & 1)];
                   },
                   tid, nt);
  }
}

// ------------------------------------------------ split x / y passes
// For padded planes larger than the LDS the x/y pass is split: x rows and y
// columns are transformed by separate work items through the workspace
// (natural order in memory between the two).  RB rows / CB columns per item.
constexpr int kRB = 16;
constexpr int kCB = 16;

template <typename T>
struct SplitArgs {
  Tables<T> t;
  const int32_t* items;
  const T* in[9];      // x forward: field inputs
  T* out[6];           // x inverse: field outputs
  cx<T>* spec;
  int64_t sbias;
  const PushBlk* push;       // x inverse: fused E,B guard exchange (or null)
  const int32_t* push_off;
};

// x forward: kRB rows of (box, z, field): packed real rows -> half spectrum rows.
template <typename T, int MAXR, class Bar, class Eng = FftValu>
PSATD_HD void body_x_fwd(const SplitArgs<T>& a, int item, int tid, int nt, cx<T>* lds, Bar bar, Eng eng = Eng{}) {
  const int s = find_box(a.items, a.t.nsub, item);
  const BoxD& bx = a.t.box[s];
  const int Px = bx.P[0], Py = bx.P[1], Pz = bx.P[2];
  const int nrb = (Py + kRB - 1) / kRB;
  const int local = item - a.items[s];
  const int f = local / (Pz * nrb);
  const int r = local - f * Pz * nrb;
  const int z = r / nrb;
  const int y0 = (r - z * nrb) * kRB;
  const int ny = (Py - y0) < kRB ? (Py - y0) : kRB;
  const int Nh = Px >> 1, H = bx.H, ld = bx.ld;
  const FftPlanD* plx = a.t.plans + bx.planx;
  cx<T>* twx = lds + kRB * ld;
  cx<T>* twr = twx + Nh;
  int32_t* posx = reinterpret_cast<int32_t*>(twr + Px);
  for (int i = tid; i < Nh; i += nt) posx[i] = plan_pos(plx, i);
  bar();
  const cx<T>* src = reinterpret_cast<const cx<T>*>(a.in[f] + bx.foff + ((int64_t)z * Py + y0) * Px);
  const cx<T>* gtx = a.t.tw + plx->tw;
  const cx<T>* gtr = a.t.tw + bx.twr;
  const int nrow = ny * Nh;
  const FastDiv dNh = make_fastdiv((uint32_t)Nh);
  copy_batched<8, cx<T>>(nrow + Nh + Px, tid, nt,
                         [&](int i) {
                           if (i < nrow) return src[i];
                           const int j = i - nrow;
                           return j < Nh ? gtx[j] : gtr[j - Nh];
                         },
                         [&](int i, cx<T> v) {
                           if (i < nrow) {
                             const int y = (int)fdiv((uint32_t)i, dNh);
                             lds[y * ld + posx[i - y * Nh]] = v;
                           } else {
                             twx[i - nrow] = v;  // twx, twr contiguous
                           }
                         });
  bar();
  eng.template dit<-1, MAXR>(lds, ny, ld, 1, plx, twx, tid, nt, bar);
  pair_pass_rows<true>(lds, ny, ld, Nh, twr, tid, nt);
  bar();
  cx<T>* dst = spec_at(a.spec, bx, a.sbias, f) + ((int64_t)z * Py + y0) * H;
  const FastDiv dH = make_fastdiv((uint32_t)H);
  copy_batched<8, cx<T>>(ny * H, tid, nt,
                         [&](int i) {
                           const int y = (int)fdiv((uint32_t)i, dH);
                           return lds[y * ld + (i - y * H)];
                         },
                         [&](int i, cx<T> v) { dst[i] = v; });
}

// y columns: kCB half-spectrum columns of (box, z, field), in place in the
// workspace; DIR -1: forward over all planes and 9 fields; +1: inverse over
// interior planes and the 6 outputs.
template <typename T, int DIR, int MAXR, class Bar, class Eng = FftValu>
PSATD_HD void body_y(const SplitArgs<T>& a, int item, int tid, int nt, cx<T>* lds, Bar bar, Eng eng = Eng{}) {
  const int s = find_box(a.items, a.t.nsub, item);
  const BoxD& bx = a.t.box[s];
  const int Py = bx.P[1], H = bx.H;
  const int ncb = (H + kCB - 1) / kCB;
  const int nzp = DIR < 0 ? bx.P[2] : bx.n[2];
  const int local = item - a.items[s];
  const int f = local / (nzp * ncb);
  const int r = local - f * nzp * ncb;
  const int zz = r / ncb;
  const int z = DIR < 0 ? zz : bx.g[2] + zz;
  const int c0 = (r - zz * ncb) * kCB;
  const int nc = (H - c0) < kCB ? (H - c0) : kCB;
  const FftPlanD* ply = a.t.plans + bx.plany;
  cx<T>* twy = lds + Py * kCB;
  int32_t* posy = reinterpret_cast<int32_t*>(twy + Py);
  for (int i = tid; i < Py; i += nt) posy[i] = plan_pos(ply, i);
  bar();
  cx<T>* col = spec_at(a.spec, bx, a.sbias, f) + (int64_t)z * Py * H + c0;
  const cx<T>* gty = a.t.tw + ply->tw;
  const int ntot = Py * kCB;
  copy_batched<8, cx<T>>(ntot + Py, tid, nt,
                         [&](int i) {
                           if (i >= ntot) return gty[i - ntot];
                           const int y = i / kCB, c = i % kCB;
                           return c < nc ? col[(int64_t)y * H + c] : cx<T>{T(0), T(0)};
                         },
                         [&](int i, cx<T> v) {
                           if (i >= ntot) {
                             twy[i - ntot] = v;
                             return;
                           }
                           const int y = i / kCB, c = i % kCB;
                           lds[(DIR < 0 ? y : posy[y]) * kCB + c] = v;
                         });
  bar();
  if (DIR < 0)
    eng.template dif<-1, MAXR>(lds, nc, 1, kCB, ply, twy, tid, nt, bar);
  else
    eng.template dit<+1, MAXR>(lds, nc, 1, kCB, ply, twy, tid, nt, bar);
  copy_batched<8, cx<T>>(ntot, tid, nt,
                         [&](int i) {
                           const int y = i / kCB, c = i % kCB;
                           return lds[(DIR < 0 ? posy[y] : y) * kCB + c];
                         },
                         [&](int i, cx<T> v) {
                           const int y = i / kCB, c = i % kCB;
                           if (c < nc) col[(int64_t)y * H + c] = v;
                         });
}

// x inverse: kRB interior rows of (box, interior z, output field):
// half spectrum rows -> real rows, interior cells written (INC: added).
template <typename T, bool INC, int MAXR, bool PUSH = false, class Bar, class Eng = FftValu>
PSATD_HD void body_x_inv(const SplitArgs<T>& a, int item, int tid, int nt, cx<T>* lds, Bar bar, Eng eng = Eng{}) {
  const int s = find_box(a.items, a.t.nsub, item);
  const BoxD& bx = a.t.box[s];
  const int Px = bx.P[0], Py = bx.P[1], Pz = bx.P[2];
  const int nyi = bx.n[1], nz = bx.n[2];
  const int nrb = (nyi + kRB - 1) / kRB;
  const int local = item - a.items[s];
  const int f = local / (nz * nrb);
  const int r = local - f * nz * nrb;
  const int zz = r / nrb;
  const int z = bx.g[2] + zz;
  const int yy0 = (r - zz * nrb) * kRB;
  const int ny = (nyi - yy0) < kRB ? (nyi - yy0) : kRB;
  const int y0 = bx.g[1] + yy0;
  const int Nh = Px >> 1, H = bx.H, ld = bx.ld;
  const FftPlanD* plx = a.t.plans + bx.planx;
  cx<T>* twx = lds + kRB * ld;
  cx<T>* twr = twx + Nh;
  int32_t* posx = reinterpret_cast<int32_t*>(twr + Px);
  for (int i = tid; i < Nh; i += nt) posx[i] = plan_pos(plx, i);
  const cx<T>* src = spec_at(a.spec, bx, a.sbias, f) + ((int64_t)z * Py + y0) * H;
  const cx<T>* gtx = a.t.tw + plx->tw;
  const cx<T>* gtr = a.t.tw + bx.twr;
  const int nrow = ny * H;
  const FastDiv dH = make_fastdiv((uint32_t)H);
  copy_batched<8, cx<T>>(nrow + Nh + Px, tid, nt,
                         [&](int i) {
                           if (i < nrow) return src[i];
                           const int j = i - nrow;
                           return j < Nh ? gtx[j] : gtr[j - Nh];
                         },
                         [&](int i, cx<T> v) {
                           if (i < nrow) {
                             const int y = (int)fdiv((uint32_t)i, dH);
                             lds[y * ld + (i - y * H)] = v;
                           } else {
                             twx[i - nrow] = v;
                           }
                         });
  bar();
  pair_pass_rows<false>(lds, ny, ld, Nh, twr, tid, nt);
  bar();
  eng.template dif<+1, MAXR>(lds, ny, ld, 1, plx, twx, tid, nt, bar);
  const double sc = 1.0 / ((double)Px * (double)Py * (double)Pz);
  const int nx = bx.n[0], gx = bx.g[0];
  T* dst = a.out[f] + bx.foff + ((int64_t)z * Py + y0) * Px;
  const FastDiv dnx = make_fastdiv((uint32_t)nx);
  [[maybe_unused]] T* ldsT = reinterpret_cast<T*>(lds);
  constexpr bool push = PUSH;  // the fused E,B exchange (compiled only where used)
  copy_batched<8, T>(ny * nx, tid, nt,
                     [&](int i) {
                       const int y = (int)fdiv((uint32_t)i, dnx);
                       const int x = gx + (i - y * nx);
                       const cx<T> v = lds[y * ld + posx[x >> 1]];
                       return (T)((double)((x & 1) ? v.y : v.x) * sc);
                     },
                     [&](int i, T v) {
                       const int y = (int)fdiv((uint32_t)i, dnx);
                       const int x = gx + (i - y * nx);
                       T* q = dst + y * Px + x;
                       const T nv = INC ? *q + v : v;
                       *q = nv;
                       if constexpr (push) ldsT[2 * (y * ld + posx[x >> 1]) + (x & 1)] = nv;
                     });
  if constexpr (push) {
    bar();
    push_guards<T>(a.push, a.push_off[s], a.push_off[s + 1], a.t.box, a.out[f], zz, yy0, yy0 + ny,
                   [&](int yi, int xi) {
                     const int x = gx + xi;
                     return ldsT[2 * ((yi - yy0) * ld + posx[x >> 1]) + (x & 1)];
                   },
                   tid, nt);
  }
}

// --------------------------------------------------------------- exchange

// A guard piece as the fill reads it: the first cell of its first z-plane in
// the owner's interior and in the destination's guard region, and the
// pitches, worked out on the host (one load per work item instead of a chain
// through the piece and both box descriptors).
struct FillPiece {
  int64_t so, dof;    // first cell (plane 0): owner, destination
  int32_t sPl, dPl;   // plane pitches (elements)
  int32_t sP0, dP0;   // row pitches (elements)
  int32_t ly, lx;     // rows per plane, row length
  int32_t vec, pad_;  // 16-byte accesses: offsets, pitches and lx multiples of 16 bytes
};

template <typename T>
struct FillArgs {
  const FillPiece* piece;   // guard pieces (each guard cell in exactly one)
  const int32_t* items;     // prefix over pieces of lz
  const int32_t* piece_of;  // item -> piece
  int32_t ncomp;
  T* comp[9];
};

// 16 bytes of T, copied as one vector access.
template <typename T>
struct alignas(16) Vec16 {
  T v[16 / sizeof(T)];
};

// Fig. 3 step 3: every guard cell takes the value of the owner of its global
// index (mod N).  One item = one z-plane of one guard piece: ly rows of lx
// cells, contiguous in the owner's interior and in the destination's guard
// region, copied for every component (16-byte accesses when rows and bases
// are 16-byte aligned).
template <typename T>
PSATD_HD void body_fill(const FillArgs<T>& a, int item, int tid, int nt) {
  const int b = a.piece_of[item];
  const FillPiece k = a.piece[b];
  const int zi = item - a.items[b];
  const int sP0 = k.sP0, dP0 = k.dP0;
  const int64_t so = k.so + (int64_t)zi * k.sPl;
  const int64_t dof = k.dof + (int64_t)zi * k.dPl;
  constexpr int V = 16 / (int)sizeof(T);
  const bool vec = k.vec != 0;
  const int W = vec ? V : 1;  // elements per access
  const int lw = k.lx / W;
  const int n = k.ly * lw;
  const FastDiv dn = make_fastdiv((uint32_t)n);
  const FastDiv dl = make_fastdiv((uint32_t)lw);
  auto at = [&](int i, int64_t base, int pitch, int& c) {
    c = (int)fdiv((uint32_t)i, dn);
    const int e = i - c * n;
    const int r = (int)fdiv((uint32_t)e, dl);
    return base + (int64_t)r * pitch + (int64_t)(e - r * lw) * W;
  };
  if (vec) {
    copy_batched<4, Vec16<T>>(n * a.ncomp, tid, nt,
        [&](int i) {
          int c;
          const int64_t o = at(i, so, sP0, c);
          return *reinterpret_cast<const Vec16<T>*>(a.comp[c] + o);
        },
        [&](int i, Vec16<T> v) {
          int c;
          const int64_t o = at(i, dof, dP0, c);
          *reinterpret_cast<Vec16<T>*>(a.comp[c] + o) = v;
        });
  } else {
    copy_batched<8, T>(n * a.ncomp, tid, nt,
        [&](int i) {
          int c;
          const int64_t o = at(i, so, sP0, c);  // sets c before the buffer is chosen
          return a.comp[c][o];
        },
        [&](int i, T v) {
          int c;
          const int64_t o = at(i, dof, dP0, c);
          a.comp[c][o] = v;
        });
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
