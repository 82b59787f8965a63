// Host-side planning of the local-FFT PSATD step (no HIP runtime calls):
// validation of the decomposition (Sec. 3.2: boxes tiling the periodic grid,
// guard cells per side), per-box padded extents, FFT radix schedules and their
// twiddle / position tables, modified-wavenumber table layout (Sec. 3.1),
// owner lookup, neighbour lists and the work lists of every phase.
#pragma once
#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <tuple>
#include <vector>

#include "psatd.h"
#include "psatd_device.hpp"

namespace psatd {

// ------------------------------------------------------------ host tables
struct HostTables {
  int64_t N[3];
  double d[3];
  int nsub;
  int p;
  double dt, c;
  int prec, jmode;
  std::vector<BoxD> box;
  std::vector<FftPlanD> plans;
  std::vector<long double> twr, twi;  // all twiddle tables, forward sign
  std::vector<KEntry> kent;
  int32_t kmod_len = 0;
  int32_t kmax_len = 0;
  std::vector<int32_t> cut[3];
  int32_t ncut[3];
  std::vector<int32_t> owner;
  std::vector<int32_t> nbr_off, nbr;
  std::vector<int32_t> itemsF, itemsU, itemsI, itemsP, itemsN;
  std::vector<int32_t> itemsXF, itemsYF, itemsYI, itemsXI;  // split x/y passes
  bool split = false;  // x/y pass split into x rows and y columns (large planes)
  std::vector<PushBlk> push;      // fused E,B exchange: guard pieces per source box
  std::vector<int32_t> push_off;  // nsub + 1
  std::vector<FillPiece> fillp;   // guard fill: the pieces with offsets and pitches
  std::vector<int32_t> itemsG;    // guard fill: prefix over pieces of their z extent
  std::vector<int32_t> pieceOf;   // guard fill: item -> piece
  bool fuse_eb = false;           // E,B guards written by the inverse pass
  std::vector<PullPiece> pullp;   // guard regions per destination box, for the forward pass
  std::vector<int32_t> pull_off;  // nsub + 1
  bool pull_eb = false;           // the forward pass reads E,B guard cells from their owners
  int ldsX = 0, ldsY = 0;
  std::vector<Batch> batches;
  int64_t batch_slab = 0;     // complex elements of one spectral field slab of the largest batch
  int32_t batch_boxes = 0;
  int64_t field_elems = 0;
  int64_t slab = 0;
  int ldsF = 0, ldsI = 0, ldsU = 0, PB = 0;
  int maxr = 16;      // largest radix of the x/y schedules (8 or 16; 11 always)
  int maxrz = 16;     // largest radix of the z schedules
  std::vector<char> plan_z;  // per plan: 1 if it is a z schedule
  int spl = 0;        // BF16 terms of the matrix-core first stage (0: VALU form)
  int ntxy = 512;     // threads per work-group of the x/y passes
  int ntu = 512;      // threads per work-group of the z-update (1024 for FP32 by default)
  bool zreg = false;  // the register z pass applies (FP32 VALU form, every padded z length scheduled)
  std::vector<int32_t> boxlds;     // dynamic LDS bytes of one x/y plane of each box
  std::vector<XyClass> xyc;       // x/y launch classes (empty: one launch for every box)
  std::vector<int32_t> itemsXYC;  // their work lists
  std::vector<ZClass> zcls;       // z launch classes (empty: one tile size for every box)
  std::vector<int32_t> itemsZC;   // their work lists
  std::vector<ZGroup> zgroups;    // one per distinct padded z length
  std::vector<int32_t> itemsZR;   // their work lists, nsub + 1 prefix entries each
};

inline bool is_f64(int prec) { return prec == PSATD_F64; }
inline size_t real_size(int prec) { return is_f64(prec) ? 8 : 4; }

// Radix schedules: maxr 16 allows every codelet, maxr 8 the radices up to 8 plus 11.
// Every factorisation of n into exactly `left` radices from R (ordered as in R).
inline void factor_all(int n, int left, const int* R, int nr, std::vector<int>& acc,
                       std::vector<std::vector<int>>& out) {
  if (left == 0) {
    if (n == 1) out.push_back(acc);
    return;
  }
  for (int i = 0; i < nr; ++i) {
    if (n % R[i]) continue;
    acc.push_back(R[i]);
    factor_all(n / R[i], left - 1, R, nr, acc, out);
    acc.pop_back();
  }
}

// Fewest stages; among those the most balanced (largest smallest radix: fewer
// index operations per element in the small-radix stage), then the largest
// first radix.
inline bool factorize(int N, std::vector<int>& out, int maxr = 16) {
  static const int R16[] = {16, 12, 11, 10, 8, 7, 6, 5, 4, 3, 2};
  static const int R8[] = {11, 8, 7, 6, 5, 4, 3, 2};
  const int* R = maxr >= 16 ? R16 : R8;
  const int nr = maxr >= 16 ? 11 : 8;
  out.clear();
  if (N == 1) return true;
  for (int depth = 1; depth <= kMaxStages; ++depth) {
    std::vector<std::vector<int>> all;
    std::vector<int> acc;
    factor_all(N, depth, R, nr, acc, all);
    if (all.empty()) continue;
    const std::vector<int>* best = nullptr;
    int bmin = -1, bfirst = -1;
    for (const auto& f : all) {
      const int mn = *std::min_element(f.begin(), f.end());
      if (mn > bmin || (mn == bmin && f[0] > bfirst)) {
        best = &f;
        bmin = mn;
        bfirst = f[0];
      }
    }
    out = *best;
    return true;
  }
  return false;
}

// Schedule of a transform: with a matrix-core first stage (spl > 0) every
// length divisible by 16 starts with radix 16, the rest as factorize().
inline bool schedule(int N, std::vector<int>& out, int maxr, int spl) {
  if (spl > 0 && N % 16 == 0) {
    std::vector<int> rest;
    if (!factorize(N / 16, rest, maxr) || rest.size() + 1 > (size_t)kMaxStages) return false;
    out.assign(1, 16);
    out.insert(out.end(), rest.begin(), rest.end());
    return true;
  }
  return factorize(N, out, maxr);
}

// Fills the stage fields of a plan of length pl.N from a radix list.
inline void set_stages(FftPlanD& pl, const std::vector<int>& rad) {
  const int N = pl.N;
  pl.nstages = (int)rad.size();
  int prod = 1;
  for (int st = 0; st < kMaxStages; ++st) {
    if (st < pl.nstages) {
      pl.radix[st] = rad[st];
      pl.prod[st] = prod;
      prod *= rad[st];
      pl.stride[st] = N / prod;
    } else {
      pl.radix[st] = 1;
      pl.prod[st] = prod;
      pl.stride[st] = 1;
    }
    pl.rdiv[st] = make_fastdiv((uint32_t)pl.radix[st]);
    pl.sdiv[st] = make_fastdiv((uint32_t)pl.stride[st]);
  }
}

inline bool small_primes_only(int64_t n) {
  for (int p : {2, 3, 5, 7, 11})
    while (n % p == 0) n /= p;
  return n == 1;
}

// Writes the N-entry twiddle table of a plan (at pl.tw) for its current radix
// schedule: by stage and butterfly, W_N^{j t prod_s} for j < stride_s,
// t = 1..radix_s-1, then ones up to N entries.  Sets pl.twoff.
inline void write_plan_twiddles(HostTables& h, FftPlanD& pl) {
  const int N = pl.N;
  const long double PI = 3.141592653589793238462643383279502884L;
  int o = 0;
  for (int st = 0; st < kMaxStages; ++st) {
    pl.twoff[st] = o;
    if (st >= pl.nstages) continue;
    for (int j = 0; j < pl.stride[st]; ++j)
      for (int t = 1; t < pl.radix[st]; ++t, ++o) {
        const int64_t e = (int64_t)j * t * pl.prod[st];  // < N
        h.twr[pl.tw + o] = cosl(2.0L * PI * e / N);
        h.twi[pl.tw + o] = -sinl(2.0L * PI * e / N);
      }
  }
  for (; o < N; ++o) {  // the stages take N - 1 entries
    h.twr[pl.tw + o] = 1.0L;
    h.twi[pl.tw + o] = 0.0L;
  }
}

// Adds (or finds) an FFT plan of length N for the x/y passes or (zp) the z
// pass, which keep schedules of their own (each pass has its largest radix);
// returns its index or -1.
inline int add_plan(HostTables& h, int N, bool zp) {
  for (size_t i = 0; i < h.plans.size(); ++i)
    if (h.plans[i].N == N && (h.plan_z[i] != 0) == zp) return (int)i;
  std::vector<int> rad;
  if (!schedule(N, rad, zp ? h.maxrz : h.maxr, h.spl)) return -1;
  FftPlanD pl{};
  pl.N = N;
  set_stages(pl, rad);
  pl.tw = (int32_t)h.twr.size();
  h.twr.resize(h.twr.size() + N);
  h.twi.resize(h.twi.size() + N);
  write_plan_twiddles(h, pl);
  h.plans.push_back(pl);
  h.plan_z.push_back(zp ? 1 : 0);
  return (int)h.plans.size() - 1;
}

// twiddle table W_N^e without a plan (real <-> half spectrum, N = padded x)
inline int add_twiddle(HostTables& h, int N, std::vector<std::pair<int, int>>& cache) {
  for (auto& c : cache)
    if (c.first == N) return c.second;
  const int off = (int)h.twr.size();
  const long double PI = 3.141592653589793238462643383279502884L;
  for (int e = 0; e < N; ++e) {
    h.twr.push_back(cosl(2.0L * PI * e / N));
    h.twi.push_back(-sinl(2.0L * PI * e / N));
  }
  cache.push_back({N, off});
  return off;
}

inline int add_kentry(HostTables& h, int N, double du) {
  for (auto& k : h.kent)
    if (k.N == N && k.du == du) return k.off;
  KEntry k;
  k.N = N;
  k.du = du;
  k.off = h.kmod_len;
  h.kmod_len += N;
  h.kmax_len = std::max(h.kmax_len, N);
  h.kent.push_back(k);
  return k.off;
}

// Groups of consecutive boxes pushed through the FFT/update passes together.
inline void set_batches(HostTables& h, int per) {
  h.batch_boxes = per;
  if (per <= 0 || per > h.nsub) per = h.nsub;
  h.batches.clear();
  h.batch_slab = 0;
  for (int b0 = 0; b0 < h.nsub; b0 += per) {
    const int b1 = std::min(h.nsub, b0 + per);
    Batch b;
    b.b0 = b0;
    b.b1 = b1;
    b.F0 = h.itemsF[b0];
    b.nF = h.itemsF[b1] - h.itemsF[b0];
    b.U0 = h.itemsU[b0];
    b.nU = h.itemsU[b1] - h.itemsU[b0];
    b.I0 = h.itemsI[b0];
    b.nI = h.itemsI[b1] - h.itemsI[b0];
    b.sbias = h.box[b0].soff;
    const int64_t end = (b1 < h.nsub) ? h.box[b1].soff : h.slab;
    h.batch_slab = std::max(h.batch_slab, end - b.sbias);
    h.batches.push_back(b);
  }
}

// Work list of the z-update for a tile of PB pencils (9 fields staged in LDS,
// plus the z twiddles).
inline void set_z_tile(HostTables& h, int PB) {
  const int csz = (int)(2 * real_size(h.prec));
  int maxPz = 0;
  h.itemsU.assign(h.nsub + 1, 0);
  for (int s = 0; s < h.nsub; ++s) {
    const BoxD& b = h.box[s];
    h.itemsU[s + 1] = h.itemsU[s] + (int32_t)(((int64_t)b.P[1] * b.H + PB - 1) / PB);
    maxPz = std::max(maxPz, b.P[2]);
  }
  h.PB = PB;
  h.ldsU = maxPz * (9 * PB + 1) * csz + maxPz * 4;  // staged fields, z twiddles, z indices
  if (!h.batches.empty()) set_batches(h, h.batch_boxes);
}

inline bool z_tile_fits(const HostTables& h, int maxPz, int PB) {
  const int csz = (int)(2 * real_size(h.prec));
  return (int64_t)maxPz * (9 * PB + 1) * csz + maxPz * 4 <= kMaxDynLds;
}

// Dynamic LDS of a z tile of PB pencils of padded z length Pz.
inline int64_t z_tile_lds(const HostTables& h, int Pz, int PB) {
  return (int64_t)Pz * (9 * PB + 1) * (int64_t)(2 * real_size(h.prec)) + (int64_t)Pz * 4;
}

// Pencils per z tile of one box on its own.  FP32: the widest of 10, 8 and 6
// pencils of which two tiles fit a compute unit's LDS (the 128-VGPR kernel
// holds two tiles per CU whatever their width, and wider tiles read longer
// runs: 96^3 boxes with 10 instead of 8 pencils, step 2.72 -> 2.69 ms;
// 176^3 boxes with 6 instead of 4, z pass 30.3 -> 26.5 ms), else 4.  FP64: 8
// where one tile fits, else 4.  0 when not even a 4-pencil tile fits.
inline int z_pencils_for(const HostTables& h, int Pz) {
  if (is_f64(h.prec)) {
    if (z_tile_lds(h, Pz, 8) <= kMaxDynLds) return 8;
  } else {
    for (int PB : {10, 8, 6})
      if (2 * z_tile_lds(h, Pz, PB) <= kMaxDynLds) return PB;
  }
  return z_tile_lds(h, Pz, 4) <= kMaxDynLds ? 4 : 0;
}

// Launch classes of the z pass: boxes grouped by their own tile size, each
// class launched with the LDS of its longest padded z, so the short-z boxes
// of an uneven decomposition keep 8-pencil tiles, two per compute unit, next
// to 4-pencil tiles of the long ones.  None when every box takes one size.
inline void build_z_classes(HostTables& h) {
  h.zcls.clear();
  h.itemsZC.clear();
  std::vector<int> pb(h.nsub);
  int used = 0;  // bit PB / 2 per tile size
  for (int s = 0; s < h.nsub; ++s) {
    pb[s] = z_pencils_for(h, h.box[s].P[2]);
    if (!pb[s]) return;
    used |= 1 << (pb[s] / 2);
  }
  if ((used & (used - 1)) == 0) return;  // one size: one launch
  for (int PB : {10, 8, 6, 4}) {
    if (!(used & (1 << (PB / 2)))) continue;
    ZClass k{};
    k.PB = PB;
    k.U = (int32_t)h.itemsZC.size();
    int32_t acc = 0;
    h.itemsZC.push_back(0);
    for (int s = 0; s < h.nsub; ++s) {
      const BoxD& b = h.box[s];
      if (pb[s] == PB) {
        acc += (int32_t)(((int64_t)b.P[1] * b.H + PB - 1) / PB);
        k.lds = std::max<int32_t>(k.lds, (int32_t)z_tile_lds(h, b.P[2], PB));
      }
      h.itemsZC.push_back(acc);
    }
    k.nU = acc;
    h.zcls.push_back(k);
  }
}

// The largest dynamic LDS any z launch of the plan may ask for.
inline int32_t z_lds_max(const HostTables& h) {
  int32_t m = h.ldsU;
  for (const ZClass& k : h.zcls) m = std::max(m, k.lds);
  return m;
}

// Re-derives every FFT schedule with radices up to maxr (twiddle tables
// depend on the length only and are kept).  False if a length has no
// schedule of at most kMaxStages stages.
inline bool set_max_radix(HostTables& h, int maxr, int maxrz) {
  std::vector<FftPlanD> plans = h.plans;
  for (size_t i = 0; i < plans.size(); ++i) {
    std::vector<int> rad;
    if (!schedule(plans[i].N, rad, h.plan_z[i] ? maxrz : maxr, h.spl)) return false;
    set_stages(plans[i], rad);
  }
  for (FftPlanD& pl : plans) write_plan_twiddles(h, pl);  // the layout follows the schedule
  h.plans = plans;
  h.maxr = maxr;
  h.maxrz = maxrz;
  return true;
}

inline int max_padded_z(const HostTables& h) {
  int m = 0;
  for (const BoxD& b : h.box) m = std::max(m, b.P[2]);
  return m;
}

// Runs of padded positions q of box d (global coordinate lo_d - g_d + q mod N)
// that fall on the interior [lo_s, lo_s + n_s) of box s, as (i0, q0, len) with
// i the interior index of s; consecutive q with consecutive i form one run.
struct Run {
  int32_t i0, q0, len;
};
inline void axis_runs(int64_t lo_s, int64_t n_s, int64_t lo_d, int64_t g_d, int64_t P_d, int64_t N,
                      std::vector<Run>& out) {
  out.clear();
  for (int64_t q = 0; q < P_d; ++q) {
    const int64_t G = ((lo_d - g_d + q) % N + N) % N;
    const int64_t i = ((G - lo_s) % N + N) % N;
    if (i >= n_s) continue;
    if (!out.empty()) {
      Run& r = out.back();
      if (r.q0 + r.len == q && r.i0 + r.len == i) {
        ++r.len;
        continue;
      }
    }
    out.push_back({(int32_t)i, (int32_t)q, 1});
  }
}

// Guard pieces for the fused E,B exchange (every guard cell of every box in
// exactly one piece; the interior of each box itself excluded).
inline void build_push(HostTables& h) {
  const int nsub = h.nsub;
  h.push.clear();
  h.push_off.assign(nsub + 1, 0);
  std::vector<Run> rz, ry, rx;
  for (int s = 0; s < nsub; ++s) {
    const BoxD& a = h.box[s];
    for (int d = 0; d < nsub; ++d) {
      const BoxD& b = h.box[d];
      axis_runs(a.lo[2], a.n[2], b.lo[2], b.g[2], b.P[2], h.N[2], rz);
      if (rz.empty()) continue;
      axis_runs(a.lo[1], a.n[1], b.lo[1], b.g[1], b.P[1], h.N[1], ry);
      if (ry.empty()) continue;
      axis_runs(a.lo[0], a.n[0], b.lo[0], b.g[0], b.P[0], h.N[0], rx);
      if (rx.empty()) continue;
      for (const Run& z : rz)
        for (const Run& y : ry)
          for (const Run& x : rx) {
            const bool own = d == s && z.q0 == b.g[2] && y.q0 == b.g[1] && x.q0 == b.g[0] &&
                             z.i0 == 0 && y.i0 == 0 && x.i0 == 0;
            if (own) continue;  // the interior itself
            h.push.push_back({s, d, z.i0, z.len, z.q0, y.i0, y.len, y.q0, x.i0, x.len, x.q0});
          }
    }
    h.push_off[s + 1] = (int32_t)h.push.size();
  }
  // the pieces as the guard fill reads them
  const int V = 16 / real_size(h.prec);  // elements per 16-byte access
  h.fillp.clear();
  for (const PushBlk& k : h.push) {
    const BoxD& sb = h.box[k.src];
    const BoxD& db = h.box[k.dst];
    FillPiece f{};
    f.sP0 = sb.P[0];
    f.dP0 = db.P[0];
    f.sPl = sb.P[0] * sb.P[1];
    f.dPl = db.P[0] * db.P[1];
    f.ly = k.ly;
    f.lx = k.lx;
    f.so = sb.foff + ((int64_t)(sb.g[2] + k.z0) * sb.P[1] + (sb.g[1] + k.y0)) * sb.P[0] + sb.g[0] + k.x0;
    f.dof = db.foff + ((int64_t)k.qz * db.P[1] + k.qy) * db.P[0] + k.qx;
    f.vec = (k.lx % V == 0 && f.so % V == 0 && f.dof % V == 0 && f.sP0 % V == 0 && f.dP0 % V == 0 &&
             f.sPl % V == 0 && f.dPl % V == 0);
    h.fillp.push_back(f);
  }
  // the same pieces by destination box, as the forward pass pulls them
  h.pullp.clear();
  h.pull_off.assign(h.nsub + 1, 0);
  for (int d = 0; d < h.nsub; ++d) {
    for (size_t i = 0; i < h.push.size(); ++i) {
      const PushBlk& k = h.push[i];
      if (k.dst != d) continue;
      const BoxD& sb = h.box[k.src];
      PullPiece q{};
      q.so = h.fillp[i].so;
      q.sPl = sb.P[0] * sb.P[1];
      q.sP0 = sb.P[0];
      q.qz = k.qz;
      q.lz = k.lz;
      q.qy = k.qy;
      q.ly = k.ly;
      q.qx = k.qx;
      q.lx = k.lx;
      h.pullp.push_back(q);
    }
    h.pull_off[d + 1] = (int32_t)h.pullp.size();
  }
  // work list of the guard fill: one item per z-plane of every piece
  h.itemsG.assign(h.push.size() + 1, 0);
  for (size_t b = 0; b < h.push.size(); ++b) h.itemsG[b + 1] = h.itemsG[b] + h.push[b].lz;
  h.pieceOf.resize(h.itemsG.back());
  for (size_t b = 0; b < h.push.size(); ++b)
    for (int32_t i = h.itemsG[b]; i < h.itemsG[b + 1]; ++i) h.pieceOf[i] = (int32_t)b;
}

// Threads per x/y work-group for planes of `lds` bytes: the fewest (256, 512
// or 1024) that still keep 16 waves on a compute unit, given how many planes
// fit its LDS.
inline int xy_threads_for(int lds) {
  const int per_cu = lds > 0 ? std::max(1, kMaxDynLds / lds) : 1;
  for (int nt : {256, 512})
    if (per_cu * nt / 64 >= 16) return nt;
  return 1024;
}

// Launch classes of the x/y passes: boxes grouped by their group size, each
// class launched with its own LDS (the largest plane among its boxes), so
// small boxes are not held to one group per compute unit by the largest box
// of an uneven decomposition.  None when every box has the same group size or
// the planes take the split passes.
inline void build_xy_classes(HostTables& h) {
  h.xyc.clear();
  h.itemsXYC.clear();
  if (h.split) return;
  const int sizes[kMaxXyClasses] = {256, 512, 1024};
  std::vector<int> cls(h.nsub);
  int used = 0;
  for (int s = 0; s < h.nsub; ++s) {
    const int nt = xy_threads_for(h.boxlds[s]);
    cls[s] = nt == 256 ? 0 : (nt == 512 ? 1 : 2);
    used |= 1 << cls[s];
  }
  if (used == 1 || used == 2 || used == 4) return;  // one class: one launch
  auto prefix = [&](int c, auto count) {
    const int32_t off = (int32_t)h.itemsXYC.size();
    int32_t acc = 0;
    h.itemsXYC.push_back(0);
    for (int s = 0; s < h.nsub; ++s) {
      if (cls[s] == c) acc += (int32_t)count(h.box[s]);
      h.itemsXYC.push_back(acc);
    }
    return std::make_pair(off, acc);
  };
  for (int c = 0; c < kMaxXyClasses; ++c) {
    if (!(used & (1 << c))) continue;
    XyClass k{};
    k.nt = sizes[c];
    for (int s = 0; s < h.nsub; ++s)
      if (cls[s] == c) k.lds = std::max(k.lds, h.boxlds[s]);
    std::tie(k.F, k.nF) = prefix(c, [](const BoxD& b) { return (int64_t)b.P[2] * 9; });
    std::tie(k.P, k.nP) = prefix(c, [](const BoxD& b) { return (int64_t)b.P[2]; });
    std::tie(k.I, k.nI) = prefix(c, [](const BoxD& b) { return (int64_t)b.n[2] * 6; });
    std::tie(k.N, k.nN) = prefix(c, [](const BoxD& b) { return (int64_t)b.n[2]; });
    h.xyc.push_back(k);
  }
}

// Pencils per work-group of the register z pass for padded z length N (0: no schedule).
inline int zreg_pencils_of(int N) {
#define PSATD_ZREG_P(N_, L_, W_, MINW_) \
  if (N == N_) return zreg_pencils(L_, W_);
  PSATD_ZREG_SHAPES(PSATD_ZREG_P)
#undef PSATD_ZREG_P
  return 0;
}

// Groups of the register z pass: every distinct padded z length must have a
// schedule (else the LDS-staged z pass runs for all boxes).
inline void build_zreg(HostTables& h) {
  h.zreg = false;
  h.zgroups.clear();
  h.itemsZR.clear();
  if (h.prec != PSATD_F32_VALU) return;
  std::vector<int> lens;
  for (const BoxD& b : h.box)
    if (std::find(lens.begin(), lens.end(), b.P[2]) == lens.end()) lens.push_back(b.P[2]);
  if ((int)lens.size() > kMaxZGroups) return;
  for (int N : lens)
    if (!zreg_pencils_of(N)) return;
  for (const BoxD& b : h.box)  // the kernel addresses a box's 9 fields with 32-bit byte offsets
    if (9 * b.svol * 8 >= ((int64_t)1 << 31)) return;
  for (int N : lens) {
    const int P = zreg_pencils_of(N);
    ZGroup g{N, (int32_t)h.itemsZR.size(), 0, 0};
    int32_t acc = 0;
    h.itemsZR.push_back(0);
    for (const BoxD& b : h.box) {
      if (b.P[2] == N) acc += (int32_t)(((int64_t)b.P[1] * b.H + P - 1) / P);
      h.itemsZR.push_back(acc);
    }
    g.n = acc;
    h.zgroups.push_back(g);
  }
  h.zreg = true;
}

// Does the circular interval [a, a+len) (len < N) meet [lo, lo+n) on Z_N?
inline bool circ_meets(int64_t a, int64_t len, int64_t lo, int64_t n, int64_t N) {
  if (len >= N) return true;
  for (int k = -2; k <= 2; ++k) {
    const int64_t s = a + k * N, e = s + len;
    if (s < lo + n && lo < e) return true;
  }
  return false;
}

inline psatd_status build_host(HostTables& h, std::string& err, const int64_t grid_n[3],
                        const double grid_d[3], int32_t nsub, const int64_t* lo, const int64_t* n,
                        const int32_t* guard, int32_t order_p, double dt, double c,
                        int32_t precision, int32_t jmode) {
  auto bad = [&](psatd_status st, const std::string& m) {
    err = m;
    return st;
  };
  if (!grid_n || !grid_d || !lo || !n || !guard) return bad(PSATD_E_INVALID, "null pointer argument");
  if (nsub < 1) return bad(PSATD_E_INVALID, "nsub must be >= 1");
  for (int u = 0; u < 3; ++u) {
    if (grid_n[u] < 1 || grid_n[u] > (1 << 24)) return bad(PSATD_E_INVALID, "grid_n out of range");
    if (!(grid_d[u] > 0.0) || !std::isfinite(grid_d[u])) return bad(PSATD_E_INVALID, "grid_d must be finite and > 0");
  }
  if (order_p < 0 || (order_p % 2) != 0 || order_p == 1)
    return bad(PSATD_E_INVALID, "order_p must be 0 (infinite) or even >= 2");
  if (!(dt != 0.0) || !std::isfinite(dt)) return bad(PSATD_E_INVALID, "dt must be finite and nonzero");
  if (!(c > 0.0) || !std::isfinite(c)) return bad(PSATD_E_INVALID, "c must be finite and > 0");
  if (precision < PSATD_F64 || precision > PSATD_F32_BF16X6) return bad(PSATD_E_INVALID, "unknown precision");
  if (jmode != PSATD_J_REPLICATED && jmode != PSATD_J_DEPOSITED) return bad(PSATD_E_INVALID, "unknown jmode");

  for (int u = 0; u < 3; ++u) {
    h.N[u] = grid_n[u];
    h.d[u] = grid_d[u];
  }
  h.nsub = nsub;
  h.p = order_p;
  h.dt = dt;
  h.c = c;
  h.prec = precision;
  h.jmode = jmode;
  h.spl = precision == PSATD_F32_BF16X3 ? 2 : (precision == PSATD_F32_BF16X6 ? 3 : 0);

  // boxes inside the grid, guards >= 0
  for (int s = 0; s < nsub; ++s)
    for (int u = 0; u < 3; ++u) {
      const int64_t l = lo[3 * s + u], m = n[3 * s + u];
      if (m < 1 || l < 0 || l + m > grid_n[u]) return bad(PSATD_E_INVALID, "box " + std::to_string(s) + " outside the grid");
      if (guard[3 * s + u] < 0) return bad(PSATD_E_INVALID, "negative guard width");
      if (m + 2 * (int64_t)guard[3 * s + u] > (1 << 20)) return bad(PSATD_E_INVALID, "padded length too large");
    }
  // refined cuts and owner table: exact tiling
  for (int u = 0; u < 3; ++u) {
    std::vector<int64_t> pts{0, grid_n[u]};
    for (int s = 0; s < nsub; ++s) {
      pts.push_back(lo[3 * s + u]);
      pts.push_back(lo[3 * s + u] + n[3 * s + u]);
    }
    std::sort(pts.begin(), pts.end());
    pts.erase(std::unique(pts.begin(), pts.end()), pts.end());
    h.ncut[u] = (int32_t)pts.size() - 1;
    h.cut[u].assign(grid_n[u], 0);
    for (int i = 0; i < h.ncut[u]; ++i)
      for (int64_t x = pts[i]; x < pts[i + 1]; ++x) h.cut[u][x] = i;
  }
  const int64_t ncell = (int64_t)h.ncut[0] * h.ncut[1] * h.ncut[2];
  if (ncell > (int64_t)1 << 26) return bad(PSATD_E_UNSUPPORTED, "decomposition too fine");
  h.owner.assign(ncell, -1);
  for (int s = 0; s < nsub; ++s) {
    int c0[3], c1[3];
    for (int u = 0; u < 3; ++u) {
      c0[u] = h.cut[u][lo[3 * s + u]];
      c1[u] = h.cut[u][lo[3 * s + u] + n[3 * s + u] - 1] + 1;
    }
    for (int cz = c0[2]; cz < c1[2]; ++cz)
      for (int cy = c0[1]; cy < c1[1]; ++cy)
        for (int cx = c0[0]; cx < c1[0]; ++cx) {
          int32_t& o = h.owner[((int64_t)cz * h.ncut[1] + cy) * h.ncut[0] + cx];
          if (o != -1) return bad(PSATD_E_INVALID, "boxes " + std::to_string(o) + " and " + std::to_string(s) + " overlap");
          o = s;
        }
  }
  for (int32_t o : h.owner)
    if (o < 0) return bad(PSATD_E_INVALID, "boxes leave part of the grid uncovered");

  // per box: padded extents, FFT plans, tables, offsets
  const bool f64 = is_f64(precision);
  const int csz = (int)(2 * real_size(precision));
  std::vector<std::pair<int, int>> twcache;
  h.box.resize(nsub);
  int64_t foff = 0, soff = 0;
  int maxPz = 0;
  for (int s = 0; s < nsub; ++s) {
    BoxD& b = h.box[s];
    std::memset(&b, 0, sizeof(b));
    for (int u = 0; u < 3; ++u) {
      b.lo[u] = (int32_t)lo[3 * s + u];
      b.n[u] = (int32_t)n[3 * s + u];
      b.g[u] = guard[3 * s + u];
      b.P[u] = b.n[u] + 2 * b.g[u];
      if (!small_primes_only(b.P[u]))
        return bad(PSATD_E_UNSUPPORTED, "padded length " + std::to_string(b.P[u]) + " has a prime factor > 11");
    }
    if (b.P[0] % 2) return bad(PSATD_E_UNSUPPORTED, "padded x length must be even");
    b.H = b.P[0] / 2 + 1;
    b.ld = (b.H % 2) ? b.H : b.H + 1;
    b.planx = add_plan(h, b.P[0] / 2, false);
    b.plany = add_plan(h, b.P[1], false);
    b.planz = add_plan(h, b.P[2], true);
    if (b.planx < 0 || b.plany < 0 || b.planz < 0)
      return bad(PSATD_E_UNSUPPORTED, "no radix schedule of <= 4 stages for a padded length");
    b.twr = add_twiddle(h, b.P[0], twcache);
    b.kx = add_kentry(h, b.P[0], grid_d[0]);
    b.ky = add_kentry(h, b.P[1], grid_d[1]);
    b.kz = add_kentry(h, b.P[2], grid_d[2]);
    // The box starts where its first interior x cell begins a 128-byte line
    // (to within the 16 bytes that keep vector accesses aligned): then the
    // interior rows, and the guard rows pulled from them, are whole lines
    // whenever the row pitch is.  The gap costs under 128 bytes per box.
    {
      const int64_t line = 128 / (int64_t)real_size(precision), vec = 16 / (int64_t)real_size(precision);
      const int64_t t = (line - b.g[0] % line) % line;
      const int64_t want = (t + vec - 1) / vec * vec % line;
      foff += ((want - foff) % line + line) % line;
    }
    b.foff = foff;
    b.soff = soff;
    b.svol = (int64_t)b.H * b.P[1] * b.P[2];
    foff += (int64_t)b.P[0] * b.P[1] * b.P[2];
    soff += (int64_t)b.H * b.P[1] * b.P[2];
    // plane + twiddles of the x plan, the y plan and W_Px + position tables
    h.boxlds.push_back((b.P[1] * b.ld + b.P[0] / 2 + b.P[1] + b.P[0]) * csz + (b.P[0] / 2 + b.P[1]) * 4);
    h.ldsF = std::max<int>(h.ldsF, h.boxlds.back());
    h.ldsI = h.ldsF;
    maxPz = std::max(maxPz, b.P[2]);
  }
  if (h.twr.size() > (size_t)INT32_MAX / 2)
    return bad(PSATD_E_UNSUPPORTED, "tables too large");
  h.field_elems = foff;
  h.slab = soff;
  // planes that do not fit the LDS take the split x-row / y-column passes
  h.split = h.ldsF > kMaxDynLds;
  for (const BoxD& b : h.box) {
    h.ldsX = std::max<int>(h.ldsX, (kRB * b.ld + b.P[0] / 2 + b.P[0]) * csz + (b.P[0] / 2) * 4);
    h.ldsY = std::max<int>(h.ldsY, (b.P[1] * kCB + b.P[1]) * csz + b.P[1] * 4);
  }
  if (h.ldsX > kMaxDynLds || h.ldsY > kMaxDynLds)
    return bad(PSATD_E_UNSUPPORTED, "padded lengths too large for the split x/y passes");
  // z-update tile: PB consecutive (ky, kx) pencils (128-byte rows when possible)
  {
    // Two FP32 tiles per CU, so one tile's loads overlap the other's
    // transforms, each as wide as two still fit (z_pencils_for: 10 pencils for
    // 96-long z, 6 for 176; one 8-pencil tile of 176 would fill a CU alone, and
    // 4 pencils took configuration 5's z pass 35.5 -> 30.4 ms, 6 to 26.5 ms).
    // FP64 keeps 8: its 4-pencil tiles measured slower on 96^3 boxes.
    int PB = 8;
    while (PB > 4 && !z_tile_fits(h, maxPz, PB)) PB /= 2;
    if (!f64 && PB == 8) {
      const int own = z_pencils_for(h, maxPz);
      if (own) PB = own;
    }
    if (!z_tile_fits(h, maxPz, PB))
      return bad(PSATD_E_UNSUPPORTED, "padded z length too large for the z-update kernel");
    h.PB = PB;
  }

  // neighbours: boxes whose padded region meets the interior of s (for the
  // deposited-current sum), ascending
  h.nbr_off.assign(nsub + 1, 0);
  h.nbr.clear();
  if (jmode == PSATD_J_DEPOSITED) {
    for (int s = 0; s < nsub; ++s) {
      for (int s2 = 0; s2 < nsub; ++s2) {
        bool meets = true;
        for (int u = 0; u < 3 && meets; ++u)
          meets = circ_meets((int64_t)h.box[s2].lo[u] - h.box[s2].g[u], h.box[s2].P[u], h.box[s].lo[u],
                             h.box[s].n[u], grid_n[u]);
        if (meets) h.nbr.push_back(s2);
      }
      h.nbr_off[s + 1] = (int32_t)h.nbr.size();
    }
  }
  // work lists
  auto prefix = [&](std::vector<int32_t>& v, auto count) {
    v.assign(nsub + 1, 0);
    for (int s = 0; s < nsub; ++s) v[s + 1] = v[s] + (int32_t)count(h.box[s]);
  };
  const int PB = h.PB;
  (void)PB;
  prefix(h.itemsF, [](const BoxD& b) { return (int64_t)b.P[2] * 9; });
  set_z_tile(h, PB);
  prefix(h.itemsI, [](const BoxD& b) { return (int64_t)b.n[2] * 6; });
  prefix(h.itemsP, [](const BoxD& b) { return (int64_t)b.P[2]; });
  prefix(h.itemsN, [](const BoxD& b) { return (int64_t)b.n[2]; });
  prefix(h.itemsXF, [](const BoxD& b) { return (int64_t)b.P[2] * 9 * ((b.P[1] + kRB - 1) / kRB); });
  prefix(h.itemsYF, [](const BoxD& b) { return (int64_t)b.P[2] * 9 * ((b.H + kCB - 1) / kCB); });
  prefix(h.itemsYI, [](const BoxD& b) { return (int64_t)b.n[2] * 6 * ((b.H + kCB - 1) / kCB); });
  prefix(h.itemsXI, [](const BoxD& b) { return (int64_t)b.n[2] * 6 * ((b.n[1] + kRB - 1) / kRB); });
  build_push(h);
  build_zreg(h);
  set_batches(h, 0);
  // launch-shape defaults (measured on 96^3 and 176^3 boxes): x/y groups of
  // the fewest threads that still keep 16 waves on a CU given how many planes
  // fit its LDS (96^3 FP32: four 40 KB planes x 256 threads; 176^3 FP32: one
  // 127 KB plane x 1024 threads); 512-thread z tiles of 8 pencils; FP64
  // x/y stages of radix <= 8 where a plane fits the LDS (radix 16 measured
  // slower there: 2.41 -> 3.66 ms on 96^3 boxes), radix 16 in the split x/y
  // passes and the z pass (faster: z pass 2.93 -> 2.59 ms on 96^3 boxes,
  // 176^3 steps 221-227 -> 215 ms)
  h.ntu = 512;
  h.ntxy = xy_threads_for(h.ldsF);
  build_xy_classes(h);
  build_z_classes(h);
  if (f64 && !h.split && !set_max_radix(h, 8, 16)) return bad(PSATD_E_UNSUPPORTED, "no radix-8 schedule");
  return PSATD_OK;
}

}  // namespace psatd
