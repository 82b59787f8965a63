// Host-only self-check of the planner (plan_host.hpp), built with the address
// and undefined-behaviour sanitizers on the host side by test_plan_sanitized.py.
//
// For every decomposition of a list (uniform, uneven, guards wider than the
// neighbouring interiors, self-wrapping single boxes, odd grids) and every
// precision and current mode it builds the host tables and checks what the
// kernels rely on (Sec. 3.2, Fig. 3):
//   * every guard cell of every padded box lies in exactly one exchange
//     piece, whose source is the owner of that global cell, and no interior
//     cell lies in any piece;
//   * every piece's first and last element lie inside its source and
//     destination boxes' field ranges, and the pull list is the push list
//     regrouped by destination;
//   * the work-list prefixes and spectral offsets add up, and the boxes' field
//     offsets are ordered, aligned and closely packed;
// then it re-tiles the z pass, re-batches and re-schedules the radices.
// Invalid decompositions must be rejected with an error, not undefined
// behaviour.  Prints "plan_check: ok ..." and exits 0, or names the first
// failure and exits 1.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "plan_host.hpp"

using namespace psatd;

namespace {

int g_fail = 0;

#define CHECK(cond, ...)                             \
  do {                                               \
    if (!(cond)) {                                   \
      std::fprintf(stderr, "plan_check: " __VA_ARGS__); \
      std::fprintf(stderr, "\n");                    \
      ++g_fail;                                      \
      return false;                                  \
    }                                                \
  } while (0)

struct Dec {
  std::string name;
  int64_t N[3];
  std::vector<int64_t> lo, n;
  std::vector<int32_t> g;
};

int64_t wrap(int64_t v, int64_t N) { return ((v % N) + N) % N; }

// Cuts along each axis (ascending, first 0, last N) and one guard triple per box.
Dec tiled(const std::string& name, const int64_t N[3], const std::vector<int64_t> cuts[3],
          const std::vector<int32_t>& guards_xyz) {
  Dec d;
  d.name = name;
  for (int u = 0; u < 3; ++u) d.N[u] = N[u];
  size_t b = 0;
  for (size_t k = 0; k + 1 < cuts[2].size(); ++k)
    for (size_t j = 0; j + 1 < cuts[1].size(); ++j)
      for (size_t i = 0; i + 1 < cuts[0].size(); ++i, ++b) {
        d.lo.insert(d.lo.end(), {cuts[0][i], cuts[1][j], cuts[2][k]});
        d.n.insert(d.n.end(), {cuts[0][i + 1] - cuts[0][i], cuts[1][j + 1] - cuts[1][j], cuts[2][k + 1] - cuts[2][k]});
        const size_t gi = 3 * (b % (guards_xyz.size() / 3));
        d.g.insert(d.g.end(), {guards_xyz[gi], guards_xyz[gi + 1], guards_xyz[gi + 2]});
      }
  return d;
}

Dec uniform(const std::string& name, int64_t N0, int64_t N1, int64_t N2, int b0, int b1, int b2, int32_t gw) {
  const int64_t N[3] = {N0, N1, N2};
  const int bb[3] = {b0, b1, b2};
  std::vector<int64_t> cuts[3];
  for (int u = 0; u < 3; ++u)
    for (int i = 0; i <= bb[u]; ++i) cuts[u].push_back(N[u] * i / bb[u]);
  return tiled(name, N, cuts, {gw, gw, gw});
}

bool t_plan_z_sized(const HostTables& h) { return h.plan_z.size() == h.plans.size(); }

bool check_tables(const Dec& d, const HostTables& h, bool pieces = true) {
  const int nsub = h.nsub;
  // owners of every global cell (brute force)
  auto owner_of = [&](const int64_t G[3]) {
    for (int s = 0; s < nsub; ++s) {
      bool in = true;
      for (int u = 0; u < 3 && in; ++u) in = G[u] >= d.lo[3 * s + u] && G[u] < d.lo[3 * s + u] + d.n[3 * s + u];
      if (in) return s;
    }
    return -1;
  };
  int64_t foff = 0, soff = 0;
  const int64_t line = 128 / (int64_t)real_size(h.prec), vec = 16 / (int64_t)real_size(h.prec);
  for (int s = 0; s < nsub; ++s) {
    const BoxD& b = h.box[s];
    // boxes in order, no overlap, a gap of less than one line, 16-byte
    // aligned, the first interior x cell within 16 bytes of a line start
    CHECK(b.foff >= foff && b.foff - foff < line && b.foff % vec == 0 && (b.foff + b.g[0]) % line < vec &&
              b.soff == soff,
          "%s: box %d offsets", d.name.c_str(), s);
    foff = b.foff;
    CHECK(b.svol == (int64_t)b.H * b.P[1] * b.P[2], "%s: box %d svol", d.name.c_str(), s);
    foff += (int64_t)b.P[0] * b.P[1] * b.P[2];
    soff += b.svol;
  }
  CHECK(h.field_elems == foff, "%s: field_elems", d.name.c_str());
  CHECK((int)h.push_off.size() == nsub + 1 && (int)h.pull_off.size() == nsub + 1, "%s: piece offsets", d.name.c_str());
  CHECK(h.pullp.size() == h.push.size() && h.fillp.size() == h.push.size(), "%s: piece counts", d.name.c_str());
  // coverage of every padded box by the pieces that target it
  for (int dst = 0; dst < (pieces ? nsub : 0); ++dst) {
    const BoxD& db = h.box[dst];
    std::vector<int> cover((size_t)db.P[0] * db.P[1] * db.P[2], 0);
    for (size_t i = 0; i < h.push.size(); ++i) {
      const PushBlk& k = h.push[i];
      if (k.dst != dst) continue;
      const BoxD& sb = h.box[k.src];
      CHECK(k.lz > 0 && k.ly > 0 && k.lx > 0, "%s: empty piece %zu", d.name.c_str(), i);
      CHECK(k.qz >= 0 && k.qz + k.lz <= db.P[2] && k.qy >= 0 && k.qy + k.ly <= db.P[1] && k.qx >= 0 &&
                k.qx + k.lx <= db.P[0],
            "%s: piece %zu outside its destination", d.name.c_str(), i);
      CHECK(k.z0 >= 0 && k.z0 + k.lz <= sb.n[2] && k.y0 >= 0 && k.y0 + k.ly <= sb.n[1] && k.x0 >= 0 &&
                k.x0 + k.lx <= sb.n[0],
            "%s: piece %zu outside its source interior", d.name.c_str(), i);
      for (int z = 0; z < k.lz; ++z)
        for (int y = 0; y < k.ly; ++y)
          for (int x = 0; x < k.lx; ++x) {
            const int q[3] = {k.qx + x, k.qy + y, k.qz + z};
            const int64_t G[3] = {wrap(db.lo[0] - db.g[0] + q[0], d.N[0]), wrap(db.lo[1] - db.g[1] + q[1], d.N[1]),
                                  wrap(db.lo[2] - db.g[2] + q[2], d.N[2])};
            const int64_t S[3] = {sb.lo[0] + k.x0 + x, sb.lo[1] + k.y0 + y, sb.lo[2] + k.z0 + z};
            CHECK(S[0] == G[0] && S[1] == G[1] && S[2] == G[2], "%s: piece %zu copies the wrong cell", d.name.c_str(), i);
            CHECK(owner_of(G) == k.src, "%s: piece %zu source is not the owner", d.name.c_str(), i);
            ++cover[((size_t)q[2] * db.P[1] + q[1]) * db.P[0] + q[0]];
          }
      // first and last element of the piece in both field ranges
      const FillPiece& f = h.fillp[i];
      const int64_t slast = f.so + (int64_t)(k.lz - 1) * f.sPl + (int64_t)(k.ly - 1) * f.sP0 + k.lx - 1;
      const int64_t dlast = f.dof + (int64_t)(k.lz - 1) * f.dPl + (int64_t)(k.ly - 1) * f.dP0 + k.lx - 1;
      const int64_t svol = (int64_t)sb.P[0] * sb.P[1] * sb.P[2], dvol = (int64_t)db.P[0] * db.P[1] * db.P[2];
      CHECK(f.so >= sb.foff && slast < sb.foff + svol, "%s: piece %zu source range", d.name.c_str(), i);
      CHECK(f.dof >= db.foff && dlast < db.foff + dvol, "%s: piece %zu destination range", d.name.c_str(), i);
    }
    for (int z = 0; z < db.P[2]; ++z)
      for (int y = 0; y < db.P[1]; ++y)
        for (int x = 0; x < db.P[0]; ++x) {
          const bool interior = z >= db.g[2] && z < db.g[2] + db.n[2] && y >= db.g[1] && y < db.g[1] + db.n[1] &&
                                x >= db.g[0] && x < db.g[0] + db.n[0];
          const int c = cover[((size_t)z * db.P[1] + y) * db.P[0] + x];
          CHECK(c == (interior ? 0 : 1), "%s: box %d cell (%d,%d,%d) covered %d times", d.name.c_str(), dst, x, y,
                z, c);
        }
    // the pull list of dst is its push pieces, in push order
    size_t j = h.pull_off[dst];
    for (size_t i = 0; i < h.push.size(); ++i) {
      if (h.push[i].dst != dst) continue;
      CHECK(j < (size_t)h.pull_off[dst + 1] && h.pullp[j].so == h.fillp[i].so && h.pullp[j].qz == h.push[i].qz &&
                h.pullp[j].lx == h.push[i].lx,
            "%s: pull list of box %d", d.name.c_str(), dst);
      ++j;
    }
    CHECK(j == (size_t)h.pull_off[dst + 1], "%s: pull count of box %d", d.name.c_str(), dst);
  }
  // work lists
  int64_t f = 0, in = 0, gz = 0;
  for (const BoxD& b : h.box) {
    f += (int64_t)b.P[2] * 9;
    in += (int64_t)b.n[2] * 6;
  }
  for (const PushBlk& k : h.push) gz += k.lz;
  CHECK(h.itemsF.back() == f && h.itemsI.back() == in, "%s: pass work lists", d.name.c_str());
  CHECK(h.itemsG.back() == gz && (int64_t)h.pieceOf.size() == gz, "%s: fill work list", d.name.c_str());
  for (int s = 0; s < nsub; ++s)
    CHECK(h.itemsU[s + 1] - h.itemsU[s] == (h.box[s].P[1] * h.box[s].H + h.PB - 1) / h.PB,
          "%s: z work list of box %d", d.name.c_str(), s);
  // x/y launch classes: every box in exactly one, with its whole work, within the class's LDS
  if (!h.xyc.empty()) {
    CHECK(h.xyc.size() >= 2 && h.xyc.size() <= (size_t)kMaxXyClasses, "%s: class count", d.name.c_str());
    for (int s = 0; s < nsub; ++s) {
      int in = 0;
      for (const XyClass& k : h.xyc) {
        const int32_t* F = h.itemsXYC.data() + k.F;
        const int32_t* I = h.itemsXYC.data() + k.I;
        const int cf = F[s + 1] - F[s], ci = I[s + 1] - I[s];
        if (!cf && !ci) continue;
        ++in;
        CHECK(cf == 9 * h.box[s].P[2] && ci == 6 * h.box[s].n[2], "%s: class work of box %d", d.name.c_str(), s);
        CHECK(h.boxlds[s] <= k.lds && k.lds <= kMaxDynLds, "%s: class LDS of box %d", d.name.c_str(), s);
        CHECK(k.nt == xy_threads_for(h.boxlds[s]), "%s: class threads of box %d", d.name.c_str(), s);
      }
      CHECK(in == 1, "%s: box %d in %d classes", d.name.c_str(), s, in);
    }
    int64_t tf = 0, ti = 0;
    for (const XyClass& k : h.xyc) {
      tf += k.nF;
      ti += k.nI;
      CHECK(h.itemsXYC[k.F + nsub] == k.nF && h.itemsXYC[k.P + nsub] == k.nP && h.itemsXYC[k.I + nsub] == k.nI &&
                h.itemsXYC[k.N + nsub] == k.nN,
            "%s: class totals", d.name.c_str());
    }
    CHECK(tf == h.itemsF.back() && ti == h.itemsI.back(), "%s: class work lists add up", d.name.c_str());
  }
  // z launch classes: every box in exactly one, with all its tiles, within the class's LDS
  if (!h.zcls.empty()) {
    CHECK(h.zcls.size() >= 2 && h.zcls.size() <= (size_t)kMaxZClasses, "%s: z class count", d.name.c_str());
    for (size_t c = 1; c < h.zcls.size(); ++c)
      CHECK(h.zcls[c].PB < h.zcls[c - 1].PB, "%s: z classes by tile size", d.name.c_str());
    for (int s = 0; s < nsub; ++s) {
      int in = 0;
      for (const ZClass& k : h.zcls) {
        const int32_t* U = h.itemsZC.data() + k.U;
        const int cu = U[s + 1] - U[s];
        if (!cu) continue;
        ++in;
        CHECK(k.PB == z_pencils_for(h, h.box[s].P[2]), "%s: z class of box %d", d.name.c_str(), s);
        CHECK(cu == (h.box[s].P[1] * h.box[s].H + k.PB - 1) / k.PB, "%s: z class work of box %d", d.name.c_str(), s);
        CHECK(z_tile_lds(h, h.box[s].P[2], k.PB) <= k.lds && k.lds <= kMaxDynLds, "%s: z class LDS of box %d",
              d.name.c_str(), s);
      }
      CHECK(in == 1, "%s: box %d in %d z classes", d.name.c_str(), s, in);
    }
    for (const ZClass& k : h.zcls) CHECK(h.itemsZC[k.U + nsub] == k.nU, "%s: z class totals", d.name.c_str());
  }
  return true;
}

int g_classes = 0;   // built plans with several x/y launch classes
int g_zclasses = 0;  // built plans with several z launch classes
int g_zclasses3 = 0; // ... with four (10, 8, 6 and 4 pencils)

int run_case(const Dec& d, int prec, int jmode, int p, bool expect_ok, int& built) {
  HostTables h;
  std::string err;
  const double dd[3] = {1.0, 0.75, 1.25};
  const int nsub = (int)d.lo.size() / 3;
  const psatd_status st = build_host(h, err, d.N, dd, nsub, d.lo.data(), d.n.data(), d.g.data(), p, 0.5, 1.0, prec, jmode);
  if (!expect_ok) {
    if (st == PSATD_OK) {
      std::fprintf(stderr, "plan_check: %s: accepted an invalid decomposition\n", d.name.c_str());
      ++g_fail;
    } else if (err.empty()) {
      std::fprintf(stderr, "plan_check: %s: rejected without a message\n", d.name.c_str());
      ++g_fail;
    }
    return 0;
  }
  if (st == PSATD_E_UNSUPPORTED) return 0;  // e.g. a padded length with a large prime factor
  if (st != PSATD_OK) {
    std::fprintf(stderr, "plan_check: %s: rejected (%s)\n", d.name.c_str(), err.c_str());
    ++g_fail;
    return 0;
  }
  ++built;
  if (!h.xyc.empty()) ++g_classes;
  if (!h.zcls.empty()) ++g_zclasses;
  if (h.zcls.size() == 4) ++g_zclasses3;
  if (!check_tables(d, h)) return 0;
  // the launch-shape knobs that rebuild host tables
  const int maxPz = max_padded_z(h);
  for (int PB : {2, 4, 8, 16})
    if (z_tile_fits(h, maxPz, PB)) {
      set_z_tile(h, PB);
      if (!check_tables(d, h, false)) return 0;
    }
  for (int per : {1, 2, 3, nsub}) set_batches(h, per);
  set_batches(h, 0);
  // each pass's schedules within its own radix limit (11 always allowed); a
  // box's x/y and z lengths have plans of their own kind
  auto radices_ok = [&](const HostTables& t) {
    for (size_t i = 0; i < t.plans.size(); ++i) {
      const int lim = t.plan_z[i] ? t.maxrz : t.maxr;
      int prod = 1;
      for (int st = 0; st < t.plans[i].nstages; ++st) {
        const int R = t.plans[i].radix[st];
        if (R > lim && R != 11) return false;
        prod *= R;
      }
      if (prod != t.plans[i].N) return false;
    }
    for (const BoxD& b : t.box)
      if (t.plan_z[b.planx] || t.plan_z[b.plany] || !t.plan_z[b.planz]) return false;
    return true;
  };
  CHECK(t_plan_z_sized(h) && radices_ok(h), "%s: radix limits", d.name.c_str());
  for (int r : {8, 16})
    for (int rz : {8, 16}) {
      if (h.spl && (r < 16 || rz < 16)) continue;  // matrix-core forms: a radix-16 first stage, refused by the API
      HostTables t = h;
      if (set_max_radix(t, r, rz)) CHECK(radices_ok(t), "%s: radix limits %d/%d", d.name.c_str(), r, rz);
    }
  return 1;
}

}  // namespace

int main() {
  std::vector<Dec> ok, bad;
  ok.push_back(uniform("one box, no guards", 16, 16, 16, 1, 1, 1, 0));
  ok.push_back(uniform("one box wrapping onto itself", 16, 12, 10, 1, 1, 1, 4));
  ok.push_back(uniform("3x3x3, g=4", 48, 48, 48, 3, 3, 3, 4));
  ok.push_back(uniform("3x3x3, g=12", 48, 48, 48, 3, 3, 3, 12));
  ok.push_back(uniform("2x2x2 anisotropic", 32, 24, 20, 2, 2, 2, 2));
  ok.push_back(uniform("4x1x1, g=16", 128, 32, 32, 4, 1, 1, 16));
  {
    const int64_t N[3] = {64, 64, 64};
    std::vector<int64_t> cuts[3] = {{0, 16, 64}, {0, 64}, {0, 64}};
    ok.push_back(tiled("guards wider than the neighbour", N, cuts, {24, 8, 8}));
  }
  {
    const int64_t N[3] = {144, 144, 96};
    std::vector<int64_t> cuts[3] = {{0, 48, 112, 144}, {0, 64, 144}, {0, 48, 96}};
    ok.push_back(tiled("uneven, mixed guards", N, cuts, {8, 16, 8, 16, 8, 16, 16, 8, 16}));
  }
  {
    // planes of very different sizes: several x/y launch classes
    const int64_t N[3] = {192, 64, 48};
    std::vector<int64_t> cuts[3] = {{0, 32, 192}, {0, 64}, {0, 16, 48}};
    ok.push_back(tiled("x/y launch classes", N, cuts, {8, 8, 8, 8, 8, 8}));
  }
  {
    // padded z lengths of 128 and 160: 8- and 6-pencil FP32 z tiles (FP64 8 and 4)
    const int64_t N[3] = {32, 32, 256};
    std::vector<int64_t> cuts[3] = {{0, 32}, {0, 32}, {0, 112, 256}};
    ok.push_back(tiled("z launch classes", N, cuts, {8, 8, 8, 8, 8, 8}));
  }
  {
    // padded z lengths of 80, 112, 176 and 240: 10-, 8-, 6- and 4-pencil FP32 z tiles
    const int64_t N[3] = {32, 32, 544};
    std::vector<int64_t> cuts[3] = {{0, 32}, {0, 32}, {0, 64, 160, 320, 544}};
    ok.push_back(tiled("four z launch classes", N, cuts, {8, 8, 8, 8, 8, 8}));
  }
  {
    const int64_t N[3] = {20, 21, 15};
    std::vector<int64_t> cuts[3] = {{0, 20}, {0, 21}, {0, 15}};
    ok.push_back(tiled("odd grid, one box", N, cuts, {2, 2, 0}));
  }
  {
    // seeded random cuts (linear congruential draws), guards from {2, 4, 6}
    uint64_t r = 12345;
    auto next = [&](int m) {
      r = r * 6364136223846793005ull + 1442695040888963407ull;
      return (int)((r >> 33) % (uint64_t)m);
    };
    for (int t = 0; t < 6; ++t) {
      const int64_t N[3] = {48, 40, 36};
      std::vector<int64_t> cuts[3];
      for (int u = 0; u < 3; ++u) {
        cuts[u] = {0};
        while (cuts[u].back() < N[u]) {
          const int64_t len = std::min<int64_t>(N[u] - cuts[u].back(), 6 + 2 * next(6));
          cuts[u].push_back(cuts[u].back() + len);
        }
      }
      std::vector<int32_t> gs;
      for (int i = 0; i < 3 * 7; ++i) gs.push_back(2 + 2 * next(3));
      ok.push_back(tiled("random uneven " + std::to_string(t), N, cuts, gs));
    }
  }
  // invalid decompositions
  {
    Dec d = uniform("overlap", 32, 32, 32, 2, 1, 1, 2);
    d.lo[3] = 8;  // second box starts inside the first
    bad.push_back(d);
    Dec e = uniform("gap", 32, 32, 32, 2, 1, 1, 2);
    e.n[0] = 8;
    bad.push_back(e);
    Dec f = uniform("outside", 32, 32, 32, 2, 1, 1, 2);
    f.n[3] = 40;
    bad.push_back(f);
    Dec g = uniform("negative guard", 32, 32, 32, 2, 1, 1, 2);
    g.g[1] = -1;
    bad.push_back(g);
    Dec z = uniform("empty box", 32, 32, 32, 2, 1, 1, 2);
    z.n[5] = 0;
    bad.push_back(z);
  }
  int built = 0, passed = 0;
  // (the exchange pieces do not depend on the order; the z tile and the
  // radix schedules depend on the precision)
  const int precs[] = {PSATD_F64, PSATD_F32_VALU, PSATD_F32_BF16X6};
  for (const Dec& d : ok)
    for (int prec : precs)
      for (int jm : {PSATD_J_REPLICATED, PSATD_J_DEPOSITED})
        passed += run_case(d, prec, jm, jm == PSATD_J_REPLICATED ? 16 : 0, true, built);
  for (const Dec& d : bad) run_case(d, PSATD_F32_VALU, PSATD_J_REPLICATED, 16, false, built);
  // scalar argument errors
  {
    const Dec& d = ok[2];
    HostTables h;
    std::string err;
    const double dd[3] = {1, 1, 1};
    const int nsub = (int)d.lo.size() / 3;
    const psatd_status s1 = build_host(h, err, d.N, dd, nsub, d.lo.data(), d.n.data(), d.g.data(), 3, 0.5, 1.0,
                                       PSATD_F32_VALU, PSATD_J_REPLICATED);
    const psatd_status s2 = build_host(h, err, d.N, dd, nsub, d.lo.data(), d.n.data(), d.g.data(), 16, 0.0, 1.0,
                                       PSATD_F32_VALU, PSATD_J_REPLICATED);
    const psatd_status s3 = build_host(h, err, d.N, dd, 0, d.lo.data(), d.n.data(), d.g.data(), 16, 0.5, 1.0,
                                       PSATD_F32_VALU, PSATD_J_REPLICATED);
    const psatd_status s4 = build_host(h, err, d.N, dd, nsub, d.lo.data(), d.n.data(), nullptr, 16, 0.5, 1.0,
                                       PSATD_F32_VALU, PSATD_J_REPLICATED);
    if (s1 == PSATD_OK || s2 == PSATD_OK || s3 == PSATD_OK || s4 == PSATD_OK) {
      std::fprintf(stderr, "plan_check: an invalid scalar argument was accepted\n");
      ++g_fail;
    }
  }
  if (g_fail || built < 30 || passed != built || g_classes == 0 || g_zclasses == 0 || g_zclasses3 == 0) {
    std::fprintf(stderr, "plan_check: FAILED (%d failures, %d built, %d passed)\n", g_fail, built, passed);
    return 1;
  }
  std::printf("plan_check: ok (%d decompositions x forms built and checked, %d with x/y and %d with z launch "
              "classes, %zu invalid rejected)\n", built, g_classes, g_zclasses, bad.size());
  return 0;
}
