// Host side of libpsatd.so: plan construction (Sec. 3.2 decomposition, Sec. 3.1
// operator), validation, device tables, step enqueue, graph capture and the
// C-ABI declared in include/psatd.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <fstream>
#include <map>
#include <mutex>
#include <sstream>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "psatd.h"
#include "plan_host.hpp"
#include "psatd_launch.hpp"

using namespace psatd;

namespace {

thread_local std::string g_last_error = "";

// Spectral workspace of psatd_step_noalloc: a file-scope device array, one
// copy per GPU, alive until the process ends.  In host code `scratch` only
// names the symbol; its device address on each GPU comes from
// hipGetSymbolAddress, resolved once per device at plan creation with that
// device current, and only that address is ever passed to a kernel.
constexpr int64_t kScratchBytes = PSATD_NOALLOC_SCRATCH_BYTES;
__device__ __align__(256) static unsigned char scratch[kScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hipError_t resolve_scratch(int device) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_ptr[device]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch_ptr[device] = ptr;
  return hipSuccess;
}

void* scratch_of(int device) {
  if (device < 0 || device >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch_ptr[device];
}

struct GraphEntry {
  void* ptr[9];
  int32_t nsteps;
  hipGraph_t graph;
  hipGraphExec_t exec;
};

}  // namespace

// ---------------------------------------------------------------- the plan
struct psatd_plan_s {
  HostTables h;
  DevPlan dp;
  hipStream_t stream = nullptr;
  hipStream_t cap_stream = nullptr;
  int device = 0;
  void* blob = nullptr;  // device tables
  int32_t* d_itemsU = nullptr;  // z-update work list (depends on the z tile)
  int32_t tune[PSATD_NTUNE] = {0, 1, 0, 0, 0, 0, 0, 16, 256, 512, 0, 1, 0, 0};
  void* ws = nullptr;
  int64_t ws_bytes = 0;
  bool ws_owned = false;
  std::vector<GraphEntry> graphs;
  std::string err;
};

namespace {

psatd_status fail(psatd_plan_t p, psatd_status st, const std::string& m) {
  if (p) p->err = m; else g_last_error = m;
  return st;
}

#define HIPCHK(plan, call)                                                                    \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail(plan, e_ == hipErrorOutOfMemory ? PSATD_E_NOMEM : PSATD_E_HIP,              \
                  std::string(#call) + ": " + hipGetErrorString(e_));                         \
  } while (0)

// The twiddle tables in the plan's device type (FP64 or FP32 pairs).
std::vector<unsigned char> device_twiddles(const HostTables& h) {
  const size_t n = h.twr.size();
  std::vector<unsigned char> out;
  if (is_f64(h.prec)) {
    std::vector<cx<double>> t(n);
    for (size_t i = 0; i < n; ++i) t[i] = {(double)h.twr[i], (double)h.twi[i]};
    out.assign(reinterpret_cast<const unsigned char*>(t.data()),
               reinterpret_cast<const unsigned char*>(t.data() + n));
  } else {
    std::vector<cx<float>> t(n);
    for (size_t i = 0; i < n; ++i) t[i] = {(float)h.twr[i], (float)h.twi[i]};
    out.assign(reinterpret_cast<const unsigned char*>(t.data()),
               reinterpret_cast<const unsigned char*>(t.data() + n));
  }
  return out;
}

int64_t workspace_need(const psatd_plan_s* p) {
  return 9 * p->h.batch_slab * (int64_t)(2 * real_size(p->h.prec));
}

void drop_graphs(psatd_plan_t p) {
  for (auto& g : p->graphs) {
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
  }
  p->graphs.clear();
}

psatd_status ensure_workspace(psatd_plan_t p) {
  if (p->ws && p->ws_bytes >= workspace_need(p)) return PSATD_OK;
  if (p->ws && !p->ws_owned)
    return fail(p, PSATD_E_INVALID, "caller workspace smaller than psatd_workspace_bytes");
  if (p->ws) {
    HIPCHK(p, hipStreamSynchronize(p->stream));
    HIPCHK(p, hipFree(p->ws));
    p->ws = nullptr;
  }
  const int64_t need = workspace_need(p);
  HIPCHK(p, hipMalloc(&p->ws, (size_t)std::max<int64_t>(need, 256)));
  p->ws_bytes = need;
  p->ws_owned = true;
  return PSATD_OK;
}

bool aligned16(const void* q) { return ((uintptr_t)q & 15u) == 0; }

psatd_status check_fields(psatd_plan_t p, void* const* v, int count, const char* what) {
  if (!v) return fail(p, PSATD_E_INVALID, std::string(what) + ": null array");
  for (int i = 0; i < count; ++i) {
    if (!v[i]) return fail(p, PSATD_E_INVALID, std::string(what) + ": null buffer");
    if (!aligned16(v[i])) return fail(p, PSATD_E_INVALID, std::string(what) + ": buffer not 16-byte aligned");
  }
  return PSATD_OK;
}

// One step: exchange_J, every batch through F -> U -> I, exchange_EB.  If prof
// is given, an event pair brackets every launch, tagged with its phase.
// first: the first step since J was (re)deposited or changed.  J is read-only
// in the step, so its guard exchange (sum and/or fill) is needed only then;
// later steps of a run with J held fixed find it already consistent.
// last: the run's last step.  With the pulled E,B exchange the guard copies
// are refreshed only then (every forward pass of the run reads guard cells
// from their owners), so the state is consistent again on return.
psatd_status enqueue_step(psatd_plan_t p, void* const E[3], void* const B[3], void* const J[3],
                          hipStream_t st, bool first, bool last,
                          std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>>* prof = nullptr,
                          void* ws = nullptr) {
  const DevPlan& d = p->dp;
  if (!ws) ws = p->ws;
  void* eb[6] = {E[0], E[1], E[2], B[0], B[1], B[2]};
  void* in9[9] = {E[0], E[1], E[2], B[0], B[1], B[2], J[0], J[1], J[2]};
  size_t ip = 0;
  auto mark = [&](int phase, bool start) -> psatd_status {
    if (!prof) return PSATD_OK;
    if (start) {
      if (ip >= prof->size()) return fail(p, PSATD_E_STATE, "profiling event pool exhausted");
      (*prof)[ip].first = phase;
      HIPCHK(p, hipEventRecord((*prof)[ip].second.first, st));
    } else {
      HIPCHK(p, hipEventRecord((*prof)[ip].second.second, st));
      ++ip;
    }
    return PSATD_OK;
  };
  psatd_status r;
#define PSATD_MARK(ph, s0) \
  if ((r = mark(ph, s0)) != PSATD_OK) return r
  if (first) {
    PSATD_MARK(kPhaseExchJ, true);
    if (p->h.jmode == PSATD_J_DEPOSITED) HIPCHK(p, launch_sum(d, J, st));
    HIPCHK(p, launch_fill(d, J, 3, st));
    PSATD_MARK(kPhaseExchJ, false);
  }
  for (const Batch& b : p->h.batches) {
    PSATD_MARK(kPhaseFwd, true);
    if (d.split) {
      HIPCHK(p, launch_x_fwd(d, in9, ws, st));
      HIPCHK(p, launch_y(d, -1, ws, st));
    } else {
      HIPCHK(p, launch_fwd(d, b, in9, ws, st));
    }
    PSATD_MARK(kPhaseFwd, false);
    PSATD_MARK(kPhaseUpd, true);
    if (d.zreg && p->h.batches.size() == 1)
      HIPCHK(p, launch_upd_reg(d, ws, st));
    else
      HIPCHK(p, launch_upd(d, b, ws, st));
    PSATD_MARK(kPhaseUpd, false);
    PSATD_MARK(kPhaseInv, true);
    if (d.split) {
      HIPCHK(p, launch_y(d, 1, ws, st));
      HIPCHK(p, launch_x_inv(d, ws, eb, st));
    } else {
      HIPCHK(p, launch_inv(d, b, ws, eb, st));
    }
    PSATD_MARK(kPhaseInv, false);
  }
  PSATD_MARK(kPhaseExchEB, true);
  if (!d.fuse && (!d.pull || last)) HIPCHK(p, launch_fill(d, eb, 6, st));  // fused: written by the inverse pass
  PSATD_MARK(kPhaseExchEB, false);
#undef PSATD_MARK
  return PSATD_OK;
}

// LDS of the heat z pass: PB staged pencils, the z twiddles and z indices.
int32_t heat_lds(const HostTables& h) {
  const int maxPz = max_padded_z(h);
  return (int32_t)((int64_t)maxPz * (h.PB + 1) * (int64_t)(2 * real_size(h.prec)) + (int64_t)maxPz * 4);
}

psatd_status check_step_args(psatd_plan_t p, void* const E[3], void* const B[3], void* const J[3]) {
  if (!p) return fail(nullptr, PSATD_E_INVALID, "null plan");
  psatd_status r;
  if ((r = check_fields(p, E, 3, "E")) != PSATD_OK) return r;
  if ((r = check_fields(p, B, 3, "B")) != PSATD_OK) return r;
  if ((r = check_fields(p, J, 3, "J")) != PSATD_OK) return r;
  return ensure_workspace(p);
}

}  // namespace

extern "C" {

psatd_status psatd_validate(const int64_t grid_n[3], const double grid_d[3], int32_t nsub,
                            const int64_t* lo, const int64_t* n, const int32_t* guard,
                            int32_t order_p, double dt, double c, int32_t precision,
                            int32_t jmode, int64_t* field_elems) {
  try {
    HostTables h;
    std::string err;
    psatd_status st = build_host(h, err, grid_n, grid_d, nsub, lo, n, guard, order_p, dt, c,
                                 precision, jmode);
    if (st != PSATD_OK) return fail(nullptr, st, err);
    if (field_elems) *field_elems = h.field_elems;
    return PSATD_OK;
  } catch (const std::bad_alloc&) {
    return fail(nullptr, PSATD_E_NOMEM, "host allocation failed");
  } catch (...) {
    return fail(nullptr, PSATD_E_INVALID, "unexpected host exception");
  }
}

psatd_status psatd_plan(psatd_plan_t* out, const int64_t grid_n[3], const double grid_d[3],
                        int32_t nsub, const int64_t* lo, const int64_t* n, const int32_t* guard,
                        int32_t order_p, double dt, double c, int32_t precision, int32_t jmode,
                        void* stream) {
  if (!out) return fail(nullptr, PSATD_E_INVALID, "null output pointer");
  *out = nullptr;
  psatd_plan_s* p = nullptr;
  try {
    p = new psatd_plan_s();
  } catch (...) {
    return fail(nullptr, PSATD_E_NOMEM, "host allocation failed");
  }
  psatd_status st;
  try {
    std::string err;
    st = build_host(p->h, err, grid_n, grid_d, nsub, lo, n, guard, order_p, dt, c, precision, jmode);
    if (st != PSATD_OK) {
      delete p;
      return fail(nullptr, st, err);
    }
  } catch (...) {
    delete p;
    return fail(nullptr, PSATD_E_NOMEM, "host allocation failed");
  }
  HostTables& h = p->h;
  p->stream = reinterpret_cast<hipStream_t>(stream);
  auto hipfail = [&](hipError_t e, const char* what) {
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    psatd_destroy(p);
    return fail(nullptr, e == hipErrorOutOfMemory ? PSATD_E_NOMEM : PSATD_E_HIP, m);
  };
  hipError_t e;
  if ((e = hipGetDevice(&p->device)) != hipSuccess) return hipfail(e, "hipGetDevice");
  if ((e = resolve_scratch(p->device)) != hipSuccess) return hipfail(e, "hipGetSymbolAddress(scratch)");
  if ((e = hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking)) != hipSuccess)
    return hipfail(e, "hipStreamCreateWithFlags");

  // one device blob for every table
  const bool f64 = is_f64(h.prec);
  const size_t cs = 2 * real_size(h.prec);
  std::vector<std::pair<size_t, size_t>> parts;  // (offset, bytes)
  size_t total = 0;
  auto reserve = [&](size_t bytes) {
    const size_t off = total;
    total += (bytes + 255) & ~(size_t)255;
    return off;
  };
  const size_t o_box = reserve(h.box.size() * sizeof(BoxD));
  const size_t o_plan = reserve(h.plans.size() * sizeof(FftPlanD));
  const size_t o_tw = reserve(h.twr.size() * cs);
  const size_t o_kmod = reserve((size_t)h.kmod_len * 8);
  const size_t o_kent = reserve(h.kent.size() * sizeof(KEntry));
  const size_t o_nbo = reserve(h.nbr_off.size() * 4);
  const size_t o_nbr = reserve(std::max<size_t>(h.nbr.size(), 1) * 4);
  const size_t o_iF = reserve(h.itemsF.size() * 4);
  const size_t o_iI = reserve(h.itemsI.size() * 4);
  const size_t o_iP = reserve(h.itemsP.size() * 4);
  const size_t o_iN = reserve(h.itemsN.size() * 4);
  const size_t o_iXF = reserve(h.itemsXF.size() * 4);
  const size_t o_iYF = reserve(h.itemsYF.size() * 4);
  const size_t o_iYI = reserve(h.itemsYI.size() * 4);
  const size_t o_iXI = reserve(h.itemsXI.size() * 4);
  const size_t o_push = reserve(std::max<size_t>(h.push.size(), 1) * sizeof(PushBlk));
  const size_t o_pof = reserve(h.push_off.size() * 4);
  const size_t o_iG = reserve(h.itemsG.size() * 4);
  const size_t o_fp = reserve(std::max<size_t>(h.fillp.size(), 1) * sizeof(FillPiece));
  const size_t o_pOf = reserve(std::max<size_t>(h.pieceOf.size(), 1) * 4);
  const size_t o_iZR = reserve(std::max<size_t>(h.itemsZR.size(), 1) * 4);
  const size_t o_pull = reserve(std::max<size_t>(h.pullp.size(), 1) * sizeof(PullPiece));
  const size_t o_poff = reserve(h.pull_off.size() * 4);
  const size_t o_xyc = reserve(std::max<size_t>(h.itemsXYC.size(), 1) * 4);
  const size_t o_zc = reserve(std::max<size_t>(h.itemsZC.size(), 1) * 4);
  std::vector<unsigned char> hb(total, 0);
  auto put = [&](size_t off, const void* src, size_t bytes) {
    if (bytes) std::memcpy(hb.data() + off, src, bytes);
  };
  put(o_box, h.box.data(), h.box.size() * sizeof(BoxD));
  put(o_plan, h.plans.data(), h.plans.size() * sizeof(FftPlanD));
  {
    const std::vector<unsigned char> t = device_twiddles(h);
    put(o_tw, t.data(), t.size());
  }
  put(o_kent, h.kent.data(), h.kent.size() * sizeof(KEntry));
  put(o_nbo, h.nbr_off.data(), h.nbr_off.size() * 4);
  put(o_nbr, h.nbr.data(), h.nbr.size() * 4);
  put(o_iF, h.itemsF.data(), h.itemsF.size() * 4);
  put(o_iI, h.itemsI.data(), h.itemsI.size() * 4);
  put(o_iP, h.itemsP.data(), h.itemsP.size() * 4);
  put(o_iN, h.itemsN.data(), h.itemsN.size() * 4);
  put(o_iXF, h.itemsXF.data(), h.itemsXF.size() * 4);
  put(o_iYF, h.itemsYF.data(), h.itemsYF.size() * 4);
  put(o_iYI, h.itemsYI.data(), h.itemsYI.size() * 4);
  put(o_iXI, h.itemsXI.data(), h.itemsXI.size() * 4);
  put(o_push, h.push.data(), h.push.size() * sizeof(PushBlk));
  put(o_pof, h.push_off.data(), h.push_off.size() * 4);
  put(o_iG, h.itemsG.data(), h.itemsG.size() * 4);
  put(o_fp, h.fillp.data(), h.fillp.size() * sizeof(FillPiece));
  put(o_pOf, h.pieceOf.data(), h.pieceOf.size() * 4);
  put(o_iZR, h.itemsZR.data(), h.itemsZR.size() * 4);
  put(o_pull, h.pullp.data(), h.pullp.size() * sizeof(PullPiece));
  put(o_poff, h.pull_off.data(), h.pull_off.size() * 4);
  put(o_xyc, h.itemsXYC.data(), h.itemsXYC.size() * 4);
  put(o_zc, h.itemsZC.data(), h.itemsZC.size() * 4);
  if ((e = hipMalloc(&p->blob, total)) != hipSuccess) return hipfail(e, "hipMalloc(tables)");
  if ((e = hipMemcpy(p->blob, hb.data(), total, hipMemcpyHostToDevice)) != hipSuccess)
    return hipfail(e, "hipMemcpy(tables)");
  if ((e = hipMalloc(&p->d_itemsU, h.itemsU.size() * 4)) != hipSuccess) return hipfail(e, "hipMalloc(work list)");
  if ((e = hipMemcpy(p->d_itemsU, h.itemsU.data(), h.itemsU.size() * 4, hipMemcpyHostToDevice)) != hipSuccess)
    return hipfail(e, "hipMemcpy(work list)");
  // boxes of several tile sizes: one z launch per class (z_pencils 0)
  p->tune[PSATD_TUNE_Z_PENCILS] = h.zcls.empty() ? h.PB : 0;
  p->tune[PSATD_TUNE_MAX_RADIX] = h.maxr;
  p->tune[PSATD_TUNE_MAX_RADIX_Z] = h.maxrz;
  // boxes of several plane sizes: one x/y launch per class (xy_threads 0)
  p->tune[PSATD_TUNE_XY_THREADS] = h.xyc.size() > 1 ? 0 : h.ntxy;
  p->tune[PSATD_TUNE_Z_THREADS] = h.ntu;
  p->tune[PSATD_TUNE_SPLIT_XY] = h.split ? 1 : 0;
  unsigned char* B = reinterpret_cast<unsigned char*>(p->blob);
  // (a1) modified wavenumbers, FP64, on the device
  if ((e = launch_modk(reinterpret_cast<const KEntry*>(B + o_kent), (int)h.kent.size(), h.kmax_len, h.p,
                       reinterpret_cast<double*>(B + o_kmod), p->cap_stream)) != hipSuccess)
    return hipfail(e, "modified-wavenumber kernel");
  if ((e = hipStreamSynchronize(p->cap_stream)) != hipSuccess) return hipfail(e, "modified-wavenumber kernel");
  if ((e = prepare_kernels(f64, h.spl, h.ldsF, h.ldsI, z_lds_max(h), h.ldsX, h.ldsY)) != hipSuccess)
    return hipfail(e, "hipFuncSetAttribute");

  DevPlan& d = p->dp;
  std::memset(&d, 0, sizeof(d));
  d.f64 = f64;
  d.nsub = h.nsub;
  for (int u = 0; u < 3; ++u) d.N[u] = (int32_t)h.N[u];
  d.box = reinterpret_cast<const BoxD*>(B + o_box);
  d.plans = reinterpret_cast<const FftPlanD*>(B + o_plan);
  d.tw = B + o_tw;
  d.kmod = reinterpret_cast<const double*>(B + o_kmod);
  d.nbr_off = reinterpret_cast<const int32_t*>(B + o_nbo);
  d.nbr = reinterpret_cast<const int32_t*>(B + o_nbr);
  d.itemsF = reinterpret_cast<const int32_t*>(B + o_iF);
  d.itemsU = p->d_itemsU;
  d.itemsI = reinterpret_cast<const int32_t*>(B + o_iI);
  d.itemsP = reinterpret_cast<const int32_t*>(B + o_iP);
  d.itemsN = reinterpret_cast<const int32_t*>(B + o_iN);
  d.itemsXF = reinterpret_cast<const int32_t*>(B + o_iXF);
  d.itemsYF = reinterpret_cast<const int32_t*>(B + o_iYF);
  d.itemsYI = reinterpret_cast<const int32_t*>(B + o_iYI);
  d.itemsXI = reinterpret_cast<const int32_t*>(B + o_iXI);
  d.nXF = h.itemsXF.back();
  d.nYF = h.itemsYF.back();
  d.nYI = h.itemsYI.back();
  d.nXI = h.itemsXI.back();
  d.ldsX = h.ldsX;
  d.ldsY = h.ldsY;
  d.split = h.split ? 1 : 0;
  d.push = reinterpret_cast<const PushBlk*>(B + o_push);
  d.push_off = reinterpret_cast<const int32_t*>(B + o_pof);
  d.itemsG = reinterpret_cast<const int32_t*>(B + o_iG);
  d.fillp = reinterpret_cast<const FillPiece*>(B + o_fp);
  d.pieceOf = reinterpret_cast<const int32_t*>(B + o_pOf);
  d.npiece = (int32_t)h.push.size();
  d.nG = h.itemsG.back();
  d.itemsZR = reinterpret_cast<const int32_t*>(B + o_iZR);
  d.nzg = (int32_t)h.zgroups.size();
  for (int i = 0; i < d.nzg; ++i) d.zg[i] = h.zgroups[i];
  d.zreg = 0;  // opt-in: measured slower than the LDS-staged z pass on 96^3 and 176^3 boxes
  d.pullp = reinterpret_cast<const PullPiece*>(B + o_pull);
  d.pull_off = reinterpret_cast<const int32_t*>(B + o_poff);

  p->tune[PSATD_TUNE_Z_REG] = d.zreg;
  d.fuse = (h.fuse_eb && h.batches.size() == 1) ? 1 : 0;
  d.spl = h.spl;
  p->tune[PSATD_TUNE_FUSE_EB] = d.fuse;
  d.pull = (!h.split && !d.fuse && h.batches.size() == 1) ? 1 : 0;
  p->tune[PSATD_TUNE_PULL_EB] = d.pull;
  d.nF = h.itemsF.back();
  d.nU = h.itemsU.back();
  d.nI = h.itemsI.back();
  d.nP = h.itemsP.back();
  d.nN = h.itemsN.back();
  d.ldsF = h.ldsF;
  d.ldsI = h.ldsI;
  d.ldsU = h.ldsU;
  d.PB = h.PB;
  d.zcl = h.zcls.empty() ? 0 : 1;
  d.nzc = (int32_t)h.zcls.size();
  for (int i = 0; i < d.nzc; ++i) d.zc[i] = h.zcls[i];
  d.itemsZC = reinterpret_cast<const int32_t*>(B + o_zc);
  d.ldsH = heat_lds(h);
  d.ntu = h.ntu;
  d.ntxy = p->tune[PSATD_TUNE_XY_THREADS];
  d.nxyc = (int32_t)h.xyc.size();
  for (int i = 0; i < d.nxyc; ++i) d.xyc[i] = h.xyc[i];
  d.itemsXYC = reinterpret_cast<const int32_t*>(B + o_xyc);
  d.maxr = h.maxr;
  d.maxrz = h.maxrz;
  d.xcd = 1;
  d.slab = h.batch_slab;
  d.c = h.c;
  d.dt = h.dt;
  *out = p;
  return PSATD_OK;
}

void psatd_destroy(psatd_plan_t p) {
  if (!p) return;
  drop_graphs(p);
  if (p->ws_owned && p->ws) (void)hipFree(p->ws);
  if (p->blob) (void)hipFree(p->blob);
  if (p->d_itemsU) (void)hipFree(p->d_itemsU);
  if (p->cap_stream) (void)hipStreamDestroy(p->cap_stream);
  delete p;
}

psatd_status psatd_field_elems(psatd_plan_t p, int64_t* total) {
  if (!p || !total) return fail(p, PSATD_E_INVALID, "null argument");
  *total = p->h.field_elems;
  return PSATD_OK;
}

psatd_status psatd_field_layout(psatd_plan_t p, int32_t s, int64_t padded_n[3], int64_t* offset) {
  if (!p || !padded_n || !offset) return fail(p, PSATD_E_INVALID, "null argument");
  if (s < 0 || s >= p->h.nsub) return fail(p, PSATD_E_INVALID, "subdomain index out of range");
  const BoxD& b = p->h.box[s];
  for (int u = 0; u < 3; ++u) padded_n[u] = b.P[u];
  *offset = b.foff;
  return PSATD_OK;
}

psatd_status psatd_workspace_bytes(psatd_plan_t p, int64_t* bytes) {
  if (!p || !bytes) return fail(p, PSATD_E_INVALID, "null argument");
  *bytes = workspace_need(p);
  return PSATD_OK;
}

psatd_status psatd_set_workspace(psatd_plan_t p, void* dev, int64_t bytes) {
  if (!p) return fail(p, PSATD_E_INVALID, "null plan");
  if (dev && bytes < workspace_need(p)) return fail(p, PSATD_E_INVALID, "workspace too small");
  if (dev && ((uintptr_t)dev & 255u)) return fail(p, PSATD_E_INVALID, "workspace not 256-byte aligned");
  drop_graphs(p);
  if (p->ws_owned && p->ws) HIPCHK(p, hipFree(p->ws));
  p->ws = dev;
  p->ws_bytes = dev ? bytes : 0;
  p->ws_owned = false;
  return PSATD_OK;
}

psatd_status psatd_step(psatd_plan_t p, void* const E[3], void* const B[3], void* const J[3]) {
  psatd_status r = check_step_args(p, E, B, J);
  if (r != PSATD_OK) return r;
  return enqueue_step(p, E, B, J, p->stream, true, true);
}

psatd_status psatd_step_noalloc(psatd_plan_t p, void* const E[3], void* const B[3], void* const J[3]) {
  if (!p) return fail(nullptr, PSATD_E_INVALID, "null plan");
  psatd_status r;
  if ((r = check_fields(p, E, 3, "E")) != PSATD_OK) return r;
  if ((r = check_fields(p, B, 3, "B")) != PSATD_OK) return r;
  if ((r = check_fields(p, J, 3, "J")) != PSATD_OK) return r;
  const int64_t need = workspace_need(p);
  if (need > kScratchBytes)
    return fail(p, PSATD_E_INVALID,
                "the plan's workspace (" + std::to_string(need) + " bytes) exceeds the static scratch of " +
                    std::to_string(kScratchBytes) + " bytes; batch the boxes (PSATD_TUNE_BATCH_BOXES)");
  void* ws = scratch_of(p->device);
  if (!ws) return fail(p, PSATD_E_STATE, "static scratch not resolved on the plan's device");
  return enqueue_step(p, E, B, J, p->stream, true, true, nullptr, ws);
}

psatd_status psatd_run(psatd_plan_t p, void* const E[3], void* const B[3], void* const J[3],
                       int32_t nsteps) {
  psatd_status r = check_step_args(p, E, B, J);
  if (r != PSATD_OK) return r;
  if (nsteps < 0) return fail(p, PSATD_E_INVALID, "nsteps < 0");
  if (nsteps == 0) return PSATD_OK;
  void* key[9] = {E[0], E[1], E[2], B[0], B[1], B[2], J[0], J[1], J[2]};
  GraphEntry* ge = nullptr;
  for (auto& g : p->graphs)
    if (g.nsteps == nsteps && std::memcmp(g.ptr, key, sizeof(key)) == 0) ge = &g;
  if (!ge) {
    if (p->graphs.size() >= 8) drop_graphs(p);
    GraphEntry g{};
    std::memcpy(g.ptr, key, sizeof(key));
    g.nsteps = nsteps;
    HIPCHK(p, hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeRelaxed));
    psatd_status er = PSATD_OK;
    for (int i = 0; i < nsteps && er == PSATD_OK; ++i)
      er = enqueue_step(p, E, B, J, p->cap_stream, i == 0, i == nsteps - 1);
    hipGraph_t graph = nullptr;
    hipError_t e2 = hipStreamEndCapture(p->cap_stream, &graph);
    if (er != PSATD_OK) {
      if (graph) (void)hipGraphDestroy(graph);
      return er;
    }
    if (e2 != hipSuccess) return fail(p, PSATD_E_HIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e2));
    g.graph = graph;
    hipError_t e3 = hipGraphInstantiate(&g.exec, graph, nullptr, nullptr, 0);
    if (e3 != hipSuccess) {
      (void)hipGraphDestroy(graph);
      return fail(p, PSATD_E_HIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e3));
    }
    p->graphs.push_back(g);
    ge = &p->graphs.back();
  }
  HIPCHK(p, hipGraphLaunch(ge->exec, p->stream));
  return PSATD_OK;
}

psatd_status psatd_heat_run(psatd_plan_t p, void* u, double diffusivity, int32_t nsteps) {
  if (!p) return fail(nullptr, PSATD_E_INVALID, "null plan");
  void* one[1] = {u};
  psatd_status r = check_fields(p, one, 1, "u");
  if (r != PSATD_OK) return r;
  if (!(diffusivity >= 0.0) || !std::isfinite(diffusivity))
    return fail(p, PSATD_E_INVALID, "diffusivity must be finite and >= 0");
  if (nsteps < 0) return fail(p, PSATD_E_INVALID, "nsteps < 0");
  if (p->dp.split) return fail(p, PSATD_E_UNSUPPORTED, "the heat step needs padded planes that fit the LDS");
  if (p->h.batches.size() != 1) return fail(p, PSATD_E_STATE, "the heat step needs all boxes in one batch");
  if ((r = ensure_workspace(p)) != PSATD_OK) return r;
  const DevPlan& d = p->dp;
  const Batch all{0, d.nsub, 0, d.nP, 0, d.nU, 0, d.nN, 0};
  void* in9[9] = {u, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
  void* out6[6] = {u, nullptr, nullptr, nullptr, nullptr, nullptr};
  for (int i = 0; i < nsteps; ++i) {
    HIPCHK(p, launch_fwd(d, all, in9, p->ws, p->stream, true));
    HIPCHK(p, launch_heat_z(d, p->ws, diffusivity, d.dt, p->stream));
    HIPCHK(p, launch_inv(d, all, p->ws, out6, p->stream, true));
    HIPCHK(p, launch_fill(d, out6, 1, p->stream));
  }
  return PSATD_OK;
}

namespace {

// nsteps eager steps with an event pair around every launch.  exchange_J: the
// first step exchanges J (sum in deposited mode, owner copy in replicated
// mode); the later steps find it consistent (psatd_run semantics).  Without
// it no step touches J.
psatd_status run_profiled(psatd_plan_t p, void* const E[3], void* const B[3], void* const J[3], int32_t nsteps,
                          double* phase_ms, bool exchange_J) {
  const size_t npairs = 2 + 3 * p->h.batches.size();
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev(npairs);
  psatd_status out = PSATD_OK;
  size_t made = 0;
  for (; made < npairs; ++made) {
    if (hipEventCreate(&ev[made].second.first) != hipSuccess) { out = fail(p, PSATD_E_HIP, "hipEventCreate"); break; }
    if (hipEventCreate(&ev[made].second.second) != hipSuccess) {
      (void)hipEventDestroy(ev[made].second.first);
      out = fail(p, PSATD_E_HIP, "hipEventCreate");
      break;
    }
  }
  double acc[kNumPhases] = {0, 0, 0, 0, 0};
  for (int stp = 0; stp < nsteps && out == PSATD_OK; ++stp) {
    const bool first = exchange_J && stp == 0;
    const size_t used = first ? npairs : npairs - 1;  // pairs recorded by this step
    out = enqueue_step(p, E, B, J, p->stream, first, stp == nsteps - 1, &ev);
    if (out != PSATD_OK) break;
    if (hipEventSynchronize(ev[used - 1].second.second) != hipSuccess) { out = fail(p, PSATD_E_HIP, "hipEventSynchronize"); break; }
    for (size_t i = 0; i < used; ++i) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, ev[i].second.first, ev[i].second.second) != hipSuccess) {
        out = fail(p, PSATD_E_HIP, "hipEventElapsedTime");
        break;
      }
      acc[ev[i].first] += ms;
    }
  }
  for (size_t i = 0; i < made; ++i) {
    (void)hipEventDestroy(ev[i].second.first);
    (void)hipEventDestroy(ev[i].second.second);
  }
  if (out != PSATD_OK) return out;
  for (int ph = 0; ph < kNumPhases; ++ph) phase_ms[ph] = acc[ph] / nsteps;
  return PSATD_OK;
}

}  // namespace

psatd_status psatd_run_profiled(psatd_plan_t p, void* const E[3], void* const B[3], void* const J[3],
                                int32_t nsteps, double* phase_ms) {
  psatd_status r = check_step_args(p, E, B, J);
  if (r != PSATD_OK) return r;
  if (nsteps < 1 || !phase_ms) return fail(p, PSATD_E_INVALID, "nsteps < 1 or null phase_ms");
  return run_profiled(p, E, B, J, nsteps, phase_ms, true);
}

psatd_status psatd_scatter(psatd_plan_t p, const void* const global[3], void* const padded[3]) {
  if (!p) return fail(nullptr, PSATD_E_INVALID, "null plan");
  psatd_status r;
  if ((r = check_fields(p, const_cast<void* const*>(global), 3, "global")) != PSATD_OK) return r;
  if ((r = check_fields(p, padded, 3, "padded")) != PSATD_OK) return r;
  HIPCHK(p, launch_scatter(p->dp, global, padded, p->stream));
  return PSATD_OK;
}

psatd_status psatd_gather(psatd_plan_t p, const void* const padded[3], void* const global[3]) {
  if (!p) return fail(nullptr, PSATD_E_INVALID, "null plan");
  psatd_status r;
  if ((r = check_fields(p, const_cast<void* const*>(padded), 3, "padded")) != PSATD_OK) return r;
  if ((r = check_fields(p, global, 3, "global")) != PSATD_OK) return r;
  HIPCHK(p, launch_gather(p->dp, padded, global, p->stream));
  return PSATD_OK;
}

psatd_status psatd_modified_k(psatd_plan_t p, int32_t s, int32_t axis, double* out, int64_t len) {
  if (!p || !out) return fail(p, PSATD_E_INVALID, "null argument");
  if (s < 0 || s >= p->h.nsub || axis < 0 || axis > 2) return fail(p, PSATD_E_INVALID, "index out of range");
  const BoxD& b = p->h.box[s];
  if (len != b.P[axis]) return fail(p, PSATD_E_INVALID, "len must equal the padded length of the axis");
  const int off = axis == 0 ? b.kx : (axis == 1 ? b.ky : b.kz);
  HIPCHK(p, hipStreamSynchronize(p->stream));
  HIPCHK(p, hipMemcpy(out, p->dp.kmod + off, (size_t)len * 8, hipMemcpyDeviceToHost));
  return PSATD_OK;
}

psatd_status psatd_set_tuning(psatd_plan_t p, int32_t key, int32_t value) {
  if (!p) return fail(nullptr, PSATD_E_INVALID, "null plan");
  if (key < 0 || key >= PSATD_NTUNE) return fail(p, PSATD_E_INVALID, "unknown tuning key");
  DevPlan& d = p->dp;
  switch (key) {
    case PSATD_TUNE_Z_PENCILS: {
      if (value == 0) {  // one launch per class of tile size
        if (p->h.zcls.empty() || p->h.batches.size() > 1)
          return fail(p, PSATD_E_INVALID,
                      "per-class z launches need an unbatched plan whose boxes take several tile sizes");
        d.zcl = 1;
        break;
      }
      if (value != 4 && value != 6 && value != 8 && value != 10 && value != 16)
        return fail(p, PSATD_E_INVALID, "z pencils must be 0 (per launch class), 4, 6, 8 or 16");
      if (!z_tile_fits(p->h, max_padded_z(p->h), value))
        return fail(p, PSATD_E_INVALID, "z tile does not fit the LDS");
      HIPCHK(p, hipStreamSynchronize(p->stream));
      set_z_tile(p->h, value);
      HIPCHK(p, hipMemcpy(p->d_itemsU, p->h.itemsU.data(), p->h.itemsU.size() * 4, hipMemcpyHostToDevice));
      HIPCHK(p, prepare_kernels(d.f64, d.spl, p->h.ldsF, p->h.ldsI, z_lds_max(p->h), p->h.ldsX, p->h.ldsY));
      d.zcl = 0;
      d.PB = p->h.PB;
      d.ldsU = p->h.ldsU;
      d.ldsH = heat_lds(p->h);
      d.nU = p->h.itemsU.back();
      break;
    }
    case PSATD_TUNE_SPLIT_XY: {
      if (value != 0 && value != 1) return fail(p, PSATD_E_INVALID, "split must be 0 or 1");
      if (!value && p->h.ldsF > kMaxDynLds) return fail(p, PSATD_E_INVALID, "the padded planes need the split passes");
      if (value && p->h.batches.size() > 1) return fail(p, PSATD_E_INVALID, "the split passes do not batch");
      p->h.split = value != 0;
      d.split = value;
      if (value) {  // the split x pass reads its rows in place
        d.pull = 0;
        p->tune[PSATD_TUNE_PULL_EB] = 0;
      }
      break;
    }
    case PSATD_TUNE_BATCH_BOXES: {
      if (value < 0) return fail(p, PSATD_E_INVALID, "boxes per batch must be >= 0");
      if (value > 0 && value < p->h.nsub && p->h.split)
        return fail(p, PSATD_E_INVALID, "the split x/y passes do not batch");
      HIPCHK(p, hipStreamSynchronize(p->stream));
      set_batches(p->h, value);
      d.slab = p->h.batch_slab;
      if (p->h.batches.size() > 1) {  // a later batch must still read its old guards
        p->h.fuse_eb = false;
        d.fuse = 0;
        p->tune[PSATD_TUNE_FUSE_EB] = 0;
        d.pull = 0;  // and its owners' old interiors
        p->tune[PSATD_TUNE_PULL_EB] = 0;
        if (d.ntxy == 0) {  // batches launch every box of a batch with one group size
          d.ntxy = p->h.ntxy;
          p->tune[PSATD_TUNE_XY_THREADS] = p->h.ntxy;
        }
        if (d.zcl) {  // and one tile size
          d.zcl = 0;
          p->tune[PSATD_TUNE_Z_PENCILS] = p->h.PB;
        }
      }
      break;
    }
    case PSATD_TUNE_FUSE_EB: {
      if (value != 0 && value != 1) return fail(p, PSATD_E_INVALID, "fuse must be 0 or 1");
      if (value && p->h.batches.size() > 1)
        return fail(p, PSATD_E_INVALID, "the fused E,B exchange needs all boxes in one batch");
      p->h.fuse_eb = value != 0;
      d.fuse = value;
      if (value) {  // the inverse pass keeps every guard copy current
        d.pull = 0;
        p->tune[PSATD_TUNE_PULL_EB] = 0;
      }
      break;
    }
    case PSATD_TUNE_PULL_EB: {
      if (value != 0 && value != 1) return fail(p, PSATD_E_INVALID, "pull_eb must be 0 or 1");
      if (value && (p->h.batches.size() > 1 || d.split || d.fuse))
        return fail(p, PSATD_E_INVALID, "the pulled E,B exchange needs one batch, unsplit x/y passes and no fused exchange");
      d.pull = value;
      break;
    }
    case PSATD_TUNE_Z_REG:
      if (value != 0 && value != 1) return fail(p, PSATD_E_INVALID, "z_reg must be 0 or 1");
      if (value && !p->h.zreg)
        return fail(p, PSATD_E_INVALID, "no register z schedule for this plan (FP32 VALU form, compiled lengths)");
      d.zreg = value;
      break;
    case PSATD_TUNE_XCD_REMAP:
      if (value != 0 && value != 1) return fail(p, PSATD_E_INVALID, "xcd remap must be 0 or 1");
      d.xcd = value;
      break;
    case PSATD_TUNE_MAX_RADIX:
    case PSATD_TUNE_MAX_RADIX_Z: {
      if (value != 8 && value != 16) return fail(p, PSATD_E_INVALID, "max radix must be 8 or 16");
      if (value != 16 && p->h.spl) return fail(p, PSATD_E_INVALID, "the matrix-core forms use radix <= 16");
      const bool zk = key == PSATD_TUNE_MAX_RADIX_Z;
      HostTables trial = p->h;
      if (!set_max_radix(trial, zk ? p->h.maxr : value, zk ? value : p->h.maxrz))
        return fail(p, PSATD_E_INVALID, "a padded length has no schedule with this max radix");
      HIPCHK(p, hipStreamSynchronize(p->stream));
      HIPCHK(p, hipMemcpy(const_cast<FftPlanD*>(d.plans), trial.plans.data(),
                          trial.plans.size() * sizeof(FftPlanD), hipMemcpyHostToDevice));
      {  // the twiddle tables follow the radix schedule
        const std::vector<unsigned char> t = device_twiddles(trial);
        HIPCHK(p, hipMemcpy(const_cast<void*>(d.tw), t.data(), t.size(), hipMemcpyHostToDevice));
      }
      p->h.plans = trial.plans;
      p->h.twr = trial.twr;
      p->h.twi = trial.twi;
      p->h.maxr = trial.maxr;
      p->h.maxrz = trial.maxrz;
      d.maxr = trial.maxr;
      d.maxrz = trial.maxrz;
      break;
    }
    case PSATD_TUNE_XY_THREADS:
      if (value != 0 && value != 256 && value != 512 && value != 1024)
        return fail(p, PSATD_E_INVALID, "x/y threads must be 0 (per launch class), 256, 512 or 1024");
      if (value == 0 && (p->h.xyc.size() < 2 || p->h.batches.size() > 1))
        return fail(p, PSATD_E_INVALID,
                    "per-class x/y launches need an unbatched plan whose boxes have several plane sizes");
      if (value) p->h.ntxy = value;
      d.ntxy = value;
      break;
    case PSATD_TUNE_Z_THREADS:
      if (value != 512 && value != 1024) return fail(p, PSATD_E_INVALID, "z threads must be 512 or 1024");
      p->h.ntu = value;
      d.ntu = value;
      break;
    default: {
      if (value < 0) return fail(p, PSATD_E_INVALID, "grid size must be >= 0");
      static const int phase_of[] = {0, 0, kPhaseFwd, kPhaseUpd, kPhaseInv, kPhaseExchEB, 0, 0, 0, 0, 0, 0, 0, 0, 0};
      d.grid_cap[phase_of[key]] = value;
      if (key == PSATD_TUNE_GRID_EXCH) d.grid_cap[kPhaseExchJ] = value;
    }
  }
  p->tune[key] = value;
  drop_graphs(p);
  return PSATD_OK;
}

psatd_status psatd_get_tuning(psatd_plan_t p, int32_t key, int32_t* value) {
  if (!p || !value) return fail(p, PSATD_E_INVALID, "null argument");
  if (key < 0 || key >= PSATD_NTUNE) return fail(p, PSATD_E_INVALID, "unknown tuning key");
  *value = p->tune[key];
  return PSATD_OK;
}

namespace {

// Mean ms per step of each phase over nsteps, J left as it is (the tuner has
// exchanged it once already).
psatd_status time_phases(psatd_plan_t p, void* const E[3], void* const B[3], void* const J[3], int nsteps,
                         double* ms) {
  return run_profiled(p, E, B, J, nsteps, ms, false);
}

std::string tune_key(psatd_plan_t p) {
  hipDeviceProp_t prop;
  std::string dev = "gpu";
  if (hipGetDeviceProperties(&prop, p->device) == hipSuccess) dev = prop.gcnArchName;
  for (char& ch : dev)
    if (ch == ' ' || ch == ':') ch = '_';
  std::map<std::string, int> shapes;
  for (const BoxD& b : p->h.box)
    shapes[std::to_string(b.P[0]) + "x" + std::to_string(b.P[1]) + "x" + std::to_string(b.P[2])]++;
  std::ostringstream k;
  k << dev << "|prec" << p->h.prec << "|batch" << p->h.batch_boxes << "|";
  for (auto& kv : shapes) k << kv.first << "*" << kv.second << ",";
  return k.str();
}

}  // namespace

psatd_status psatd_autotune(psatd_plan_t p, void* const E[3], void* const B[3], void* const J[3],
                            int32_t steps, const char* cache_path, double* best_ms) {
  psatd_status r = check_step_args(p, E, B, J);
  if (r != PSATD_OK) return r;
  if (steps < 1) return fail(p, PSATD_E_INVALID, "steps_per_trial < 1");
  const std::string key = tune_key(p);
  constexpr int nk = 6;
  static const int keys[nk] = {PSATD_TUNE_MAX_RADIX, PSATD_TUNE_XY_THREADS, PSATD_TUNE_Z_PENCILS,
                               PSATD_TUNE_Z_THREADS, PSATD_TUNE_XCD_REMAP, PSATD_TUNE_MAX_RADIX_Z};
  if (cache_path) {
    std::ifstream in(cache_path);
    std::string line;
    while (std::getline(in, line)) {
      std::istringstream ls(line);
      std::string k;
      int v[nk];
      if (!(ls >> k >> v[0] >> v[1] >> v[2] >> v[3] >> v[4] >> v[5]) || k != key) continue;
      for (int i = 0; i < nk; ++i)
        if ((r = psatd_set_tuning(p, keys[i], v[i])) != PSATD_OK) return r;
      if (best_ms) *best_ms = 0.0;
      return PSATD_OK;
    }
  }
  // J is exchanged once, as psatd_step would (summed in deposited mode); the
  // trial steps then leave it alone, so deposited currents are summed exactly
  // once however many candidates are timed.
  HIPCHK(p, hipStreamSynchronize(p->stream));
  if (p->h.jmode == PSATD_J_DEPOSITED) HIPCHK(p, launch_sum(p->dp, J, p->stream));
  HIPCHK(p, launch_fill(p->dp, J, 3, p->stream));
  // Phases are separate kernels with radix limits of their own: the x/y
  // shape and radix and the z shape and radix are tuned independently.
  int best[nk] = {p->tune[PSATD_TUNE_MAX_RADIX], p->tune[PSATD_TUNE_XY_THREADS], p->tune[PSATD_TUNE_Z_PENCILS],
                  p->tune[PSATD_TUNE_Z_THREADS], p->tune[PSATD_TUNE_XCD_REMAP], p->tune[PSATD_TUNE_MAX_RADIX_Z]};
  double ms[kNumPhases];
  double bxy = 1e300, bz = 1e300, other = 0.0;
  for (int maxr : {16, 8}) {
    if (psatd_set_tuning(p, PSATD_TUNE_MAX_RADIX, maxr) != PSATD_OK) continue;
    if (psatd_set_tuning(p, PSATD_TUNE_MAX_RADIX_Z, maxr) != PSATD_OK) continue;
    for (int xcd : {1, 0}) {
      if ((r = psatd_set_tuning(p, PSATD_TUNE_XCD_REMAP, xcd)) != PSATD_OK) return r;
      for (int xy : {0, 256, 512, 1024}) {
        // the split x/y passes run fixed 256-thread groups: one x/y shape to time
        if (p->h.split && xy != 256) continue;
        // 0: one launch per class of plane size, for uneven boxes of an unbatched plan
        if (xy == 0 && (p->h.xyc.size() < 2 || p->h.batches.size() > 1)) continue;
        if ((r = psatd_set_tuning(p, PSATD_TUNE_XY_THREADS, xy)) != PSATD_OK) return r;
        for (int pb : {0, 16, 10, 8, 6, 4}) {  // 0: per class of tile size, when the plan has classes
          if (psatd_set_tuning(p, PSATD_TUNE_Z_PENCILS, pb) != PSATD_OK) continue;
          for (int zt : {512, 1024}) {
            if ((r = psatd_set_tuning(p, PSATD_TUNE_Z_THREADS, zt)) != PSATD_OK) return r;
            if ((r = time_phases(p, E, B, J, 1, ms)) != PSATD_OK) return r;  // warm-up
            if ((r = time_phases(p, E, B, J, steps, ms)) != PSATD_OK) return r;
            const double txy = ms[kPhaseFwd] + ms[kPhaseInv];
            const double tz = ms[kPhaseUpd];
            if (txy < bxy) { bxy = txy; best[0] = maxr; best[1] = xy; best[4] = xcd; }
            if (tz < bz) { bz = tz; best[5] = maxr; best[2] = pb; best[3] = zt; }
            other = ms[kPhaseExchJ] + ms[kPhaseExchEB];
          }
        }
      }
    }
  }
  // the radix limits first (they rebuild the schedules), then the shapes
  static const int order[nk] = {0, 5, 1, 2, 3, 4};
  for (int i : order)
    if ((r = psatd_set_tuning(p, keys[i], best[i])) != PSATD_OK) return r;
  const double best_total = bxy + bz + other;
  if (bxy >= 1e299 || bz >= 1e299) return fail(p, PSATD_E_STATE, "no launch shape could be timed");
  if (best_ms) *best_ms = best_total;
  if (cache_path) {
    std::ofstream out(cache_path, std::ios::app);
    if (out) {
      out << key;
      for (int i = 0; i < nk; ++i) out << " " << best[i];
      out << "\n";
    }
  }
  return PSATD_OK;
}

psatd_status psatd_set_stream(psatd_plan_t p, void* stream) {
  if (!p) return fail(nullptr, PSATD_E_INVALID, "null plan");
  p->stream = reinterpret_cast<hipStream_t>(stream);
  return PSATD_OK;
}

psatd_status psatd_sync(psatd_plan_t p) {
  if (!p) return fail(nullptr, PSATD_E_INVALID, "null plan");
  HIPCHK(p, hipStreamSynchronize(p->stream));
  return PSATD_OK;
}

const char* psatd_status_string(psatd_status st) {
  switch (st) {
    case PSATD_OK: return "PSATD_OK";
    case PSATD_E_INVALID: return "PSATD_E_INVALID";
    case PSATD_E_NOMEM: return "PSATD_E_NOMEM";
    case PSATD_E_HIP: return "PSATD_E_HIP";
    case PSATD_E_UNSUPPORTED: return "PSATD_E_UNSUPPORTED";
    case PSATD_E_STATE: return "PSATD_E_STATE";
  }
  return "PSATD_E_UNKNOWN";
}

const char* psatd_last_error(psatd_plan_t p) { return p ? p->err.c_str() : g_last_error.c_str(); }

const char* psatd_version(void) { return "0.1.0"; }

}  // extern "C"
