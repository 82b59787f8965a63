// __global__ wrappers and launchers for the phases of the local-FFT PSATD step.
//
// Every phase is ONE launch over a flattened work list spanning all subdomains
// (uneven sizes and guard widths included): a work-group takes items
// blockIdx.x, blockIdx.x + gridDim.x, ... so the same kernel runs either one
// work-group per item or as a persistent grid.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "mfma_dft.hpp"
#include "psatd_launch.hpp"
#include "zreg.hpp"

namespace psatd {

struct BlockBarrier {
  __device__ void operator()() const { __syncthreads(); }
};

extern __shared__ __attribute__((aligned(16))) unsigned char psatd_lds[];

// The matrix-core instruction of the split-BF16 DFT stage.
struct MmaHw {
  __device__ f32x4 operator()(bf16x8 a, bf16x8 b, f32x4 c) const {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};

// FFT engine by precision form: SPL = 0 VALU radix stages; 2 or 3 BF16 terms
// in a matrix-core first stage.
template <int SPL>
struct EngOf {
  using type = FftMfma<SPL, MmaHw>;
};
template <>
struct EngOf<0> {
  using type = FftValu;
};

// Work-groups are dispatched round-robin over the 8 XCDs; with remap, block
// b of the first 8*floor(G/8) takes item (b % 8) * (G/8) + b / 8 so that
// consecutive items (neighbouring memory) run on one XCD and share its L2.
__device__ __forceinline__ int first_item(int remap) {
  int b = blockIdx.x;
  const int G = gridDim.x;
  if (remap && G >= 8) {
    const int full = G & ~7;
    if (b < full) b = (b & 7) * (full >> 3) + (b >> 3);
  }
  return b;
}

template <typename T, int NT, int MAXR, int SPL>
__global__ __launch_bounds__(NT) void k_fwd_xy(FwdArgs<T> a, int item0, int nitems, int remap) {
  cx<T>* lds = reinterpret_cast<cx<T>*>(psatd_lds);
  for (int it = first_item(remap); it < nitems; it += gridDim.x) {
    body_fwd_xy<T, MAXR>(a, item0 + it, threadIdx.x, NT, lds, BlockBarrier{}, typename EngOf<SPL>::type{});
    __syncthreads();
  }
}

template <typename T, bool INC, int NT, int MAXR, int SPL, bool PUSH>
__global__ __launch_bounds__(NT) void k_inv_xy(InvArgs<T> a, int item0, int nitems, int remap) {
  cx<T>* lds = reinterpret_cast<cx<T>*>(psatd_lds);
  for (int it = first_item(remap); it < nitems; it += gridDim.x) {
    body_inv_xy<T, INC, MAXR, PUSH>(a, item0 + it, threadIdx.x, NT, lds, BlockBarrier{},
                                    typename EngOf<SPL>::type{});
    __syncthreads();
  }
}

// FP32: at most 128 VGPRs, so that two 512-thread tiles share a CU (four
// waves per SIMD); FP64 tiles measured slower when held to that budget.
template <typename T, int NT, int PB, bool INC, int MAXR, int SPL>
__global__ __launch_bounds__(NT, sizeof(T) == 4 ? 4 : 1) void k_z_update(UpdArgs<T> a, int item0, int nitems,
                                                                          int remap) {
  cx<T>* lds = reinterpret_cast<cx<T>*>(psatd_lds);
  for (int it = first_item(remap); it < nitems; it += gridDim.x) {
    body_z_update<T, PB, INC, MAXR>(a, item0 + it, threadIdx.x, NT, lds, BlockBarrier{},
                                    typename EngOf<SPL>::type{});
    __syncthreads();
  }
}

// Register z pass (FP32 forms, padded z length N).  The VGPR budget keeps
// at least MINW waves per SIMD resident.
template <int N, int L, int W, int MINW>
__global__ __launch_bounds__(64 * W) __attribute__((amdgpu_waves_per_eu(MINW)))
void k_z_reg(UpdArgs<float> a, const int32_t* items, int nitems, int remap) {
  __shared__ __attribute__((aligned(16))) unsigned char lds_raw[ZReg<N, L, W>::LDS_BYTES];
  cx<float>* lds = reinterpret_cast<cx<float>*>(lds_raw);
  for (int it = first_item(remap); it < nitems; it += gridDim.x) {
    body_z_reg<N, L, W>(a, items, it, threadIdx.x, lds);
    __syncthreads();
  }
}

template <typename T, int PB, bool INC, int MAXR, int SPL>
__global__ __launch_bounds__(kThreadsXY) void k_z_heat(HeatArgs<T> a, int nitems, int remap) {
  cx<T>* lds = reinterpret_cast<cx<T>*>(psatd_lds);
  for (int it = first_item(remap); it < nitems; it += gridDim.x) {
    body_z_heat<T, PB, INC, MAXR>(a, it, threadIdx.x, kThreadsXY, lds, BlockBarrier{},
                                  typename EngOf<SPL>::type{});
    __syncthreads();
  }
}

template <typename T, int MAXR, int SPL>
__global__ __launch_bounds__(kThreadsXY) void k_x_fwd(SplitArgs<T> a, int nitems, int remap) {
  cx<T>* lds = reinterpret_cast<cx<T>*>(psatd_lds);
  for (int it = first_item(remap); it < nitems; it += gridDim.x) {
    body_x_fwd<T, MAXR>(a, it, threadIdx.x, kThreadsXY, lds, BlockBarrier{}, typename EngOf<SPL>::type{});
    __syncthreads();
  }
}

template <typename T, int DIR, int MAXR, int SPL>
__global__ __launch_bounds__(kThreadsXY) void k_y(SplitArgs<T> a, int nitems, int remap) {
  cx<T>* lds = reinterpret_cast<cx<T>*>(psatd_lds);
  for (int it = first_item(remap); it < nitems; it += gridDim.x) {
    body_y<T, DIR, MAXR>(a, it, threadIdx.x, kThreadsXY, lds, BlockBarrier{}, typename EngOf<SPL>::type{});
    __syncthreads();
  }
}

template <typename T, bool INC, int MAXR, int SPL, bool PUSH>
__global__ __launch_bounds__(kThreadsXY) void k_x_inv(SplitArgs<T> a, int nitems, int remap) {
  cx<T>* lds = reinterpret_cast<cx<T>*>(psatd_lds);
  for (int it = first_item(remap); it < nitems; it += gridDim.x) {
    body_x_inv<T, INC, MAXR, PUSH>(a, it, threadIdx.x, kThreadsXY, lds, BlockBarrier{},
                                   typename EngOf<SPL>::type{});
    __syncthreads();
  }
}

template <typename T>
__global__ __launch_bounds__(kThreadsXY) void k_fill(FillArgs<T> a, int nitems, int remap) {
  for (int item = first_item(remap); item < nitems; item += gridDim.x)
    body_fill(a, item, threadIdx.x, blockDim.x);
}

template <typename T>
__global__ __launch_bounds__(kThreadsXY) void k_sum(SumArgs<T> a, int nitems) {
  for (int item = blockIdx.x; item < nitems; item += gridDim.x)
    body_sum(a, item, threadIdx.x, blockDim.x);
}

template <typename T>
__global__ __launch_bounds__(kThreadsXY) void k_scatter(ScatterArgs<T> a, int nitems) {
  for (int item = blockIdx.x; item < nitems; item += gridDim.x)
    body_scatter(a, item, threadIdx.x, blockDim.x);
}

template <typename T>
__global__ __launch_bounds__(kThreadsXY) void k_gather(ScatterArgs<T> a, int nitems) {
  for (int item = blockIdx.x; item < nitems; item += gridDim.x)
    body_gather(a, item, threadIdx.x, blockDim.x);
}

__global__ __launch_bounds__(256) void k_modk(const KEntry* ent, int nent, int maxN, int p,
                                              double* kmod) {
  const int e = blockIdx.y;
  if (e >= nent) return;
  const KEntry k = ent[e];
  for (int m = blockIdx.x * blockDim.x + threadIdx.x; m < k.N; m += gridDim.x * blockDim.x)
    kmod[k.off + m] = modified_k_entry(k.N, k.du, p, m);
}

// ------------------------------------------------------------------ helpers
static inline int grid_for(int nitems, int cap) {
  if (nitems <= 0) return 0;
  return (cap > 0 && cap < nitems) ? cap : nitems;
}

template <typename T>
static Tables<T> tables(const DevPlan& p) {
  Tables<T> t;
  t.box = p.box;
  t.nsub = p.nsub;
  t.plans = p.plans;
  t.tw = reinterpret_cast<const cx<T>*>(p.tw);
  t.kmod = p.kmod;
  return t;
}

// The FP32 path transforms increments (INC), the FP64 path the new fields.
template <typename T> struct IncOf { static constexpr bool value = sizeof(T) == 4; };

static hipError_t set_lds(const void* f, int lds) {
  return hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
}

// Calls f(std::integral_constant<int, SPL>) for the plan's precision form;
// the matrix-core forms exist for FP32 data only.
template <typename T, class F>
static hipError_t with_spl(int spl, F f) {
  if constexpr (std::is_same<T, float>::value) {
    if (spl == 2) return f(std::integral_constant<int, 2>{});
    if (spl == 3) return f(std::integral_constant<int, 3>{});
  }
  return f(std::integral_constant<int, 0>{});
}

template <typename T, int MAXR, int SPL>
static hipError_t prepare_t(int ldsF, int ldsI, int ldsU, int ldsX, int ldsY) {
  constexpr bool I = IncOf<T>::value;
  const void* xy[] = {(const void*)k_fwd_xy<T, 256, MAXR, SPL>, (const void*)k_fwd_xy<T, 512, MAXR, SPL>,
                      (const void*)k_fwd_xy<T, 1024, MAXR, SPL>};
  const void* inv[] = {(const void*)k_inv_xy<T, I, 256, MAXR, SPL, false>,
                       (const void*)k_inv_xy<T, I, 512, MAXR, SPL, false>,
                       (const void*)k_inv_xy<T, I, 1024, MAXR, SPL, false>,
                       (const void*)k_inv_xy<T, I, 256, MAXR, SPL, true>,
                       (const void*)k_inv_xy<T, I, 512, MAXR, SPL, true>,
                       (const void*)k_inv_xy<T, I, 1024, MAXR, SPL, true>};
  const void* upd[] = {(const void*)k_z_update<T, 512, 8, I, MAXR, SPL>,
                       (const void*)k_z_update<T, 512, 16, I, MAXR, SPL>,
                       (const void*)k_z_update<T, 1024, 8, I, MAXR, SPL>,
                       (const void*)k_z_update<T, 1024, 16, I, MAXR, SPL>,
                       (const void*)k_z_update<T, 512, 4, I, MAXR, SPL>,
                       (const void*)k_z_update<T, 512, 6, I, MAXR, SPL>,
                       (const void*)k_z_update<T, 512, 10, I, MAXR, SPL>};
  hipError_t e;
  for (const void* f : xy)
    if (ldsF <= kMaxDynLds && (e = set_lds(f, ldsF)) != hipSuccess) return e;
  for (const void* f : inv)
    if (ldsI <= kMaxDynLds && (e = set_lds(f, ldsI)) != hipSuccess) return e;
  for (const void* f : upd)
    if ((e = set_lds(f, ldsU)) != hipSuccess) return e;
  const void* heat[] = {(const void*)k_z_heat<T, 4, I, MAXR, SPL>, (const void*)k_z_heat<T, 6, I, MAXR, SPL>,
                        (const void*)k_z_heat<T, 8, I, MAXR, SPL>, (const void*)k_z_heat<T, 10, I, MAXR, SPL>,
                        (const void*)k_z_heat<T, 16, I, MAXR, SPL>};
  for (const void* f : heat)
    if ((e = set_lds(f, ldsU)) != hipSuccess) return e;
  if ((e = set_lds((const void*)k_x_fwd<T, MAXR, SPL>, ldsX)) != hipSuccess) return e;
  if ((e = set_lds((const void*)k_x_inv<T, I, MAXR, SPL, false>, ldsX)) != hipSuccess) return e;
  if ((e = set_lds((const void*)k_x_inv<T, I, MAXR, SPL, true>, ldsX)) != hipSuccess) return e;
  if ((e = set_lds((const void*)k_y<T, -1, MAXR, SPL>, ldsY)) != hipSuccess) return e;
  return set_lds((const void*)k_y<T, 1, MAXR, SPL>, ldsY);
}

hipError_t prepare_kernels(bool f64, int spl, int ldsF, int ldsI, int ldsU, int ldsX, int ldsY) {
  hipError_t e;
  if (f64) {
    if ((e = prepare_t<double, 8, 0>(ldsF, ldsI, ldsU, ldsX, ldsY)) != hipSuccess) return e;
    return prepare_t<double, 16, 0>(ldsF, ldsI, ldsU, ldsX, ldsY);
  }
  if (spl == 2) return prepare_t<float, 16, 2>(ldsF, ldsI, ldsU, ldsX, ldsY);
  if (spl == 3) return prepare_t<float, 16, 3>(ldsF, ldsI, ldsU, ldsX, ldsY);
  if ((e = prepare_t<float, 8, 0>(ldsF, ldsI, ldsU, ldsX, ldsY)) != hipSuccess) return e;
  return prepare_t<float, 16, 0>(ldsF, ldsI, ldsU, ldsX, ldsY);
}

// ---------------------------------------------------------------- launchers
template <typename T>
static hipError_t fill_t(const DevPlan& p, void* const* comps, int ncomp, hipStream_t st) {
  FillArgs<T> a;
  a.piece = p.fillp;
  a.items = p.itemsG;
  a.piece_of = p.pieceOf;
  a.ncomp = ncomp;
  for (int c = 0; c < 9; ++c) a.comp[c] = (c < ncomp) ? reinterpret_cast<T*>(comps[c]) : nullptr;
  const int g = grid_for(p.nG, p.grid_cap[kPhaseExchEB]);
  if (!g) return hipSuccess;
  hipLaunchKernelGGL(k_fill<T>, dim3(g), dim3(kThreadsXY), 0, st, a, p.nG, p.xcd);
  return hipGetLastError();
}

hipError_t launch_fill(const DevPlan& p, void* const* comps, int ncomp, hipStream_t st) {
  return p.f64 ? fill_t<double>(p, comps, ncomp, st) : fill_t<float>(p, comps, ncomp, st);
}

template <typename T>
static hipError_t sum_t(const DevPlan& p, void* const* J, hipStream_t st) {
  SumArgs<T> a;
  a.box = p.box;
  a.nsub = p.nsub;
  a.items = p.itemsN;
  a.nbr_off = p.nbr_off;
  a.nbr = p.nbr;
  for (int u = 0; u < 3; ++u) a.N[u] = p.N[u];
  for (int c = 0; c < 3; ++c) a.comp[c] = reinterpret_cast<T*>(J[c]);
  const int g = grid_for(p.nN, p.grid_cap[kPhaseExchJ]);
  if (!g) return hipSuccess;
  hipLaunchKernelGGL(k_sum<T>, dim3(g), dim3(kThreadsXY), 0, st, a, p.nN);
  return hipGetLastError();
}

hipError_t launch_sum(const DevPlan& p, void* const* J, hipStream_t st) {
  return p.f64 ? sum_t<double>(p, J, st) : sum_t<float>(p, J, st);
}

// MAXR = 8 kernels exist for the VALU form only.  MR: the pass's largest
// radix (p.maxr for the x/y passes, p.maxrz for the z passes).
#define PSATD_MAXR_SWITCH(SPL, MR, CALL8, CALL16) \
  do {                                             \
    if constexpr ((SPL) > 0) {                     \
      CALL16;                                      \
    } else if ((MR) >= 16) {                       \
      CALL16;                                      \
    } else {                                       \
      CALL8;                                       \
    }                                              \
  } while (0)

template <typename T, int NT, int MAXR, int SPL>
static hipError_t fwd_go(const DevPlan& p, const FwdArgs<T>& a, int g, int lds, int item0, int n,
                         hipStream_t st) {
  hipLaunchKernelGGL((k_fwd_xy<T, NT, MAXR, SPL>), dim3(g), dim3(NT), lds, st, a, item0, n, p.xcd);
  return hipGetLastError();
}

// One x/y launch of n items from item0 with nt threads per group.
template <typename T, class Go>
static hipError_t xy_shape(const DevPlan& p, int nt, Go go) {
  return with_spl<T>(p.spl, [&](auto sc) -> hipError_t {
    constexpr int SPL = decltype(sc)::value;
    if (nt == 1024)
      PSATD_MAXR_SWITCH(SPL, p.maxr, return (go.template run<1024, 8, SPL>()), return (go.template run<1024, 16, SPL>()));
    if (nt == 512)
      PSATD_MAXR_SWITCH(SPL, p.maxr, return (go.template run<512, 8, SPL>()), return (go.template run<512, 16, SPL>()));
    PSATD_MAXR_SWITCH(SPL, p.maxr, return (go.template run<256, 8, SPL>()), return (go.template run<256, 16, SPL>()));
    return hipSuccess;
  });
}

template <typename T>
struct FwdGo {
  const DevPlan& p;
  const FwdArgs<T>& a;
  int g, lds, item0, n;
  hipStream_t st;
  template <int NT, int MAXR, int SPL>
  hipError_t run() const { return fwd_go<T, NT, MAXR, SPL>(p, a, g, lds, item0, n, st); }
};

template <typename T>
static hipError_t fwd_t(const DevPlan& p, const Batch& b, void* const* in9, void* spec, hipStream_t st,
                        bool scalar) {
  FwdArgs<T> a;
  a.t = tables<T>(p);
  a.items = scalar ? p.itemsP : p.itemsF;  // one field: P[2] planes per box
  a.nfield = scalar ? 1 : 9;
  a.npull = (p.pull && !scalar) ? 6 : 0;
  a.pull = p.pullp;
  a.pull_off = p.pull_off;
  for (int f = 0; f < 9; ++f) a.in[f] = (f < a.nfield) ? reinterpret_cast<const T*>(in9[f]) : nullptr;
  a.spec = reinterpret_cast<cx<T>*>(spec);
  a.sbias = b.sbias;
  if (p.ntxy == 0) {  // one launch per class of plane size (unbatched plans only)
    for (int c = 0; c < p.nxyc; ++c) {
      const XyClass& k = p.xyc[c];
      a.items = p.itemsXYC + (scalar ? k.P : k.F);
      const int n = scalar ? k.nP : k.nF;
      const int g = grid_for(n, p.grid_cap[kPhaseFwd]);
      if (!g) continue;
      const hipError_t e = xy_shape<T>(p, k.nt, FwdGo<T>{p, a, g, k.lds, 0, n, st});
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const int g = grid_for(b.nF, p.grid_cap[kPhaseFwd]);
  if (!g) return hipSuccess;
  return xy_shape<T>(p, p.ntxy, FwdGo<T>{p, a, g, p.ldsF, b.F0, b.nF, st});
}

hipError_t launch_fwd(const DevPlan& p, const Batch& b, void* const* in9, void* spec, hipStream_t st,
                      bool scalar) {
  return p.f64 ? fwd_t<double>(p, b, in9, spec, st, scalar) : fwd_t<float>(p, b, in9, spec, st, scalar);
}

// One z launch: n items from item0, PB pencils per tile, lds bytes of LDS.
struct UpdLaunch {
  int g, PB, lds, item0, n;
};

template <typename T, int NT, int PB, int MAXR, int SPL>
static hipError_t upd_launch(const DevPlan& p, const UpdLaunch& l, const UpdArgs<T>& a, hipStream_t st) {
  hipLaunchKernelGGL((k_z_update<T, NT, PB, IncOf<T>::value, MAXR, SPL>), dim3(l.g), dim3(NT), l.lds, st, a,
                     l.item0, l.n, p.xcd);
  return hipGetLastError();
}

template <typename T, int MAXR, int SPL>
static hipError_t upd_shape(const DevPlan& p, const UpdLaunch& l, const UpdArgs<T>& a, hipStream_t st) {
  if (l.PB == 4) return upd_launch<T, 512, 4, MAXR, SPL>(p, l, a, st);
  if (l.PB == 6) return upd_launch<T, 512, 6, MAXR, SPL>(p, l, a, st);
  if (l.PB == 10) return upd_launch<T, 512, 10, MAXR, SPL>(p, l, a, st);
  if (p.ntu == 1024)
    return l.PB == 16 ? upd_launch<T, 1024, 16, MAXR, SPL>(p, l, a, st)
                      : upd_launch<T, 1024, 8, MAXR, SPL>(p, l, a, st);
  return l.PB == 16 ? upd_launch<T, 512, 16, MAXR, SPL>(p, l, a, st)
                    : upd_launch<T, 512, 8, MAXR, SPL>(p, l, a, st);
}

template <typename T>
static hipError_t upd_t(const DevPlan& p, const Batch& b, void* spec, hipStream_t st) {
  UpdArgs<T> a;
  a.t = tables<T>(p);
  a.items = p.itemsU;
  a.spec = reinterpret_cast<cx<T>*>(spec);
  a.sbias = b.sbias;
  a.k.c = p.c;
  a.k.dt = p.dt;
  auto go = [&](const UpdLaunch& l) -> hipError_t {
    return with_spl<T>(p.spl, [&](auto sc) -> hipError_t {
      constexpr int SPL = decltype(sc)::value;
      PSATD_MAXR_SWITCH(SPL, p.maxrz, return (upd_shape<T, 8, SPL>(p, l, a, st)),
                        return (upd_shape<T, 16, SPL>(p, l, a, st)));
      return hipSuccess;
    });
  };
  if (p.zcl) {  // one launch per class of tile size (unbatched plans only)
    for (int c = 0; c < p.nzc; ++c) {
      const ZClass& k = p.zc[c];
      a.items = p.itemsZC + k.U;
      const int g = grid_for(k.nU, p.grid_cap[kPhaseUpd]);
      if (!g) continue;
      const hipError_t e = go(UpdLaunch{g, k.PB, k.lds, 0, k.nU});
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const int g = grid_for(b.nU, p.grid_cap[kPhaseUpd]);
  if (!g) return hipSuccess;
  return go(UpdLaunch{g, p.PB, p.ldsU, b.U0, b.nU});
}

hipError_t launch_upd(const DevPlan& p, const Batch& b, void* spec, hipStream_t st) {
  return p.f64 ? upd_t<double>(p, b, spec, st) : upd_t<float>(p, b, spec, st);
}

template <int N, int L, int W, int MINW>
static hipError_t zreg_go(const UpdArgs<float>& a, const int32_t* items, int n, int cap, int remap,
                          hipStream_t st) {
  const int g = grid_for(n, cap);
  if (!g) return hipSuccess;
  hipLaunchKernelGGL((k_z_reg<N, L, W, MINW>), dim3(g), dim3(64 * W), 0, st, a, items, n, remap);
  return hipGetLastError();
}

// One launch per group of boxes sharing a padded z length (every box of the
// plan belongs to a group with a register schedule, see zreg_schedule).
hipError_t launch_upd_reg(const DevPlan& p, void* spec, hipStream_t st) {
  UpdArgs<float> a;
  a.t = tables<float>(p);
  a.items = nullptr;
  a.spec = reinterpret_cast<cx<float>*>(spec);
  a.sbias = 0;
  a.k.c = p.c;
  a.k.dt = p.dt;
  const int cap = p.grid_cap[kPhaseUpd];
  for (int i = 0; i < p.nzg; ++i) {
    const ZGroup& zg = p.zg[i];
    const int32_t* items = p.itemsZR + zg.off;
    hipError_t e = hipErrorInvalidValue;
    switch (zg.N) {
#define PSATD_ZREG_CASE(N_, L_, W_, MINW_) \
  case N_: e = zreg_go<N_, L_, W_, MINW_>(a, items, zg.n, cap, p.xcd, st); break;
      PSATD_ZREG_SHAPES(PSATD_ZREG_CASE)
#undef PSATD_ZREG_CASE
      default: break;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T, int NT, int MAXR, int SPL>
static hipError_t inv_go(const DevPlan& p, const InvArgs<T>& a, int g, int lds, int item0, int n,
                         hipStream_t st) {
  if (a.push_off)
    hipLaunchKernelGGL((k_inv_xy<T, IncOf<T>::value, NT, MAXR, SPL, true>), dim3(g), dim3(NT), lds, st, a,
                       item0, n, p.xcd);
  else
    hipLaunchKernelGGL((k_inv_xy<T, IncOf<T>::value, NT, MAXR, SPL, false>), dim3(g), dim3(NT), lds, st, a,
                       item0, n, p.xcd);
  return hipGetLastError();
}

template <typename T>
struct InvGo {
  const DevPlan& p;
  const InvArgs<T>& a;
  int g, lds, item0, n;
  hipStream_t st;
  template <int NT, int MAXR, int SPL>
  hipError_t run() const { return inv_go<T, NT, MAXR, SPL>(p, a, g, lds, item0, n, st); }
};

template <typename T>
static hipError_t inv_t(const DevPlan& p, const Batch& b, const void* spec, void* const* out6, hipStream_t st,
                        bool scalar) {
  InvArgs<T> a;
  a.t = tables<T>(p);
  a.items = scalar ? p.itemsN : p.itemsI;  // one field: n[2] planes per box
  a.spec = reinterpret_cast<const cx<T>*>(spec);
  a.sbias = b.sbias;
  for (int f = 0; f < 6; ++f) a.out[f] = (f == 0 || !scalar) ? reinterpret_cast<T*>(out6[f]) : nullptr;
  a.push = (p.fuse && !scalar) ? p.push : nullptr;
  a.push_off = (p.fuse && !scalar) ? p.push_off : nullptr;
  if (p.ntxy == 0) {  // one launch per class of plane size (unbatched plans only)
    for (int c = 0; c < p.nxyc; ++c) {
      const XyClass& k = p.xyc[c];
      a.items = p.itemsXYC + (scalar ? k.N : k.I);
      const int n = scalar ? k.nN : k.nI;
      const int g = grid_for(n, p.grid_cap[kPhaseInv]);
      if (!g) continue;
      const hipError_t e = xy_shape<T>(p, k.nt, InvGo<T>{p, a, g, k.lds, 0, n, st});
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  const int g = grid_for(b.nI, p.grid_cap[kPhaseInv]);
  if (!g) return hipSuccess;
  return xy_shape<T>(p, p.ntxy, InvGo<T>{p, a, g, p.ldsI, b.I0, b.nI, st});
}

hipError_t launch_inv(const DevPlan& p, const Batch& b, const void* spec, void* const* out6, hipStream_t st,
                      bool scalar) {
  return p.f64 ? inv_t<double>(p, b, spec, out6, st, scalar) : inv_t<float>(p, b, spec, out6, st, scalar);
}

template <typename T>
static hipError_t heat_z_t(const DevPlan& p, void* spec, double D, double dt, hipStream_t st) {
  HeatArgs<T> a;
  a.t = tables<T>(p);
  a.items = p.itemsU;
  a.spec = reinterpret_cast<cx<T>*>(spec);
  a.D = D;
  a.dt = dt;
  const int g = grid_for(p.nU, p.grid_cap[kPhaseUpd]);
  if (!g) return hipSuccess;
  constexpr bool I = IncOf<T>::value;
  return with_spl<T>(p.spl, [&](auto sc) -> hipError_t {
    constexpr int SPL = decltype(sc)::value;
    auto go = [&](auto pbc) -> hipError_t {
      constexpr int PB = decltype(pbc)::value;
      PSATD_MAXR_SWITCH(SPL, p.maxrz,
                        hipLaunchKernelGGL((k_z_heat<T, PB, I, 8, SPL>), dim3(g), dim3(kThreadsXY), p.ldsH, st,
                                           a, p.nU, p.xcd),
                        hipLaunchKernelGGL((k_z_heat<T, PB, I, 16, SPL>), dim3(g), dim3(kThreadsXY), p.ldsH, st,
                                           a, p.nU, p.xcd));
      return hipGetLastError();
    };
    if (p.PB == 4) return go(std::integral_constant<int, 4>{});
    if (p.PB == 6) return go(std::integral_constant<int, 6>{});
    if (p.PB == 10) return go(std::integral_constant<int, 10>{});
    if (p.PB == 8) return go(std::integral_constant<int, 8>{});
    return go(std::integral_constant<int, 16>{});
  });
}

hipError_t launch_heat_z(const DevPlan& p, void* spec, double D, double dt, hipStream_t st) {
  return p.f64 ? heat_z_t<double>(p, spec, D, dt, st) : heat_z_t<float>(p, spec, D, dt, st);
}

template <typename T>
static SplitArgs<T> split_args(const DevPlan& p, void* spec) {
  SplitArgs<T> a;
  a.t = tables<T>(p);
  a.items = nullptr;
  for (int f = 0; f < 9; ++f) a.in[f] = nullptr;
  for (int f = 0; f < 6; ++f) a.out[f] = nullptr;
  a.spec = reinterpret_cast<cx<T>*>(spec);
  a.sbias = 0;
  a.push = p.fuse ? p.push : nullptr;
  a.push_off = p.fuse ? p.push_off : nullptr;
  return a;
}

template <typename T>
static hipError_t x_fwd_t(const DevPlan& p, void* const* in9, void* spec, hipStream_t st) {
  SplitArgs<T> a = split_args<T>(p, spec);
  a.items = p.itemsXF;
  for (int f = 0; f < 9; ++f) a.in[f] = reinterpret_cast<const T*>(in9[f]);
  const int g = grid_for(p.nXF, p.grid_cap[kPhaseFwd]);
  if (!g) return hipSuccess;
  return with_spl<T>(p.spl, [&](auto sc) -> hipError_t {
    constexpr int SPL = decltype(sc)::value;
    PSATD_MAXR_SWITCH(SPL, p.maxr,
                      hipLaunchKernelGGL((k_x_fwd<T, 8, SPL>), dim3(g), dim3(kThreadsXY), p.ldsX, st, a,
                                         p.nXF, p.xcd),
                      hipLaunchKernelGGL((k_x_fwd<T, 16, SPL>), dim3(g), dim3(kThreadsXY), p.ldsX, st, a,
                                         p.nXF, p.xcd));
    return hipGetLastError();
  });
}

template <typename T>
static hipError_t y_t(const DevPlan& p, int dir, void* spec, hipStream_t st) {
  SplitArgs<T> a = split_args<T>(p, spec);
  a.items = dir < 0 ? p.itemsYF : p.itemsYI;
  const int n = dir < 0 ? p.nYF : p.nYI;
  const int g = grid_for(n, p.grid_cap[dir < 0 ? kPhaseFwd : kPhaseInv]);
  if (!g) return hipSuccess;
  return with_spl<T>(p.spl, [&](auto sc) -> hipError_t {
    constexpr int SPL = decltype(sc)::value;
    if (dir < 0)
      PSATD_MAXR_SWITCH(SPL, p.maxr,
                        hipLaunchKernelGGL((k_y<T, -1, 8, SPL>), dim3(g), dim3(kThreadsXY), p.ldsY, st, a, n,
                                           p.xcd),
                        hipLaunchKernelGGL((k_y<T, -1, 16, SPL>), dim3(g), dim3(kThreadsXY), p.ldsY, st, a, n,
                                           p.xcd));
    else
      PSATD_MAXR_SWITCH(SPL, p.maxr,
                        hipLaunchKernelGGL((k_y<T, 1, 8, SPL>), dim3(g), dim3(kThreadsXY), p.ldsY, st, a, n,
                                           p.xcd),
                        hipLaunchKernelGGL((k_y<T, 1, 16, SPL>), dim3(g), dim3(kThreadsXY), p.ldsY, st, a, n,
                                           p.xcd));
    return hipGetLastError();
  });
}

template <typename T>
static hipError_t x_inv_t(const DevPlan& p, const void* spec, void* const* out6, hipStream_t st) {
  SplitArgs<T> a = split_args<T>(p, const_cast<void*>(spec));
  a.items = p.itemsXI;
  for (int f = 0; f < 6; ++f) a.out[f] = reinterpret_cast<T*>(out6[f]);
  const int g = grid_for(p.nXI, p.grid_cap[kPhaseInv]);
  if (!g) return hipSuccess;
  constexpr bool I = IncOf<T>::value;
  return with_spl<T>(p.spl, [&](auto sc) -> hipError_t {
    constexpr int SPL = decltype(sc)::value;
    auto go = [&](auto pc) {
      constexpr bool PUSH = decltype(pc)::value;
      PSATD_MAXR_SWITCH(SPL, p.maxr,
                        hipLaunchKernelGGL((k_x_inv<T, I, 8, SPL, PUSH>), dim3(g), dim3(kThreadsXY), p.ldsX, st,
                                           a, p.nXI, p.xcd),
                        hipLaunchKernelGGL((k_x_inv<T, I, 16, SPL, PUSH>), dim3(g), dim3(kThreadsXY), p.ldsX, st,
                                           a, p.nXI, p.xcd));
    };
    if (a.push_off) go(std::true_type{});
    else go(std::false_type{});
    return hipGetLastError();
  });
}

#undef PSATD_MAXR_SWITCH

hipError_t launch_x_fwd(const DevPlan& p, void* const* in9, void* spec, hipStream_t st) {
  return p.f64 ? x_fwd_t<double>(p, in9, spec, st) : x_fwd_t<float>(p, in9, spec, st);
}
hipError_t launch_y(const DevPlan& p, int dir, void* spec, hipStream_t st) {
  return p.f64 ? y_t<double>(p, dir, spec, st) : y_t<float>(p, dir, spec, st);
}
hipError_t launch_x_inv(const DevPlan& p, const void* spec, void* const* out6, hipStream_t st) {
  return p.f64 ? x_inv_t<double>(p, spec, out6, st) : x_inv_t<float>(p, spec, out6, st);
}

template <typename T>
static hipError_t scat_t(const DevPlan& p, const void* const* src, void* const* dst, bool scatter,
                         hipStream_t st) {
  ScatterArgs<T> a;
  a.box = p.box;
  a.nsub = p.nsub;
  a.items = scatter ? p.itemsP : p.itemsN;
  for (int u = 0; u < 3; ++u) a.N[u] = p.N[u];
  for (int c = 0; c < 3; ++c) {
    a.src[c] = reinterpret_cast<const T*>(src[c]);
    a.dst[c] = reinterpret_cast<T*>(dst[c]);
  }
  const int n = scatter ? p.nP : p.nN;
  if (!n) return hipSuccess;
  if (scatter)
    hipLaunchKernelGGL(k_scatter<T>, dim3(n), dim3(kThreadsXY), 0, st, a, n);
  else
    hipLaunchKernelGGL(k_gather<T>, dim3(n), dim3(kThreadsXY), 0, st, a, n);
  return hipGetLastError();
}

hipError_t launch_scatter(const DevPlan& p, const void* const* glob, void* const* pad, hipStream_t st) {
  return p.f64 ? scat_t<double>(p, glob, pad, true, st) : scat_t<float>(p, glob, pad, true, st);
}

hipError_t launch_gather(const DevPlan& p, const void* const* pad, void* const* glob, hipStream_t st) {
  return p.f64 ? scat_t<double>(p, pad, glob, false, st) : scat_t<float>(p, pad, glob, false, st);
}

hipError_t launch_modk(const KEntry* entries, int nent, int maxN, int order_p, double* kmod,
                       hipStream_t st) {
  if (nent <= 0) return hipSuccess;
  const int bx = (maxN + 255) / 256;
  hipLaunchKernelGGL(k_modk, dim3(bx, nent), dim3(256), 0, st, entries, nent, maxN, order_p, kmod);
  return hipGetLastError();
}

}  // namespace psatd
