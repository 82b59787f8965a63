// __global__ wrappers and launchers for the phases of the local-FFT PSATD step.
//
// Every phase is ONE launch over a flattened work list spanning all subdomains
// (uneven sizes and guard widths included): a work-group takes items
// blockIdx.x, blockIdx.x + gridDim.x, ... so the same kernel runs either one
// work-group per item or as a persistent grid.
#include <hip/hip_runtime.h>

#include "psatd_launch.hpp"

namespace psatd {

struct BlockBarrier {
  __device__ void operator()() const { __syncthreads(); }
};

extern __shared__ __attribute__((aligned(16))) unsigned char psatd_lds[];

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

template <typename T>
__global__ __launch_bounds__(kThreadsXY) void k_fwd_xy(FwdArgs<T> a, int item0, int nitems, int remap) {
  cx<T>* lds = reinterpret_cast<cx<T>*>(psatd_lds);
  for (int it = first_item(remap); it < nitems; it += gridDim.x) {
    body_fwd_xy(a, item0 + it, threadIdx.x, blockDim.x, lds, BlockBarrier{});
    __syncthreads();
  }
}

template <typename T, bool INC>
__global__ __launch_bounds__(kThreadsXY) void k_inv_xy(InvArgs<T> a, int item0, int nitems, int remap) {
  cx<T>* lds = reinterpret_cast<cx<T>*>(psatd_lds);
  for (int it = first_item(remap); it < nitems; it += gridDim.x) {
    body_inv_xy<T, INC>(a, item0 + it, threadIdx.x, blockDim.x, lds, BlockBarrier{});
    __syncthreads();
  }
}

template <typename T, int NT, int PB, bool INC>
__global__ __launch_bounds__(NT) void k_z_update(UpdArgs<T> a, int item0, int nitems, int remap) {
  cx<T>* lds = reinterpret_cast<cx<T>*>(psatd_lds);
  for (int it = first_item(remap); it < nitems; it += gridDim.x) {
    body_z_update<T, PB, INC>(a, item0 + it, threadIdx.x, NT, lds, BlockBarrier{});
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

template <typename T>
static hipError_t set_upd_attr(int lds) {
  constexpr bool I = IncOf<T>::value;
  const void* fns[] = {
      (const void*)k_z_update<T, 512, 2, I>,  (const void*)k_z_update<T, 512, 4, I>,
      (const void*)k_z_update<T, 512, 8, I>,  (const void*)k_z_update<T, 512, 16, I>,
      (const void*)k_z_update<T, 1024, 2, I>, (const void*)k_z_update<T, 1024, 4, I>,
      (const void*)k_z_update<T, 1024, 8, I>, (const void*)k_z_update<T, 1024, 16, I>};
  for (const void* f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t prepare_kernels(bool f64, int ldsF, int ldsI, int ldsU) {
  hipError_t e;
  if (f64) {
    if ((e = hipFuncSetAttribute((const void*)k_fwd_xy<double>, hipFuncAttributeMaxDynamicSharedMemorySize, ldsF)) != hipSuccess) return e;
    if ((e = hipFuncSetAttribute((const void*)k_inv_xy<double, IncOf<double>::value>, hipFuncAttributeMaxDynamicSharedMemorySize, ldsI)) != hipSuccess) return e;
    return set_upd_attr<double>(ldsU);
  }
  if ((e = hipFuncSetAttribute((const void*)k_fwd_xy<float>, hipFuncAttributeMaxDynamicSharedMemorySize, ldsF)) != hipSuccess) return e;
  if ((e = hipFuncSetAttribute((const void*)k_inv_xy<float, IncOf<float>::value>, hipFuncAttributeMaxDynamicSharedMemorySize, ldsI)) != hipSuccess) return e;
  return set_upd_attr<float>(ldsU);
}

// ---------------------------------------------------------------- launchers
template <typename T>
static hipError_t fill_t(const DevPlan& p, void* const* comps, int ncomp, hipStream_t st) {
  FillArgs<T> a;
  a.box = p.box;
  a.nsub = p.nsub;
  a.items = p.itemsP;
  a.own = p.own;
  a.ncomp = ncomp;
  for (int c = 0; c < 9; ++c) a.comp[c] = (c < ncomp) ? reinterpret_cast<T*>(comps[c]) : nullptr;
  const int g = grid_for(p.nP, p.grid_cap[kPhaseExchEB]);
  if (!g) return hipSuccess;
  hipLaunchKernelGGL(k_fill<T>, dim3(g), dim3(kThreadsXY), 0, st, a, p.nP, p.xcd);
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

template <typename T>
static hipError_t fwd_t(const DevPlan& p, const Batch& b, void* const* in9, void* spec, hipStream_t st) {
  FwdArgs<T> a;
  a.t = tables<T>(p);
  a.items = p.itemsF;
  a.nfield = 9;
  for (int f = 0; f < 9; ++f) a.in[f] = reinterpret_cast<const T*>(in9[f]);
  a.spec = reinterpret_cast<cx<T>*>(spec);
  a.slab = p.slab;
  a.sbias = b.sbias;
  const int g = grid_for(b.nF, p.grid_cap[kPhaseFwd]);
  if (!g) return hipSuccess;
  hipLaunchKernelGGL(k_fwd_xy<T>, dim3(g), dim3(kThreadsXY), p.ldsF, st, a, b.F0, b.nF, p.xcd);
  return hipGetLastError();
}

hipError_t launch_fwd(const DevPlan& p, const Batch& b, void* const* in9, void* spec, hipStream_t st) {
  return p.f64 ? fwd_t<double>(p, b, in9, spec, st) : fwd_t<float>(p, b, in9, spec, st);
}

template <typename T, int NT, int PB>
static hipError_t upd_launch(const DevPlan& p, const Batch& b, const UpdArgs<T>& a, int g, hipStream_t st) {
  hipLaunchKernelGGL((k_z_update<T, NT, PB, IncOf<T>::value>), dim3(g), dim3(NT), p.ldsU, st, a, b.U0, b.nU, p.xcd);
  return hipGetLastError();
}

template <typename T>
static hipError_t upd_t(const DevPlan& p, const Batch& b, void* spec, hipStream_t st) {
  UpdArgs<T> a;
  a.t = tables<T>(p);
  a.items = p.itemsU;
  a.spec = reinterpret_cast<cx<T>*>(spec);
  a.slab = p.slab;
  a.sbias = b.sbias;
  a.k.c = p.c;
  a.k.dt = p.dt;
  const int g = grid_for(b.nU, p.grid_cap[kPhaseUpd]);
  if (!g) return hipSuccess;
  const bool big = p.NTU == 1024;
  switch (p.PB) {
    case 2: return big ? upd_launch<T, 1024, 2>(p, b, a, g, st) : upd_launch<T, 512, 2>(p, b, a, g, st);
    case 4: return big ? upd_launch<T, 1024, 4>(p, b, a, g, st) : upd_launch<T, 512, 4>(p, b, a, g, st);
    case 8: return big ? upd_launch<T, 1024, 8>(p, b, a, g, st) : upd_launch<T, 512, 8>(p, b, a, g, st);
    case 16: return big ? upd_launch<T, 1024, 16>(p, b, a, g, st) : upd_launch<T, 512, 16>(p, b, a, g, st);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_upd(const DevPlan& p, const Batch& b, void* spec, hipStream_t st) {
  return p.f64 ? upd_t<double>(p, b, spec, st) : upd_t<float>(p, b, spec, st);
}

template <typename T>
static hipError_t inv_t(const DevPlan& p, const Batch& b, const void* spec, void* const* out6, hipStream_t st) {
  InvArgs<T> a;
  a.t = tables<T>(p);
  a.items = p.itemsI;
  a.spec = reinterpret_cast<const cx<T>*>(spec);
  a.slab = p.slab;
  a.sbias = b.sbias;
  for (int f = 0; f < 6; ++f) a.out[f] = reinterpret_cast<T*>(out6[f]);
  const int g = grid_for(b.nI, p.grid_cap[kPhaseInv]);
  if (!g) return hipSuccess;
  hipLaunchKernelGGL((k_inv_xy<T, IncOf<T>::value>), dim3(g), dim3(kThreadsXY), p.ldsI, st, a, b.I0, b.nI, p.xcd);
  return hipGetLastError();
}

hipError_t launch_inv(const DevPlan& p, const Batch& b, const void* spec, void* const* out6, hipStream_t st) {
  return p.f64 ? inv_t<double>(p, b, spec, out6, st) : inv_t<float>(p, b, spec, out6, st);
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
