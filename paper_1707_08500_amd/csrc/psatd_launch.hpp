// Device-side view of a plan and the launchers of every phase of the step.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "psatd_device.hpp"

namespace psatd {

enum Phase { kPhaseExchJ = 0, kPhaseFwd = 1, kPhaseUpd = 2, kPhaseInv = 3, kPhaseExchEB = 4, kNumPhases = 5 };

struct DevPlan {
  bool f64;                 // element type: double (true) or float
  int32_t nsub;
  int32_t N[3];
  const BoxD* box;
  const FftPlanD* plans;
  const void* tw;           // cx<double> or cx<float> twiddles
  const double* kmod;
  const int32_t* nbr_off;
  const int32_t* nbr;
  const int32_t* itemsF;    // P[2] * 9
  const int32_t* itemsU;    // ceil(P[1] H / PB)
  const int32_t* itemsI;    // n[2] * 6
  const int32_t* itemsP;    // P[2]
  const int32_t* itemsN;    // n[2]
  const int32_t* itemsXF;   // split passes: x forward, y forward, y inverse, x inverse
  const int32_t* itemsYF;
  const int32_t* itemsYI;
  const int32_t* itemsXI;
  int32_t nXF, nYF, nYI, nXI;
  int32_t ldsX, ldsY;
  int32_t split;
  const PushBlk* push;       // guard pieces (guard fill, fused E,B exchange)
  const FillPiece* fillp;    // guard fill: pieces with offsets and pitches
  const int32_t* itemsG;     // guard fill: prefix over pieces of their z extent
  const int32_t* pieceOf;    // guard fill: item -> piece
  int32_t npiece, nG;
  const int32_t* push_off;
  int32_t fuse;              // 1: the inverse pass writes the E,B guard copies
  int32_t spl;               // BF16 terms of the matrix-core DFT stage (0: VALU only)
  int32_t nF, nU, nI, nP, nN;
  int32_t ldsF, ldsI, ldsU;  // dynamic LDS bytes per work-group
  int32_t ldsH;              // heat z pass: one staged field
  int32_t PB;                // pencils per z-update work-group (one size for every box)
  int32_t zcl;               // 1: one z launch per class of tile size (below)
  int32_t nzc;
  ZClass zc[kMaxZClasses];
  const int32_t* itemsZC;
  int32_t ntu;               // threads per z-update work-group (512 or 1024)
  int32_t ntxy;              // threads per x/y work-group (256, 512 or 1024; 0: per launch class)
  int32_t nxyc;              // x/y launch classes (used when ntxy == 0)
  XyClass xyc[kMaxXyClasses];
  const int32_t* itemsXYC;
  int32_t maxr;              // largest codelet of the x/y schedules (8 or 16)
  int32_t maxrz;             // largest codelet of the z schedules
  int32_t xcd;               // 1: consecutive items on the same XCD (L2 sharing)
  int64_t slab;              // complex elements of one spectral field slab
  double c, dt;
  int32_t grid_cap[kNumPhases];  // 0: one work-group per item; else persistent grid
  int32_t pull;                  // 1: the forward pass pulls E,B guard cells from their owners
  const PullPiece* pullp;
  const int32_t* pull_off;
  int32_t zreg;                  // 1: the z pass runs the register kernels (groups below)
  int32_t nzg;
  ZGroup zg[kMaxZGroups];
  const int32_t* itemsZR;
};

hipError_t launch_fill(const DevPlan& p, void* const* comps, int ncomp, hipStream_t st);
hipError_t launch_sum(const DevPlan& p, void* const* J, hipStream_t st);
hipError_t launch_fwd(const DevPlan& p, const Batch& b, void* const* in9, void* spec, hipStream_t st,
                      bool scalar = false);
hipError_t launch_upd(const DevPlan& p, const Batch& b, void* spec, hipStream_t st);
// the z pass with the z transforms in registers (all boxes, FP32 VALU form)
hipError_t launch_upd_reg(const DevPlan& p, void* spec, hipStream_t st);
hipError_t launch_inv(const DevPlan& p, const Batch& b, const void* spec, void* const* out6, hipStream_t st,
                      bool scalar = false);
// heat equation (Sec. 5): z pass of one field with the exp(-D |[k]|^2 dt) propagator
hipError_t launch_heat_z(const DevPlan& p, void* spec, double D, double dt, hipStream_t st);
// split x/y passes (whole plan, no batching)
hipError_t launch_x_fwd(const DevPlan& p, void* const* in9, void* spec, hipStream_t st);
hipError_t launch_y(const DevPlan& p, int dir, void* spec, hipStream_t st);
hipError_t launch_x_inv(const DevPlan& p, const void* spec, void* const* out6, hipStream_t st);
hipError_t launch_scatter(const DevPlan& p, const void* const* glob, void* const* pad, hipStream_t st);
hipError_t launch_gather(const DevPlan& p, const void* const* pad, void* const* glob, hipStream_t st);
hipError_t launch_modk(const KEntry* entries, int nent, int maxN, int order_p, double* kmod,
                       hipStream_t st);
hipError_t prepare_kernels(bool f64, int spl, int ldsF, int ldsI, int ldsU, int ldsX, int ldsY);


}  // namespace psatd
