/*
 * psatd.h -- C-ABI of libpsatd.so, the MI355X (gfx950) local-FFT PSATD field push.
 *
 * Method: H. Vincenti and J.-L. Vay, "Ultrahigh-order Maxwell solver with extreme
 * scalability for electromagnetic PIC simulations of plasmas".
 *   - Sec. 3.1, Eqs. PSATD_1 / PSATD_2: analytic k-space update of E and B over one
 *     time step, with J at the half step held constant over the step;
 *   - Sec. 3.1 (text after the equations): order-p modified wavenumbers
 *     k_u -> sum_{j=1}^{p/2} w_j sin(j k_u du)/(du/2), p -> infinity = exact k;
 *   - Sec. 3.2, Fig. 2a and Fig. 3: the global grid is cut into subdomains padded with
 *     guard cells; each padded subdomain is advanced with its own local FFT as if it
 *     were periodic, then its guard cells are replaced by the neighbours' values.
 *
 * One step, all on the device and in stream order:
 *   exchange_J  -> forward local 3D FFT of E, B, J -> k-space update ->
 *   inverse local 3D FFT of E, B -> exchange_EB.
 *
 * Units: d/dt B = -curl E, d/dt E = c^2 curl B - J (eps0 = 1, mu0 = 1/c^2); at c = 1
 * this is the paper's normalisation.
 *
 * Conventions for every array argument below:
 *   - 3-vectors of sizes are ordered (x, y, z);
 *   - a "field buffer" is ONE device buffer per vector component (E[0..2] = Ex, Ey, Ez,
 *     and likewise B and J).  It holds every subdomain's PADDED box in subdomain order;
 *     box s starts at element offset(s) (see psatd_field_layout) and is stored C-ordered
 *     [z][y][x] (x fastest) with extents n(s) + 2 guard(s).  Consecutive boxes are
 *     separated by a gap of less than 128 bytes, chosen so that each box's first interior
 *     x cell starts a 128-byte line (the kernels never touch the gaps).  The
 *     element type is double for PSATD_F64 and float for every other precision.
 *     Buffers must be 16-byte aligned (torch allocations are).
 *   - a "global buffer" is one device buffer per component holding the interior grid,
 *     C-ordered [z][y][x] with extents grid_n.
 *
 * Ownership: the caller owns every field, global and workspace buffer.  The plan owns
 * its tables, kernels' launch configuration and captured graphs.  E and B are updated
 * in place; J is read, and in PSATD_J_DEPOSITED mode its guard copies are overwritten by
 * the summed currents.
 *
 * Errors: every call returns a psatd_status; no C++ exception crosses this interface and
 * nothing here calls exit or abort.  The message of the last failure is available from
 * psatd_last_error.  Work is enqueued asynchronously on the plan's stream, so a device
 * fault surfaces at the next call that synchronises (psatd_sync).  A plan is not
 * thread-safe; distinct plans are independent.
 */
#ifndef PSATD_H
#define PSATD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct psatd_plan_s* psatd_plan_t;

typedef enum {
  PSATD_OK = 0,
  PSATD_E_INVALID = 1,     /* bad argument: see psatd_last_error */
  PSATD_E_NOMEM = 2,       /* device or host allocation failed */
  PSATD_E_HIP = 3,         /* a HIP runtime call failed */
  PSATD_E_UNSUPPORTED = 4, /* valid but not implemented (e.g. FFT length with a prime > 11) */
  PSATD_E_STATE = 5        /* call not valid in the plan's current state */
} psatd_status;

typedef enum {
  PSATD_F64 = 0,        /* FP64 state, FP64 FFT, FP64 update */
  /* FP32 state and FFT (vector ALU).  The Sec. 3.1 coefficient tables are
     evaluated in FP64; the update's multiply-adds run in FP32 on the
     increments E' - E and B' - B, which the inverse FFT carries back and adds
     to the state. */
  PSATD_F32_VALU = 1,
  /* FP32 state as PSATD_F32_VALU; in addition the first (radix-16) stage of
     every transform whose length is a multiple of 16 is a complex 16x16
     DFT-GEMM on the matrix cores with the FP32 operands split into BF16 terms
     and FP32 accumulation; the other stages run on the vector ALU. */
  PSATD_F32_BF16X3 = 2, /* 2 terms per operand, 3 products (hi*hi + hi*lo + lo*hi) */
  PSATD_F32_BF16X6 = 3  /* 3 terms per operand, the 6 products of term order <= 2 */
} psatd_precision;

typedef enum {
  PSATD_J_REPLICATED = 0, /* every guard copy of J takes the owning subdomain's value */
  PSATD_J_DEPOSITED = 1   /* J of a global cell = sum over all its padded copies, written to every copy */
} psatd_jmode;

/* Phases of one step, in execution order (for psatd_run_profiled). */
enum {
  PSATD_PHASE_EXCHANGE_J = 0,
  PSATD_PHASE_FFT_XY_FWD = 1,  /* R2C along x + C2C along y, per z-plane, 9 fields */
  PSATD_PHASE_Z_UPDATE = 2,    /* C2C along z, Eq. PSATD update, inverse C2C along z */
  PSATD_PHASE_FFT_XY_INV = 3,  /* C2C along y + C2R along x, 6 fields, interior planes */
  PSATD_PHASE_EXCHANGE_EB = 4,
  PSATD_NPHASES = 5
};

/* Launch-shape knobs (psatd_set_tuning).  None changes results beyond rounding order. */
typedef enum {
  PSATD_TUNE_Z_PENCILS = 0,  /* (ky,kx) pencils per z-update work-group: 4, 6, 8, 10 or 16
                                (LDS-limited) for every subdomain.  Default for the longest padded z: FP32
                                the widest of 10, 8 and 6 of which two tiles fit a compute unit, else 4;
                                FP64 8, else 4.  0 (default for unbatched plans whose subdomains differ
                                in that respect): one launch per class of that choice, each with the LDS
                                of its own longest padded z */
  PSATD_TUNE_XCD_REMAP = 1,  /* 1: consecutive work items on the same XCD (shared L2); 0: dispatch order */
  PSATD_TUNE_GRID_FWD = 2,   /* work-groups of the forward x/y pass: 0 = one per item, else a persistent grid */
  PSATD_TUNE_GRID_UPD = 3,   /* same for the z-update pass */
  PSATD_TUNE_GRID_INV = 4,   /* same for the inverse y/x pass */
  PSATD_TUNE_GRID_EXCH = 5,  /* same for the guard exchanges */
  PSATD_TUNE_BATCH_BOXES = 6, /* subdomains pushed through the FFT/update passes together (0 = all);
                                 the workspace then holds one batch's half spectra */
  PSATD_TUNE_MAX_RADIX = 7,   /* largest radix of the x/y passes' FFT schedules: 16, or 8 (fewer
                                 registers, more stages); radix 11 is always allowed.  Default 16, and 8
                                 for FP64 plans whose planes fit the LDS */
  PSATD_TUNE_XY_THREADS = 8,  /* threads per work-group of the x/y passes: 256, 512 or 1024 for every
                                 subdomain; 0 (default for unbatched plans whose subdomains differ in how
                                 many padded planes fit a compute unit's LDS): one launch per such class,
                                 each with the fewest threads that keep 16 waves per compute unit and the
                                 LDS of its own largest plane */
  PSATD_TUNE_Z_THREADS = 9,   /* threads per work-group of the z-update: 512 or 1024 */
  PSATD_TUNE_SPLIT_XY = 10,   /* 1: x rows and y columns in separate passes through the workspace
                                 (automatic when a padded plane exceeds the LDS; needs no batching) */
  PSATD_TUNE_FUSE_EB = 11,    /* 1: the inverse pass writes each new E, B value into every guard copy
                                 of its cell, so the E,B exchange needs no pass of its own (same bytes
                                 as the copy pass); 0 (default, faster on 96^3 boxes): a separate copy
                                 pass.  Batching (PSATD_TUNE_BATCH_BOXES) turns it off. */
  PSATD_TUNE_Z_REG = 12,      /* 1: the FP32 VALU z pass holds each z transform in registers (compiled
                                 padded z lengths only, unbatched plans); 0 (default, faster on 96^3 and
                                 176^3 boxes): the LDS-staged z pass */
  PSATD_TUNE_PULL_EB = 13,    /* 1 (default for unbatched plans whose planes fit the LDS): within a run the
                                 forward pass reads every E, B guard cell from the subdomain that owns it,
                                 so the E,B guard exchange runs once, after the run's last step (the state
                                 is consistent again on return, and every value is the one the exchange
                                 would have copied); 0: the exchange after every step */
  PSATD_TUNE_MAX_RADIX_Z = 14, /* the same for the z pass's schedules; default 16 */
  PSATD_NTUNE = 15
} psatd_tune_key;

/*
 * psatd_plan -- build a plan (Sec. 3.2 decomposition, Sec. 3.1 operator).
 *   grid_n[3]   global periodic interior cells (Nx, Ny, Nz), each >= 1
 *   grid_d[3]   cell sizes (dx, dy, dz) > 0
 *   nsub        number of subdomains >= 1
 *   lo[nsub*3]  first owned global cell of each subdomain, (x, y, z)
 *   n[nsub*3]   owned cells of each subdomain, (x, y, z); the boxes must tile the grid
 *               exactly (no overlap, no gap)
 *   guard[nsub*3] guard cells on each side, per subdomain and axis, >= 0; a guard may
 *               exceed the neighbour's size or the grid (owners are found modulo N)
 *   order_p     even >= 2 (finite-difference order of the modified wavenumber) or 0 for
 *               infinite order (exact k)
 *   dt          time step, any sign, nonzero and finite
 *   c           speed of light > 0
 *   precision   psatd_precision
 *   jmode       psatd_jmode
 *   stream      hipStream_t on which all work is enqueued (NULL = default stream)
 * Padded lengths must have prime factors <= 11 and the padded x length must be even;
 * otherwise PSATD_E_UNSUPPORTED.  Uses the current HIP device.
 * On success *out receives the plan; on failure *out is NULL.
 */
psatd_status psatd_plan(psatd_plan_t* out, const int64_t grid_n[3], const double grid_d[3],
                        int32_t nsub, const int64_t* lo, const int64_t* n, const int32_t* guard,
                        int32_t order_p, double dt, double c, int32_t precision, int32_t jmode,
                        void* stream);

/*
 * psatd_validate -- the host-side checks of psatd_plan without touching the device.
 * Same arguments (no stream).  On PSATD_OK, *field_elems (if not NULL) receives the
 * number of elements of one field buffer.  Usable without a GPU.
 */
psatd_status psatd_validate(const int64_t grid_n[3], const double grid_d[3], int32_t nsub,
                            const int64_t* lo, const int64_t* n, const int32_t* guard,
                            int32_t order_p, double dt, double c, int32_t precision,
                            int32_t jmode, int64_t* field_elems);

/* Elements of one field buffer: the padded volumes of all subdomains plus the alignment
 * gaps between them (the last box ends the buffer). */
psatd_status psatd_field_elems(psatd_plan_t plan, int64_t* total);

/* Padded extents (x, y, z) of subdomain s and its element offset in a field buffer. */
psatd_status psatd_field_layout(psatd_plan_t plan, int32_t s, int64_t padded_n[3],
                                int64_t* offset_elems);

/*
 * Workspace: device scratch for the half-spectrum intermediates.  psatd_workspace_bytes
 * gives the size; psatd_set_workspace hands the plan caller-owned device memory (at
 * least that many bytes, 256-byte aligned; NULL/0 returns to plan-owned memory, which
 * the plan allocates at the first step).  The caller keeps the memory alive while the
 * plan uses it.
 */
psatd_status psatd_workspace_bytes(psatd_plan_t plan, int64_t* bytes);
psatd_status psatd_set_workspace(psatd_plan_t plan, void* dev, int64_t bytes);

/*
 * psatd_step -- one step of the domain-decomposed method of Sec. 3.2 (the three
 * steps of Fig. 3: currents made consistent over the guard copies, every padded
 * box advanced by its own local FFT push of Sec. 3.1, guard cells of E and B
 * replaced by the owners' values), enqueued on the plan's stream.  E, B, J: arrays of 3 device field buffers.  The
 * state must be consistent on entry (every guard copy equal to its owner, as
 * psatd_scatter leaves it); it is consistent again on exit.  In PSATD_J_DEPOSITED mode
 * every call takes J as freshly deposited partial currents and sums them (after the
 * call J holds the summed, consistent currents).
 */
psatd_status psatd_step(psatd_plan_t plan, void* const E[3], void* const B[3], void* const J[3]);

/*
 * psatd_step_noalloc -- psatd_step for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid allocation): the
 * same step and results, with the spectral workspace taken from a static device array of
 * PSATD_NOALLOC_SCRATCH_BYTES bytes that the library holds on every GPU it runs on until
 * the process ends, instead of the plan's or the caller's workspace.  It calls no
 * allocating routine.  Returns PSATD_E_INVALID (nothing enqueued) when
 * psatd_workspace_bytes exceeds that size: batching the boxes (PSATD_TUNE_BATCH_BOXES)
 * shrinks the workspace to one batch.  Every call on a GPU shares that GPU's array
 * (nothing in it needs to start at zero; it keeps the last call's contents), so calls
 * that overlap in time on one GPU, from any plans or streams, race and must be ordered
 * by the caller.
 */
#define PSATD_NOALLOC_SCRATCH_BYTES (64ll << 20)
psatd_status psatd_step_noalloc(psatd_plan_t plan, void* const E[3], void* const B[3],
                                void* const J[3]);

/*
 * psatd_run -- nsteps >= 0 steps of Sec. 3.2 / Fig. 3 with J unchanged, replayed from a
 * captured HIP graph
 * (captured once per (buffers, nsteps) and cached in the plan).  J is exchanged once, at
 * the first step (summed in PSATD_J_DEPOSITED mode, filled from the owners in
 * PSATD_J_REPLICATED mode), and then held: the step never writes J, so the later steps
 * find it consistent.
 */
psatd_status psatd_run(psatd_plan_t plan, void* const E[3], void* const B[3], void* const J[3],
                       int32_t nsteps);

/*
 * psatd_heat_run -- nsteps >= 0 steps of the same local-FFT method applied to the
 * diffusion equation du/dt = D lap u (Sec. 5 names it among the initial-value problems
 * the method extends to): every padded box advanced by its exact propagator
 * u <- IFFT(exp(-D |[k]|^2 dt) FFT(u)), with the plan's order-p modified wavenumbers
 * (Sec. 3.1) and dt, then every guard copy of u takes its owner's value (Fig. 3).
 *   u            ONE device buffer of psatd_field_elems elements in the plan's layout and
 *                dtype (the F32 forms: float, the propagator applied to the increment),
 *                consistent on entry (psatd_scatter of a component does that) and on exit
 *   diffusivity  D >= 0, finite
 * Enqueued on the plan's stream (no graph).  Uses the plan's workspace.  Errors:
 * PSATD_E_UNSUPPORTED when the padded planes need the split x/y passes; PSATD_E_STATE
 * when the plan is batched (PSATD_TUNE_BATCH_BOXES).
 */
psatd_status psatd_heat_run(psatd_plan_t plan, void* u, double diffusivity, int32_t nsteps);

/*
 * psatd_run_profiled -- nsteps >= 1 steps with psatd_run semantics (J exchanged at the
 * first step only: summed in PSATD_J_DEPOSITED mode, owner-copied in
 * PSATD_J_REPLICATED mode, then held), launched directly with a HIP event pair around
 * every kernel launch; waits for completion and writes the mean milliseconds per step
 * of each phase to phase_ms[PSATD_NPHASES] (host array; the J exchange's time is
 * averaged over the nsteps steps).
 */
psatd_status psatd_run_profiled(psatd_plan_t plan, void* const E[3], void* const B[3],
                                void* const J[3], int32_t nsteps, double* phase_ms);

/*
 * psatd_scatter -- Fig. 3 step 1: global[3] (interior grid) -> padded[3] field buffers,
 * every padded cell (guards included) taking the value at its global index modulo the
 * grid (a consistent state).  psatd_gather -- padded interiors -> global[3] (each cell
 * from the subdomain that owns it).  Exact copies; the global buffers hold
 * grid_n[0] * grid_n[1] * grid_n[2] elements of the plan's element type.
 */
psatd_status psatd_scatter(psatd_plan_t plan, const void* const global[3], void* const padded[3]);
psatd_status psatd_gather(psatd_plan_t plan, const void* const padded[3], void* const global[3]);

/*
 * psatd_modified_k -- copies the plan's FP64 modified-wavenumber table of axis u
 * (0 = x, 1 = y, 2 = z) for subdomain s into host memory out[len] (len = padded length
 * of that axis), over the FFT index m = 0..len-1 (Sec. 3.1).
 */
psatd_status psatd_modified_k(psatd_plan_t plan, int32_t s, int32_t axis, double* out,
                              int64_t len);

/*
 * psatd_set_tuning / psatd_get_tuning -- launch-shape knobs (psatd_tune_key).  Setting a
 * value the plan cannot use (e.g. a z tile that does not fit the LDS) returns
 * PSATD_E_INVALID and leaves the plan unchanged.  Cached graphs are dropped.
 */
psatd_status psatd_set_tuning(psatd_plan_t plan, int32_t key, int32_t value);
psatd_status psatd_get_tuning(psatd_plan_t plan, int32_t key, int32_t* value);

/*
 * psatd_autotune -- picks the launch shapes (largest radix, x/y threads, z tile and threads,
 * XCD item order) by timing candidate settings with steps_per_trial >= 1 steps each on the
 * given buffers, phase by phase, and applies the fastest.  When it times (no cache hit), J is
 * first exchanged once as psatd_step does (summed in PSATD_J_DEPOSITED mode) and then left
 * alone by every trial; the trial steps advance E and B (tune before loading the state
 * that matters).  cache_path (may be NULL): a text file of
 * "key value..." lines; a hit applies the cached setting without timing, a miss appends the
 * new result.  The key holds the device name, the precision and the padded box shapes.
 * *best_ms (may be NULL) receives the tuned step time in milliseconds (0 on a cache hit).
 */
psatd_status psatd_autotune(psatd_plan_t plan, void* const E[3], void* const B[3], void* const J[3],
                            int32_t steps_per_trial, const char* cache_path, double* best_ms);

psatd_status psatd_set_stream(psatd_plan_t plan, void* stream);
psatd_status psatd_sync(psatd_plan_t plan); /* waits for the plan's stream */
void psatd_destroy(psatd_plan_t plan);       /* NULL-safe */

const char* psatd_status_string(psatd_status st);
/* Message of the last failure on this plan; plan == NULL gives the calling thread's last
 * failure of psatd_plan / psatd_validate.  Never NULL. */
const char* psatd_last_error(psatd_plan_t plan);
/* Library version, "major.minor.patch". */
const char* psatd_version(void);

#ifdef __cplusplus
}
#endif
#endif /* PSATD_H */
