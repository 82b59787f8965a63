"""Python binding of libpsatd.so (ctypes).

Argument marshalling only: every step of the field push runs in the HIP
library.  PyTorch supplies device memory (``tensor.data_ptr()``) and the stream
(``torch.cuda.current_stream().cuda_stream``).  If the library is missing the
import of this module raises; there is no fallback.

Names follow the C-ABI in include/psatd.h.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libpsatd.so")

F64, F32_VALU, F32_BF16X3, F32_BF16X6 = 0, 1, 2, 3
J_REPLICATED, J_DEPOSITED = 0, 1
PRECISIONS = {"f64": F64, "f32": F32_VALU, "f32_valu": F32_VALU,
              "bf16x3": F32_BF16X3, "bf16x6": F32_BF16X6}
JMODES = {"replicated": J_REPLICATED, "deposited": J_DEPOSITED}
PHASES = ("exchange_J", "fft_xy_fwd", "z_update", "fft_xy_inv", "exchange_EB")
TUNING = {"z_pencils": 0, "xcd_remap": 1, "grid_fwd": 2, "grid_upd": 3, "grid_inv": 4,
          "grid_exch": 5, "batch_boxes": 6, "max_radix": 7, "xy_threads": 8, "z_threads": 9,
          "split_xy": 10, "fuse_eb": 11, "z_reg": 12, "pull_eb": 13,
          "max_radix_z": 14}
NPHASES = len(PHASES)
NOALLOC_SCRATCH_BYTES = 64 << 20  # PSATD_NOALLOC_SCRATCH_BYTES

STATUS = {0: "PSATD_OK", 1: "PSATD_E_INVALID", 2: "PSATD_E_NOMEM", 3: "PSATD_E_HIP",
          4: "PSATD_E_UNSUPPORTED", 5: "PSATD_E_STATE"}

SYMBOLS = ("psatd_plan", "psatd_validate", "psatd_field_elems", "psatd_field_layout",
           "psatd_workspace_bytes", "psatd_set_workspace", "psatd_step", "psatd_step_noalloc", "psatd_run", "psatd_heat_run",
           "psatd_run_profiled", "psatd_scatter", "psatd_gather", "psatd_modified_k",
           "psatd_set_tuning", "psatd_get_tuning", "psatd_autotune", "psatd_set_stream", "psatd_sync", "psatd_destroy", "psatd_status_string",
           "psatd_last_error", "psatd_version")


class PsatdError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1707_08500_amd.build`")
    # torch first: its HIP runtime is then the one the library binds to, so
    # the process holds a single runtime (loaded the other way round, the
    # library's own runtime came up without a device next to torch's)
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
    I64P = ctypes.POINTER(ctypes.c_int64)
    I32P = ctypes.POINTER(ctypes.c_int32)
    DP = ctypes.POINTER(ctypes.c_double)
    VPP = ctypes.POINTER(ctypes.c_void_p)
    sig = {
        "psatd_plan": ([ctypes.POINTER(P), I64P, DP, i32, I64P, I64P, I32P, i32, f64, f64, i32, i32, P], i32),
        "psatd_validate": ([I64P, DP, i32, I64P, I64P, I32P, i32, f64, f64, i32, i32, I64P], i32),
        "psatd_field_elems": ([P, I64P], i32),
        "psatd_field_layout": ([P, i32, I64P, I64P], i32),
        "psatd_workspace_bytes": ([P, I64P], i32),
        "psatd_set_workspace": ([P, P, i64], i32),
        "psatd_step": ([P, VPP, VPP, VPP], i32),
        "psatd_step_noalloc": ([P, VPP, VPP, VPP], i32),
        "psatd_run": ([P, VPP, VPP, VPP, i32], i32),
        "psatd_run_profiled": ([P, VPP, VPP, VPP, i32, DP], i32),
        "psatd_heat_run": ([P, P, f64, i32], i32),
        "psatd_scatter": ([P, VPP, VPP], i32),
        "psatd_gather": ([P, VPP, VPP], i32),
        "psatd_modified_k": ([P, i32, i32, DP, i64], i32),
        "psatd_set_tuning": ([P, i32, i32], i32),
        "psatd_get_tuning": ([P, i32, I32P], i32),
        "psatd_autotune": ([P, VPP, VPP, VPP, i32, ctypes.c_char_p, DP], i32),
        "psatd_set_stream": ([P, P], i32),
        "psatd_sync": ([P], i32),
        "psatd_destroy": ([P], None),
        "psatd_status_string": ([i32], ctypes.c_char_p),
        "psatd_last_error": ([P], ctypes.c_char_p),
        "psatd_version": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    return lib


LIB = _load()


def _check(st, plan=None):
    if st != 0:
        msg = LIB.psatd_last_error(plan).decode()
        raise PsatdError(st, msg)


def _arrays(grid_n, grid_d, lo, n, guard):
    gn = (ctypes.c_int64 * 3)(*[int(v) for v in grid_n])
    gd = (ctypes.c_double * 3)(*[float(v) for v in grid_d])
    lo = np.ascontiguousarray(lo, dtype=np.int64).reshape(-1, 3)
    n = np.ascontiguousarray(n, dtype=np.int64).reshape(-1, 3)
    guard = np.ascontiguousarray(guard, dtype=np.int32).reshape(-1, 3)
    if not (lo.shape == n.shape == guard.shape):
        raise ValueError("lo, n, guard must all be (nsub, 3)")
    return gn, gd, lo, n, guard


def validate(grid_n, grid_d, lo, n, guard, order_p, dt, c=1.0, precision="f64",
             jmode="replicated"):
    """Host-side plan checks (no device).  Returns the field-buffer element count."""
    gn, gd, lo, n, guard = _arrays(grid_n, grid_d, lo, n, guard)
    out = ctypes.c_int64(0)
    st = LIB.psatd_validate(gn, gd, lo.shape[0],
                            lo.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                            n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                            guard.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                            int(order_p), float(dt), float(c), PRECISIONS[precision],
                            JMODES[jmode], ctypes.byref(out))
    _check(st)
    return out.value


def check_buffer(t, dtype, numel, device, what):
    """Raises ValueError unless tensor t is a contiguous CUDA tensor of the
    given dtype, element count (None: any) and device: the C-ABI takes bare
    device pointers and cannot check any of these itself."""
    if not getattr(t, "is_cuda", False):
        raise ValueError(f"{what}: not a CUDA tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{what}: on {t.device}, the plan runs on {device}")
    if t.dtype != dtype:
        raise ValueError(f"{what}: dtype {t.dtype}, the plan needs {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{what}: not contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{what}: {t.numel()} elements, the plan needs {numel}")


def _ptrs(tensors, dtype=None, numel=None, device=None, what="buffers"):
    if len(tensors) != 3:
        raise ValueError(f"{what}: need 3 component buffers")
    if dtype is not None:
        for i, t in enumerate(tensors):
            check_buffer(t, dtype, numel, device, f"{what}[{i}]")
    return (ctypes.c_void_p * 3)(*[t.data_ptr() for t in tensors])


class Plan:
    """psatd_plan(grid, decomposition, guard cells, order p, dt, c) and the calls on it."""

    def __init__(self, grid_n, grid_d, lo, n, guard, order_p, dt, c=1.0, precision="f64",
                 jmode="replicated", stream=None):
        import torch
        gn, gd, lo, n, guard = _arrays(grid_n, grid_d, lo, n, guard)
        if stream is None:
            stream = torch.cuda.current_stream().cuda_stream
        self.precision = precision
        self.dtype = torch.float64 if precision == "f64" else torch.float32
        self.nsub = lo.shape[0]
        self.grid_n = tuple(int(v) for v in grid_n)
        h = ctypes.c_void_p()
        st = LIB.psatd_plan(ctypes.byref(h), gn, gd, self.nsub,
                            lo.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                            n.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                            guard.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                            int(order_p), float(dt), float(c), PRECISIONS[precision],
                            JMODES[jmode], ctypes.c_void_p(stream))
        _check(st)
        self._h = h
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.global_elems = self.grid_n[0] * self.grid_n[1] * self.grid_n[2]
        e = ctypes.c_int64(0)
        _check(LIB.psatd_field_elems(self._h, ctypes.byref(e)), self._h)
        self.field_elems = e.value

    # -- layout
    def layout(self, s):
        pn = (ctypes.c_int64 * 3)()
        off = ctypes.c_int64(0)
        _check(LIB.psatd_field_layout(self._h, int(s), pn, ctypes.byref(off)), self._h)
        return tuple(pn), off.value

    def workspace_bytes(self):
        b = ctypes.c_int64(0)
        _check(LIB.psatd_workspace_bytes(self._h, ctypes.byref(b)), self._h)
        return b.value

    def set_workspace(self, tensor):
        if tensor is None:
            _check(LIB.psatd_set_workspace(self._h, None, 0), self._h)
        else:
            check_buffer(tensor, tensor.dtype, None, self.device, "workspace")
            _check(LIB.psatd_set_workspace(self._h, ctypes.c_void_p(tensor.data_ptr()),
                                           tensor.numel() * tensor.element_size()), self._h)

    def _fields(self, tensors, what):
        return _ptrs(tensors, self.dtype, self.field_elems, self.device, what)

    def _globals(self, tensors, what):
        return _ptrs(tensors, self.dtype, self.global_elems, self.device, what)

    def empty_fields(self, device="cuda"):
        import torch
        return [torch.zeros(self.field_elems, dtype=self.dtype, device=device) for _ in range(3)]

    # -- the step
    def step(self, E, B, J):
        _check(LIB.psatd_step(self._h, self._fields(E, "E"), self._fields(B, "B"), self._fields(J, "J")),
               self._h)

    def step_noalloc(self, E, B, J):
        """psatd_step_noalloc: one step with the library's static device scratch as the
        workspace (no allocation anywhere in the call)."""
        _check(LIB.psatd_step_noalloc(self._h, self._fields(E, "E"), self._fields(B, "B"),
                                      self._fields(J, "J")), self._h)

    def run(self, E, B, J, nsteps):
        _check(LIB.psatd_run(self._h, self._fields(E, "E"), self._fields(B, "B"), self._fields(J, "J"),
                             int(nsteps)), self._h)

    def heat_run(self, u, diffusivity, nsteps):
        """psatd_heat_run: nsteps heat-equation steps of one padded field buffer."""
        check_buffer(u, self.dtype, self.field_elems, self.device, "u")
        _check(LIB.psatd_heat_run(self._h, ctypes.c_void_p(u.data_ptr()), float(diffusivity),
                                  int(nsteps)), self._h)

    def run_profiled(self, E, B, J, nsteps):
        out = (ctypes.c_double * NPHASES)()
        _check(LIB.psatd_run_profiled(self._h, self._fields(E, "E"), self._fields(B, "B"),
                                      self._fields(J, "J"), int(nsteps), out), self._h)
        return dict(zip(PHASES, list(out)))

    def scatter(self, glob, padded):
        _check(LIB.psatd_scatter(self._h, self._globals(glob, "global"), self._fields(padded, "padded")),
               self._h)

    def gather(self, padded, glob):
        _check(LIB.psatd_gather(self._h, self._fields(padded, "padded"), self._globals(glob, "global")),
               self._h)

    def modified_k(self, s, axis):
        pn, _ = self.layout(s)
        out = np.zeros(pn[axis], dtype=np.float64)
        _check(LIB.psatd_modified_k(self._h, int(s), int(axis),
                                    out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                    int(pn[axis])), self._h)
        return out

    def set_tuning(self, **kw):
        for k, v in kw.items():
            _check(LIB.psatd_set_tuning(self._h, TUNING[k], int(v)), self._h)

    def tuning(self):
        out = {}
        for k, key in TUNING.items():
            v = ctypes.c_int32(0)
            _check(LIB.psatd_get_tuning(self._h, key, ctypes.byref(v)), self._h)
            out[k] = v.value
        return out

    def autotune(self, E, B, J, steps_per_trial=3, cache_path=None):
        """Times launch-shape candidates (advancing E, B) and applies the fastest;
        returns the tuned step time in ms (0.0 on a cache hit)."""
        out = ctypes.c_double(0.0)
        cp = cache_path.encode() if cache_path else None
        _check(LIB.psatd_autotune(self._h, self._fields(E, "E"), self._fields(B, "B"), self._fields(J, "J"),
                                  int(steps_per_trial), cp, ctypes.byref(out)), self._h)
        return out.value

    def set_stream(self, stream):
        _check(LIB.psatd_set_stream(self._h, ctypes.c_void_p(stream)), self._h)

    def sync(self):
        _check(LIB.psatd_sync(self._h), self._h)

    def close(self):
        if getattr(self, "_h", None):
            LIB.psatd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- host helpers (views of the padded layout, no arithmetic)
    def box_view(self, buf, s):
        """View of subdomain s inside a 1-D field buffer as [z][y][x]."""
        (px, py, pz), off = self.layout(s)
        return buf[off:off + px * py * pz].view(pz, py, px)
