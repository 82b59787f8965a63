"""C-ABI checks that need no GPU: the library loads, exports every symbol that
include/psatd.h declares, and the host-side validation accepts and rejects
plans as documented."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1707_08500_amd import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "psatd.h")


def declared_symbols():
    src = open(HEADER).read()
    return sorted(set(re.findall(r"\b(psatd_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    from paper_1707_08500_amd import psatd
    lib = ctypes.CDLL(psatd.LIB_PATH)
    names = declared_symbols()
    assert len(names) >= 18
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(psatd.SYMBOLS)
    assert psatd.LIB.psatd_version().decode().count(".") == 2


def test_status_strings():
    from paper_1707_08500_amd import psatd
    for code, name in psatd.STATUS.items():
        assert psatd.LIB.psatd_status_string(code).decode() == name


def good_case():
    lo, n, g = synth.uniform_decomposition((256, 256, 256), (4, 4, 4), 16)
    return dict(grid_n=(256, 256, 256), grid_d=(1.0, 1.0, 1.0), lo=lo, n=n, guard=g,
                order_p=32, dt=0.5, c=1.0)


def test_validate_accepts_config2_layout():
    from paper_1707_08500_amd import psatd
    # boxes back to back except for the gap (< one 128-byte line) that starts
    # each box's first interior x cell on a line: none in FP64 with 16 guards
    # (16 doubles = one line), 16 floats before the first box in FP32
    elems = psatd.validate(**good_case())
    assert elems == 64 * 96 ** 3
    elems32 = psatd.validate(**good_case(), precision="f32")
    assert elems32 == elems + 16


def test_validate_uneven_decomposition():
    from paper_1707_08500_amd import psatd
    lo, n, g = synth.uneven_decomposition((512, 512, 256), case=4)
    elems = psatd.validate((512, 512, 256), (1.0, 1.0, 1.0), lo, n, g, 64, 0.5, precision="f32")
    vol = int(np.prod(n + 2 * g, axis=1).sum())
    assert vol <= elems < vol + 32 * len(n)


@pytest.mark.parametrize("mutate,status", [
    (lambda c: c.update(order_p=3), "PSATD_E_INVALID"),
    (lambda c: c.update(order_p=-2), "PSATD_E_INVALID"),
    (lambda c: c.update(dt=0.0), "PSATD_E_INVALID"),
    (lambda c: c.update(dt=float("nan")), "PSATD_E_INVALID"),
    (lambda c: c.update(c=0.0), "PSATD_E_INVALID"),
    (lambda c: c.update(c=-1.0), "PSATD_E_INVALID"),
    (lambda c: c.update(grid_d=(1.0, 0.0, 1.0)), "PSATD_E_INVALID"),
    (lambda c: c["guard"].__setitem__((3, 1), -1), "PSATD_E_INVALID"),
    (lambda c: c["n"].__setitem__((5, 0), 32), "PSATD_E_INVALID"),      # gap
    (lambda c: c["lo"].__setitem__((5, 0), 32), "PSATD_E_INVALID"),     # overlap
    (lambda c: c["lo"].__setitem__((63, 2), 250), "PSATD_E_INVALID"),   # outside
    (lambda c: c["guard"].__setitem__((0, 2), 19), "PSATD_E_UNSUPPORTED"),  # 64 + 38 = 102 = 2 3 17
])
def test_validate_rejects(mutate, status):
    from paper_1707_08500_amd import psatd
    case = good_case()
    case["lo"] = case["lo"].copy()
    case["n"] = case["n"].copy()
    case["guard"] = case["guard"].copy()
    mutate(case)
    with pytest.raises(psatd.PsatdError) as ei:
        psatd.validate(**case)
    assert psatd.STATUS[ei.value.status] == status
    assert len(str(ei.value)) > len(status) + 2


def test_validate_prime_factor_and_parity():
    from paper_1707_08500_amd import psatd
    # padded length 13 (prime > 11)
    with pytest.raises(psatd.PsatdError) as ei:
        psatd.validate((26, 26, 26), (1, 1, 1), [[0, 0, 0]], [[26, 26, 26]], [[0, 0, 0]], 0, 0.5)
    assert ei.value.status == 4
    # odd padded x length
    with pytest.raises(psatd.PsatdError) as ei:
        psatd.validate((9, 8, 8), (1, 1, 1), [[0, 0, 0]], [[9, 8, 8]], [[0, 0, 0]], 0, 0.5)
    assert ei.value.status == 4
    # the split-BF16 forms plan like FP32 (FP32 buffers); an unknown form is rejected
    for form in ("bf16x3", "bf16x6"):
        assert psatd.validate((32, 32, 32), (1, 1, 1), [[0, 0, 0]], [[32, 32, 32]], [[0, 0, 0]], 0,
                              0.5, precision=form) == 32 ** 3
    gn = (ctypes.c_int64 * 3)(8, 8, 8)
    gd = (ctypes.c_double * 3)(1.0, 1.0, 1.0)
    lo = (ctypes.c_int64 * 3)(0, 0, 0)
    nn = (ctypes.c_int64 * 3)(8, 8, 8)
    gg = (ctypes.c_int32 * 3)(0, 0, 0)
    out = ctypes.c_int64(0)
    assert psatd.LIB.psatd_validate(gn, gd, 1, lo, nn, gg, 0, 0.5, 1.0, 7, 0, ctypes.byref(out)) == 1


def test_null_and_bad_plan_calls_are_errors_not_crashes():
    from paper_1707_08500_amd import psatd
    L = psatd.LIB
    assert L.psatd_field_elems(None, None) == 1
    assert L.psatd_sync(None) == 1
    L.psatd_destroy(None)  # NULL-safe
    assert isinstance(L.psatd_last_error(None), bytes)
    out = ctypes.c_void_p()
    gn = (ctypes.c_int64 * 3)(8, 8, 8)
    gd = (ctypes.c_double * 3)(1, 1, 1)
    st = L.psatd_plan(ctypes.byref(out), gn, gd, 0, None, None, None, 0, 0.5, 1.0, 0, 0, None)
    assert st == 1 and not out.value


class _FakeCuda:
    """Stands in for a CUDA tensor on a machine without a GPU: only the
    attributes the binding's buffer check reads."""

    def __init__(self, dtype, numel, device="cuda:0", contiguous=True):
        import torch
        self.is_cuda = True
        self.dtype = dtype
        self.device = torch.device(device)
        self._n = numel
        self._c = contiguous

    def numel(self):
        return self._n

    def is_contiguous(self):
        return self._c


def test_binding_rejects_mismatched_buffers_before_the_abi():
    """The C-ABI takes bare device pointers, so the binding checks every
    tensor first: a host tensor, another device, the wrong dtype (FP32 data
    for an FP64 plan), a strided view, or a buffer of the wrong length (e.g.
    global and padded buffers swapped) is a ValueError, never a launch."""
    import torch
    from paper_1707_08500_amd import psatd
    dev = torch.device("cuda:0")
    ok = _FakeCuda(torch.float64, 1000)
    psatd.check_buffer(ok, torch.float64, 1000, dev, "E[0]")
    cases = [
        (torch.zeros(1000, dtype=torch.float64), "not a CUDA tensor"),
        (_FakeCuda(torch.float64, 1000, device="cuda:1"), "the plan runs on"),
        (_FakeCuda(torch.float32, 1000), "the plan needs torch.float64"),
        (_FakeCuda(torch.float64, 1000, contiguous=False), "not contiguous"),
        (_FakeCuda(torch.float64, 512), "elements, the plan needs 1000"),
    ]
    for t, msg in cases:
        with pytest.raises(ValueError, match=msg):
            psatd.check_buffer(t, torch.float64, 1000, dev, "E[0]")
    with pytest.raises(ValueError, match="need 3 component buffers"):
        psatd._ptrs([ok, ok], torch.float64, 1000, dev, "E")
    with pytest.raises(ValueError, match=r"B\[2\]"):
        psatd._ptrs([ok, ok, _FakeCuda(torch.float64, 999)], torch.float64, 1000, dev, "B")
