"""CPU: the algorithmic bytes bench.py divides by the measured kernel time
(roofline.achieved), checked against a count made by hand for the 256^3 grid
cut into 4x4x4 boxes of 64^3 with 16 guard cells (padded 96^3, H = 49)."""
import os
import sys

import numpy as np
import pytest

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import bench  # noqa: E402
from paper_1707_08500_amd import synth  # noqa: E402


class FakePlan:
    """The three things algorithmic_bytes asks a plan: layout, tuning, precision."""

    def __init__(self, padded, precision, fuse=0):
        self.padded = padded
        self.precision = precision
        self.fuse = fuse

    def layout(self, s):
        return tuple(self.padded[s]), 0

    def tuning(self):
        return {"fuse_eb": self.fuse}


def cfg2():
    lo, n, g = synth.uniform_decomposition((256, 256, 256), (4, 4, 4), 16)
    padded = [tuple(int(v) for v in np.asarray(n[s]) + 2 * np.asarray(g[s])) for s in range(len(lo))]
    return lo, n, g, padded


def test_config2_bytes_fp32_increment_form():
    lo, n, g, padded = cfg2()
    assert len(lo) == 64 and set(padded) == {(96, 96, 96)}
    out, kpoints = bench.algorithmic_bytes(FakePlan(padded, "f32"), lo, n, g, 4)
    P, I, H, boxes = 96, 64, 49, 64
    guard = P ** 3 - I ** 3                        # 622592 guard cells per box
    assert kpoints == boxes * P * P * H
    # J and E,B exchange: every guard cell read once and written once
    assert out["exchange_J"] == boxes * guard * 3 * 2 * 4
    assert out["exchange_EB"] == boxes * guard * 6 * 2 * 4
    # forward x/y: 9 padded real fields read, 9 half spectra written
    assert out["fft_xy_fwd"] == boxes * (9 * P ** 3 * 4 + 9 * P * P * H * 8)
    # z pass: 9 complex read at every k-point, 6 written on the 64 interior z-planes
    assert out["z_update"] == boxes * (9 * P + 6 * I) * P * H * 8
    assert out["z_update"] == 3005743104
    # inverse: 6 half spectra of the interior planes read; the increment is added
    # to the interior cells (read and written)
    assert out["fft_xy_inv"] == boxes * (6 * I * P * H * 8 + 2 * 6 * I ** 3 * 4)


def test_fp64_writes_without_reading_and_fused_exchange_moves_nothing():
    lo, n, g, padded = cfg2()
    out, _ = bench.algorithmic_bytes(FakePlan(padded, "f64"), lo, n, g, 8)
    P, I, H, boxes = 96, 64, 49, 64
    assert out["fft_xy_inv"] == boxes * (6 * I * P * H * 16 + 6 * I ** 3 * 8)
    fused, _ = bench.algorithmic_bytes(FakePlan(padded, "f64", fuse=1), lo, n, g, 8)
    assert fused["exchange_EB"] == 0
    assert fused["fft_xy_inv"] == out["fft_xy_inv"] + boxes * (P ** 3 - I ** 3) * 6 * 8


def test_roofline_block_is_bmin_over_the_dominant_kernel():
    """roofline.achieved follows the benchmark's measurement rule: B_min = 15
    reals (read E, B, J; write E, B) per padded cell per step, over the
    event-timed launch of the dominant kernel; the kernel's own algorithmic
    bytes over the same time are reported beside it."""
    lo, n, g, padded = cfg2()
    algo, _ = bench.algorithmic_bytes(FakePlan(padded, "f32"), lo, n, g, 4)
    res = {"phases_ms": {"exchange_J": 0.05, "fft_xy_fwd": 1.0, "z_update": 1.25, "fft_xy_inv": 0.5,
                         "exchange_EB": 0.5},
           "algo_bytes": algo, "ms_per_step": 3.3,
           "tuning": {"split_xy": 0, "z_pencils": 8, "z_threads": 512, "max_radix": 16, "xy_threads": 256}}
    rf = bench.roofline_block("no_such_workload", res, "f32", (lo, n, g))
    cells = 64 * 96 ** 3
    assert rf["kernel"] == "z_update" and rf["bytes_per_launch"] == 15 * 4 * cells
    assert abs(rf["achieved"] - 15 * 4 * cells / 1.25e-3 / 1e9) < 1e-6
    assert abs(rf["frac"] - rf["achieved"] / 8000.0) < 1e-12
    assert abs(rf["kernel_own"]["achieved"] - algo["z_update"] / 1.25e-3 / 1e9) < 1e-6
    assert rf["traffic"] is None
    assert rf["kernel_instance"] == "psatd::k_z_update<float, 512, 8, true, 16, 0>"


def test_field_diagnostics_vanish_on_oracle_steps_and_see_a_planted_error():
    """The bench's div B and Gauss-law diagnostics (Sec. 3.1 with the
    continuity of a constant J) read rounding-level zeros on states the oracle's
    PSATD-global produced, and a longitudinal E error planted on the CPU shows."""
    import torch
    from oracle import psatd_oracle as O
    sys.path.insert(0, os.path.join(os.path.dirname(__file__)))
    from psatd_cases import random_fields

    N, d, p, c, dt, steps = (16, 12, 10), (1.0, 1.0, 1.0), 8, 1.0, 0.4, 3
    E0, B0, J = random_fields(N, 7, d, p)
    E, B = O.run_global(E0, B0, J, d, p, c, dt, steps)

    class Inputs:
        def __init__(self):
            self.N = N

        def field(self, which, dtype, dev):
            src = {"E": E0, "J": J}[which]
            return [torch.from_numpy(src[u].copy()).to(dev, dtype).reshape(-1) for u in range(3)]

    kt = [O.modified_k(N[u], d[u], p) for u in range(3)]
    final = [torch.from_numpy(F[u].copy()).reshape(-1) for F in (E, B) for u in range(3)]
    diag = bench.field_diagnostics(final, Inputs(), kt, steps * dt, c, dev="cpu")
    assert diag["div_B_rel"] < 1e-13
    assert diag["gauss_rel"] < 1e-13
    assert diag["energy"] == pytest.approx(0.5 * (np.sum(E * E) + np.sum(B * B)), rel=1e-12)
    # a longitudinal bump in E_x (a gradient field) breaks Gauss's law only
    x = np.arange(N[0])
    bump = np.broadcast_to(np.sin(2 * np.pi * x / N[0]), E[0].shape)
    final[0] = torch.from_numpy((E[0] + 1e-3 * bump).copy()).reshape(-1)
    bad = bench.field_diagnostics(final, Inputs(), kt, steps * dt, c, dev="cpu")
    assert bad["gauss_rel"] > 1e-5
    assert bad["div_B_rel"] < 1e-13


def test_bench_refuses_more_than_one_gpu():
    """The benchmark is the single-GPU share of a sharded run: --gpus above 1
    exits with status 2 and says so, before touching a device."""
    import subprocess
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
