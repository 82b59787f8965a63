"""Shared builders for the GPU parity tests: seeded inputs (from the synth
module, made consistent with the oracle where the method's [k] is needed),
upload/download of the padded layout, per-component comparisons."""
from __future__ import annotations

import sys

import numpy as np

from oracle import psatd_oracle as O
from paper_1707_08500_amd import synth


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def random_fields(N, seed, d=(1.0, 1.0, 1.0), p=8, divfree=True):
    """E, B, J ~ N(0, 1) on the grid; B made div-free w.r.t. the order-p [k]."""
    r = np.random.default_rng(seed)
    shape = (N[2], N[1], N[0])
    E = r.normal(size=(3,) + shape)
    B = r.normal(size=(3,) + shape)
    J = r.normal(size=(3,) + shape)
    if divfree:
        kx, ky, kz = O.k_grid(shape, d, p)
        Bk = O.fft3(B)
        k2 = kx * kx + ky * ky + kz * kz
        kB = kx * Bk[0] + ky * Bk[1] + kz * Bk[2]
        f = np.where(k2 == 0, 0.0, kB / np.where(k2 == 0, 1.0, k2))
        B = O.ifft3(Bk - np.stack([kx * f, ky * f, kz * f])).real
    return E, B, J


def deposited_partition(J, dec, seed):
    """Partial currents per padded copy: every global value of J split among
    all its copies with random positive weights (deposited mode: the sum over
    the copies is J)."""
    N = dec.N
    r = synth.rng(seed, synth.STREAM_PART)
    Jrep = O.scatter(J, dec)
    wts = [r.exponential(size=Jb.shape[1:]) for Jb in Jrep]
    wsum = np.zeros((N[2], N[1], N[0]))
    for s in range(dec.nsub):
        ix, iy, iz = dec.global_index(s)
        Z, Y, X = np.meshgrid(iz, iy, ix, indexing="ij")
        np.add.at(wsum, (Z, Y, X), wts[s])
    out = []
    for s in range(dec.nsub):
        ix, iy, iz = dec.global_index(s)
        Z, Y, X = np.meshgrid(iz, iy, ix, indexing="ij")
        out.append(J[:, Z, Y, X] * wts[s] / wsum[Z, Y, X])
    return out


def upload_boxes(case, bufs, boxes):
    """Writes per-box padded arrays (3, Pz, Py, Px) into a plan's field buffers,
    each box at the offset the plan's layout gives it (the alignment gaps
    between boxes stay zero)."""
    import torch
    for a in range(3):
        host = np.zeros(case.plan.field_elems)
        for s in range(case.dec.nsub):
            _, off = case.plan.layout(s)
            flat = boxes[s][a].ravel()
            host[off:off + flat.size] = flat
        bufs[a].copy_(torch.from_numpy(host).to("cuda", case.dtype))
    torch.cuda.synchronize()


def config2_fields(N, d, p, case=2, sigma=8.0):
    """Gaussian current pulse, Gauss-law E from a mean-free Gaussian charge
    blob (with the same order-p [k]), B = 0."""
    J = synth.current_pulses(N, d, case=case, count=1, sigma=sigma)
    rho = synth.charge_blob(N, d, case=case, sigma=sigma)
    E = O.gauss_solution(rho, d, p)
    B = np.zeros_like(E)
    return E, B, J


class GpuCase:
    """A plan plus padded device state built from global FP64 numpy fields."""

    def __init__(self, N, lo, n, g, p, dt, c, precision, jmode, E, B, J, d=(1.0, 1.0, 1.0)):
        import torch
        from paper_1707_08500_amd import psatd
        self.dec = O.Decomposition(N, lo, n, g)
        self.plan = psatd.Plan(N, d, lo, n, g, p, dt, c, precision=precision, jmode=jmode)
        self.dtype = self.plan.dtype
        self.N = N
        self.E = self.plan.empty_fields()
        self.B = self.plan.empty_fields()
        self.J = self.plan.empty_fields()
        for glob, pad in ((E, self.E), (B, self.B), (J, self.J)):
            g3 = [torch.from_numpy(np.ascontiguousarray(glob[a])).to("cuda", self.dtype).reshape(-1)
                  for a in range(3)]
            self.plan.scatter(g3, pad)
        torch.cuda.synchronize()

    def boxes(self, bufs, which=None):
        """Padded boxes (3, Pz, Py, Px) as float64 numpy, for boxes `which`."""
        which = range(self.dec.nsub) if which is None else which
        host = [b.double().cpu().numpy() for b in bufs]
        out = {}
        for s in which:
            (px, py, pz), off = self.plan.layout(s)
            out[s] = np.stack([h[off:off + px * py * pz].reshape(pz, py, px) for h in host])
        return out

    def gathered(self, bufs):
        import torch
        glob = [torch.empty(self.N[0] * self.N[1] * self.N[2], dtype=self.dtype, device="cuda")
                for _ in range(3)]
        self.plan.gather(bufs, glob)
        torch.cuda.synchronize()
        return np.stack([g.double().cpu().numpy().reshape(self.N[2], self.N[1], self.N[0])
                         for g in glob])


def rel_l2_components(x, ref):
    return [O.rel_l2(x[a], ref[a]) for a in range(3)]


def boxes_rel_l2(got: dict, ref: list):
    """Per-component rel-L2 over all padded cells of the given boxes."""
    out = []
    for a in range(3):
        num = sum(float(np.sum((got[s][a] - ref[s][a]) ** 2)) for s in got)
        den = sum(float(np.sum(ref[s][a] ** 2)) for s in got)
        out.append(np.sqrt(num / den) if den > 0 else np.sqrt(num))
    return out


def energy_rel_l2(gE: dict, gB: dict, oE: list, oB: list, c=1.0):
    """Relative L2 error in the field-energy norm sqrt(|E|^2 + c^2 |B|^2) over
    all padded cells of the given boxes (the state-level error of a path whose
    rounding is relative to the whole state, not to each component)."""
    num = den = 0.0
    for s in gE:
        num += float(np.sum((gE[s] - oE[s]) ** 2) + c * c * np.sum((gB[s] - oB[s]) ** 2))
        den += float(np.sum(oE[s] ** 2) + c * c * np.sum(oB[s] ** 2))
    return float(np.sqrt(num / den))
