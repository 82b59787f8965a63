"""Truncation sweep of the local-FFT method (Sec. 3.2, Fig. 3).

The decomposed push pads every subdomain with g guard cells and applies the
periodic PSATD operator of the padded box; its difference from PSATD-global
(one box covering the periodic grid, no guards, i.e. one global FFT per step)
is the method's truncation error.  Sec. 3.2 states that it depends on the
stencil order p, the guard width g and the mesh resolution, falls off quickly
with g, does not grow with the number of steps, and that 8 guards suffice at
p = 100 for fields resolved like the laser runs of Sec. 4 (about 60 cells per
wavelength).  The sweep measures all three axes:

* order p and guard width g (uniform boxes);
* resolution: three laser-like vacuum pulses (Gaussian envelope times a
  carrier of lambda cells, k dx = 2 pi / lambda), one along each axis, or the
  broadband input (a few long oblique waves and a Gaussian current pulse);
* time: the difference after every step count of a list.

The broadband waves are polarised orthogonally to the order-p modified wave
vector [k] of the global grid, with B = [k]^ x E / c ([k] from the library:
a one-box plan read back through the C-ABI); each pulse depends on one
coordinate only, with B = u^ x E / c.  Either way every mode is a vacuum
eigenmode of PSATD-global and the input is divergence-free for the operator
being applied.

Both runs go through the C-ABI on the GPU (the global run is a plan with a
single box and no guards), in FP64 by default so that the measured difference
is the method's, not rounding.

    python -m paper_1707_08500_amd.truncation --grid 128 --boxes 4 \
        --orders 16,32,64,100 --guards 4,8,16,24 --waves smooth,64,32,16,8 \
        --steps 20,80
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

from . import synth


def global_modified_k(N, d, p):
    """The library's FP64 order-p modified wavenumbers of the periodic grid N,
    per axis, indexed by FFT bin (a one-box plan without guards)."""
    from . import psatd
    plan = psatd.Plan(N, d, [[0, 0, 0]], [list(N)], [[0, 0, 0]], p, 0.5, precision="f32")
    try:
        return [plan.modified_k(0, u) for u in range(3)]
    finally:
        plan.close()


def _wave_pair(N, kmod, m, a, c):
    """Unit transverse polarisation of wave m (orthogonal to [k]) and the
    matching B direction [k]^ x a / c."""
    kv = np.array([kmod[u][int(m[u]) % N[u]] for u in range(3)])
    kh = kv / np.linalg.norm(kv)
    a = np.asarray(a, dtype=float)
    a = a - (a @ kh) * kh
    a = a / np.linalg.norm(a)
    return a, np.cross(kh, a) / c


def smooth_fields(N, kmod, d=(1.0, 1.0, 1.0), c=1.0, case=11, waves=4, mmax=3, sigma=4.0):
    """Broadband input: a few long oblique vacuum waves and one Gaussian current
    pulse, as global [3][z][y][x] arrays (E, B, J).  kmod: the order-p modified
    wavenumbers of the grid, per axis."""
    ms, amps, phases = synth.wave_parameters(case=case, count=waves, mmax=mmax)
    E = np.zeros((3, N[2], N[1], N[0]))
    B = np.zeros_like(E)
    for m, a, ph in zip(ms, amps, phases):
        ea, eb = _wave_pair(N, kmod, m, a, c)
        E += synth.plane_wave(N, m, ea, ph)
        B += synth.plane_wave(N, m, eb, ph)
    J = synth.current_pulses(N, d, case=case, count=1, sigma=sigma)
    return E, B, J


def resolution_fields(N, cells_per_wavelength, width=16.0, c=1.0):
    """Three forward-moving vacuum pulses, one along each axis (the x pulse
    polarised along y, y along z, z along x), each a Gaussian envelope of
    standard deviation `width` cells times a carrier of `cells_per_wavelength`
    cells, uniform across the other two axes, centred at 0.3, 0.5 and 0.7 of
    its axis so that it straddles subdomain boundaries.  Each pulse depends on
    one coordinate only, so it is divergence-free, and B = u^ x E / c: every
    mode of it, of either sign of k, then evolves as exp(-i c [k] t), a
    forward-moving eigenmode of PSATD-global at any order.  No current.
    (Plane waves are no probe here:
    a wave whose wavelength divides the padded box length is periodic on the
    box and has no truncation error at all.)"""
    E = np.zeros((3, N[2], N[1], N[0]))
    B = np.zeros_like(E)
    for u in range(3):
        L = N[u]
        x = np.arange(L, dtype=float)
        r = x - (0.3 + 0.2 * u) * L
        r -= L * np.round(r / L)
        f = np.exp(-r * r / (2.0 * width * width)) * np.cos(2 * np.pi * r / cells_per_wavelength)
        e_ax, b_ax = (u + 1) % 3, (u + 2) % 3
        shape = [1, 1, 1]
        shape[2 - u] = L  # arrays are [z][y][x]
        E[e_ax] += f.reshape(shape)
        B[b_ax] += f.reshape(shape) / c
    return E, B, np.zeros_like(E)


def run_fields(N, d, lo, n, g, p, dt, c, fields, checkpoints, precision="f64"):
    """E, B after each step count in `checkpoints` (ascending) of pushes of
    the decomposition (lo, n, g), gathered to the global grid as float64
    numpy arrays: a list of (E, B)."""
    import torch

    from . import psatd
    plan = psatd.Plan(N, d, lo, n, g, p, dt, c, precision=precision)
    try:
        dtype = plan.dtype
        bufs = []
        for F in fields:
            pad = plan.empty_fields()
            plan.scatter([torch.from_numpy(np.ascontiguousarray(F[a])).to("cuda", dtype).reshape(-1)
                          for a in range(3)], pad)
            bufs.append(pad)
        out, done = [], 0
        for k in checkpoints:
            if k > done:
                # J is replicated and unchanged between runs, so segments of
                # psatd_run compose to one run of the total step count
                plan.run(bufs[0], bufs[1], bufs[2], k - done)
                done = k
            snap = []
            for pad in bufs[:2]:
                glob = [torch.empty(N[0] * N[1] * N[2], dtype=dtype, device="cuda") for _ in range(3)]
                plan.gather(pad, glob)
                torch.cuda.synchronize()
                snap.append(np.stack([x.double().cpu().numpy().reshape(N[2], N[1], N[0]) for x in glob]))
            out.append(tuple(snap))
        return out
    finally:
        plan.close()


def _rel(x, ref):
    den = float(np.sqrt(np.sum(ref * ref)))
    return float(np.sqrt(np.sum((x - ref) ** 2)) / (den if den else 1.0))


def sweep(N, nbox, orders, guards, steps, dt=0.5, c=1.0, d=(1.0, 1.0, 1.0), precision="f64",
          waves=("smooth",), width=16.0, fields=None, log=None):
    """Rows {p, g, waves, cells_per_wavelength, kdx, steps, rel_l2_E, rel_l2_B,
    energy} of the local-vs-global difference for every order p, input
    ("smooth", or the pulses' cells per wavelength), guard width g (uniform
    boxes) and step count.  `fields(p, w)` may supply the input instead of
    the built-in ones."""
    steps = sorted({int(s) for s in (steps if hasattr(steps, "__iter__") else [steps])})
    rows = []
    for p in orders:
        kmod = global_modified_k(N, d, p) if fields is None and "smooth" in waves else None
        for w in waves:
            if fields is not None:
                F = fields(p, w)
            elif w == "smooth":
                F = smooth_fields(N, kmod, d, c)
            else:
                F = resolution_fields(N, float(w), width, c)
            ref = run_fields(N, d, [[0, 0, 0]], [list(N)], [[0, 0, 0]], p, dt, c, F, steps, precision)
            cpw = None if w == "smooth" else float(w)
            for gw in guards:
                lo, n, g = synth.uniform_decomposition(N, nbox, gw)
                loc = run_fields(N, d, lo, n, g, p, dt, c, F, steps, precision)
                for k, (El, Bl), (Eg, Bg) in zip(steps, loc, ref):
                    den = float(np.sum(Eg ** 2) + c * c * np.sum(Bg ** 2))
                    num = float(np.sum((El - Eg) ** 2) + c * c * np.sum((Bl - Bg) ** 2))
                    rows.append(dict(p=p, g=gw, waves=str(w), cells_per_wavelength=cpw,
                                     kdx=None if cpw is None else 2 * np.pi / cpw, steps=k,
                                     rel_l2_E=_rel(El, Eg), rel_l2_B=_rel(Bl, Bg),
                                     energy=float(np.sqrt(num / den))))
                if log:
                    r = rows[-1]
                    log(f"p={p} waves={w} g={gw}: {r['energy']:.3e} after {r['steps']} steps")
    return rows


def guards_needed(rows, eps, steps=None):
    """Smallest swept guard width whose energy-norm difference is <= eps, per
    (order, input), at the largest step count (or `steps`)."""
    out = {}
    k = max(r["steps"] for r in rows) if steps is None else steps
    for p in sorted({r["p"] for r in rows}):
        for w in dict.fromkeys(r["waves"] for r in rows):
            ok = [r["g"] for r in rows if r["p"] == p and r["waves"] == w and r["steps"] == k
                  and r["energy"] <= eps]
            out[(p, w)] = min(ok) if ok else None
    return out


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--grid", type=int, default=128, help="cells per axis of the periodic grid")
    ap.add_argument("--boxes", type=int, default=4, help="subdomains per axis")
    ap.add_argument("--orders", default="16,32,64,100")
    ap.add_argument("--guards", default="4,8,16,24")
    ap.add_argument("--waves", default="smooth,64,32,16,8",
                    help="inputs: 'smooth' (broadband) or the pulses' cells per wavelength")
    ap.add_argument("--width", type=float, default=16.0, help="pulse envelope standard deviation, cells")
    ap.add_argument("--steps", default="20,80", help="step counts at which the difference is taken")
    ap.add_argument("--dt", type=float, default=0.5)
    ap.add_argument("--precision", default="f64")
    ap.add_argument("--eps", default="1e-3,1e-5,1e-8")
    ap.add_argument("--json", default=None, help="also write the rows to this file")
    args = ap.parse_args(argv)
    N = (args.grid,) * 3
    nbox = (args.boxes,) * 3
    orders = [int(v) for v in args.orders.split(",")]
    guards = [int(v) for v in args.guards.split(",")]
    waves = [w if w == "smooth" else float(w) for w in args.waves.split(",")]
    steps = [int(v) for v in args.steps.split(",")]
    rows = sweep(N, nbox, orders, guards, steps, dt=args.dt, precision=args.precision, waves=waves,
                 width=args.width, log=lambda s: print(s, file=sys.stderr, flush=True))
    print(f"# local-vs-global difference, {args.grid}^3 grid, {args.boxes}^3 boxes, "
          f"dt={args.dt}, {args.precision}")
    print("p    waves   cells/wl  g    steps  rel_l2_E     rel_l2_B     energy")
    for r in rows:
        cpw = "-" if r["cells_per_wavelength"] is None else f"{r['cells_per_wavelength']:.1f}"
        print(f"{r['p']:<4d} {r['waves']:<7s} {cpw:<9s} {r['g']:<4d} {r['steps']:<6d} "
              f"{r['rel_l2_E']:.3e}    {r['rel_l2_B']:.3e}    {r['energy']:.3e}")
    for eps in (float(v) for v in args.eps.split(",")):
        need = guards_needed(rows, eps)
        print(f"# guards needed for energy-norm difference <= {eps:g} after {max(steps)} steps: "
              + ", ".join(f"p={p}/{w}: {g}" for (p, w), g in need.items()))
    if args.json:
        with open(args.json, "w") as fh:
            json.dump(rows, fh)


if __name__ == "__main__":
    main()
