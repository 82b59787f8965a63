"""Seeded synthetic inputs for the local-FFT PSATD field push.

This module holds no step of the method: it draws decompositions and builds
simple analytic fields (Gaussian current pulses, charge blobs, plane waves
with a given wave vector and amplitude vector, a laser-like pulse).  Anything
that needs the method's modified wavenumbers (polarisations orthogonal to
[k], Gauss-law fields) is built by the caller.

Random numbers: NumPy PCG64 seeded with SeedSequence([1707, 8500, case, stream]);
stream 0 = decomposition, 1 = waves, 2 = currents, 3 = charge, 4 = partitions.

Arrays are C-ordered [z][y][x]; vector fields carry a leading axis of 3
holding the (x, y, z) components.
"""
from __future__ import annotations

import numpy as np

STREAM_DECOMP, STREAM_WAVES, STREAM_J, STREAM_RHO, STREAM_PART = 0, 1, 2, 3, 4


def rng(case: int, stream: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([1707, 8500, case, stream])))


# ---------------------------------------------------------------- boxes
def uniform_decomposition(grid_n, nbox, guard):
    """Regular cut of grid_n = (Nx, Ny, Nz) into nbox = (bx, by, bz) equal boxes,
    all with the same guard width.  Returns lo, n, g as (nsub, 3) int64 arrays in
    (x, y, z), boxes ordered x fastest."""
    grid_n = [int(v) for v in grid_n]
    nbox = [int(v) for v in nbox]
    for u in range(3):
        if grid_n[u] % nbox[u]:
            raise ValueError("grid not divisible by box count")
    size = [grid_n[u] // nbox[u] for u in range(3)]
    lo, n, g = [], [], []
    for bz in range(nbox[2]):
        for by in range(nbox[1]):
            for bx in range(nbox[0]):
                lo.append([bx * size[0], by * size[1], bz * size[2]])
                n.append(size)
                g.append([int(guard)] * 3 if np.isscalar(guard) else list(guard))
    return (np.array(lo, dtype=np.int64), np.array(n, dtype=np.int64),
            np.array(g, dtype=np.int64))


def uneven_decomposition(grid_n, case, lengths=(48, 64, 80, 96), guards=(8, 16, 32)):
    """Tensor-product cut with uneven boxes: per axis, draw lengths iid uniform
    from `lengths` until their sum reaches the axis length, redrawing the whole
    axis unless the sum is exact; then one guard width per box, iid uniform from
    `guards`, used on all three axes."""
    r = rng(case, STREAM_DECOMP)
    cuts = []
    for u in range(3):
        N = int(grid_n[u])
        for _attempt in range(100000):
            seq, tot = [], 0
            while tot < N:
                v = int(r.choice(lengths))
                seq.append(v)
                tot += v
            if tot == N:
                break
        else:  # pragma: no cover
            raise RuntimeError("no exact cut found")
        cuts.append(seq)
    lo, n = [], []
    zs = np.concatenate([[0], np.cumsum(cuts[2])])
    ys = np.concatenate([[0], np.cumsum(cuts[1])])
    xs = np.concatenate([[0], np.cumsum(cuts[0])])
    for iz, nz in enumerate(cuts[2]):
        for iy, ny in enumerate(cuts[1]):
            for ix, nx in enumerate(cuts[0]):
                lo.append([xs[ix], ys[iy], zs[iz]])
                n.append([nx, ny, nz])
    g = r.choice(np.asarray(guards), size=len(lo))
    g = np.repeat(g[:, None], 3, axis=1)
    return (np.array(lo, dtype=np.int64), np.array(n, dtype=np.int64),
            np.array(g, dtype=np.int64))


# ---------------------------------------------------------------- fields
def _coords(grid_n, d):
    Nx, Ny, Nz = grid_n
    x = np.arange(Nx) * d[0]
    y = np.arange(Ny) * d[1]
    z = np.arange(Nz) * d[2]
    return x[None, None, :], y[None, :, None], z[:, None, None]


def min_image(delta, L):
    return delta - L * np.round(delta / L)


def gaussian_blob(grid_n, d, center, sigma):
    """exp(-r^2 / (2 sigma^2)) with the minimum-image distance on the periodic
    grid; shape (Nz, Ny, Nx)."""
    X, Y, Z = _coords(grid_n, d)
    L = [grid_n[u] * d[u] for u in range(3)]
    rx = min_image(X - center[0], L[0])
    ry = min_image(Y - center[1], L[1])
    rz = min_image(Z - center[2], L[2])
    return np.exp(-(rx * rx + ry * ry + rz * rz) / (2.0 * sigma * sigma))


def random_unit_vectors(r, count):
    v = r.normal(size=(count, 3))
    return v / np.linalg.norm(v, axis=1, keepdims=True)


def current_pulse_params(grid_n, d, case, count=1, amp_range=(0.5, 1.0)):
    """The draws behind current_pulses: centres (count, 3) uniform on the grid,
    amplitudes uniform in amp_range, directions uniform on the sphere."""
    r = rng(case, STREAM_J)
    L = np.array([grid_n[u] * d[u] for u in range(3)])
    centres = r.uniform(0.0, 1.0, size=(count, 3)) * L
    amps = r.uniform(amp_range[0], amp_range[1], size=count)
    dirs = random_unit_vectors(r, count)
    return centres, amps, dirs


def current_pulses(grid_n, d, case, count=1, sigma=8.0, amp_range=(0.5, 1.0)):
    """Sum of `count` Gaussian current pulses: centre uniform on the grid,
    amplitude uniform in amp_range, direction uniform on the sphere.
    Returns (3, Nz, Ny, Nx) float64."""
    centres, amps, dirs = current_pulse_params(grid_n, d, case, count, amp_range)
    J = np.zeros((3, grid_n[2], grid_n[1], grid_n[0]))
    for i in range(count):
        g = gaussian_blob(grid_n, d, centres[i], sigma) * amps[i]
        for a in range(3):
            J[a] += dirs[i, a] * g
    return J


def charge_blob(grid_n, d, case, sigma=8.0, amp_range=(0.5, 1.0)):
    """Seeded Gaussian charge blob with its mean removed (shape (Nz, Ny, Nx))."""
    r = rng(case, STREAM_RHO)
    L = np.array([grid_n[u] * d[u] for u in range(3)])
    centre = r.uniform(0.0, 1.0, size=3) * L
    q = r.uniform(*amp_range)
    rho = q * gaussian_blob(grid_n, d, centre, sigma)
    return rho - rho.mean()


def wave_parameters(case, count, mmax, exclude_nyquist_of=None):
    """`count` integer wave-index vectors m (x, y, z), iid uniform in
    [-mmax, mmax]^3 without 0, plus raw N(0, I) amplitude vectors and phases
    U(0, 2 pi).  The caller projects the amplitudes (e.g. orthogonal to [k])."""
    r = rng(case, STREAM_WAVES)
    ms = []
    while len(ms) < count:
        m = r.integers(-mmax, mmax + 1, size=3)
        if not m.any():
            continue
        if exclude_nyquist_of is not None and any(
                2 * abs(int(m[u])) == exclude_nyquist_of[u] for u in range(3)):
            continue
        ms.append(m)
    amps = r.normal(size=(count, 3))
    phases = r.uniform(0.0, 2.0 * np.pi, size=count)
    return np.array(ms, dtype=np.int64), amps, phases


def plane_wave(grid_n, m, vec, phase, t_phase=0.0):
    """vec * cos(k.x + phase - t_phase) with k_u = 2 pi m_u / N_u on grid
    indices; returns (3, Nz, Ny, Nx)."""
    Nx, Ny, Nz = grid_n
    i = np.arange(Nx)[None, None, :]
    j = np.arange(Ny)[None, :, None]
    l = np.arange(Nz)[:, None, None]
    arg = (2 * np.pi * m[0] * i / Nx + 2 * np.pi * m[1] * j / Ny
           + 2 * np.pi * m[2] * l / Nz + phase - t_phase)
    cs = np.cos(arg)
    return np.stack([vec[0] * cs, vec[1] * cs, vec[2] * cs])


def laser_pulse(grid_n, d, c=1.0, wavelength=32.0, x_c=256.0, width=64.0):
    """Linearly polarised pulse along +x: E_y = cos(2 pi (x - x_c)/wavelength)
    exp(-(x - x_c)^2 / (2 width^2)), B_z = E_y / c, uniform in y and z.
    Returns E, B as (3, Nz, Ny, Nx)."""
    Nx, Ny, Nz = grid_n
    x = np.arange(Nx) * d[0]
    prof = np.cos(2 * np.pi * (x - x_c) / wavelength) * np.exp(-(x - x_c) ** 2 / (2 * width ** 2))
    E = np.zeros((3, Nz, Ny, Nx))
    B = np.zeros((3, Nz, Ny, Nx))
    E[1] = prof[None, None, :]
    B[2] = prof[None, None, :] / c
    return E, B


def partition_weights(r, ncopies):
    """Random weights summing to 1 over `ncopies` copies (Dirichlet(1))."""
    w = r.exponential(size=ncopies)
    return w / w.sum()
