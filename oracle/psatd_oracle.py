"""Plain FP64 CPU oracle for the local-FFT PSATD field push.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline
leg of the benchmark may import this module.  The product path (the HIP library
and its Python binding) never imports, calls or links it, and this module
imports nothing from the product package.

What it computes (Vincenti & Vay, "Ultrahigh-order Maxwell solver with extreme
scalability for electromagnetic PIC simulations of plasmas"):

* ``fd_weights``      -- the order-p centred nodal finite-difference weights w_j
                          that enter the modified-wavenumber substitution of
                          Sec. 3.1 (text after Eq. PSATD_2).
* ``modified_k``      -- that substitution, k_u -> sum_j w_j sin(j k_u du)/(du/2),
                          per axis over the FFT index, and the exact k for
                          infinite order (Sec. 3.1).
* ``psatd_coefficients`` / ``psatd_update`` -- the analytic k-space time update,
                          Eqs. PSATD_1 and PSATD_2 (Sec. 3.1), written for a
                          general speed of light c (reduces to the printed c=1
                          form).
* ``step_global``     -- one PSATD step on a periodic grid: forward FFT, update,
                          inverse FFT ("O-global", the PSATD-global method of
                          Sec. 3.2 / Fig. 2b, as mathematics, not distributed);
                          real-to-complex transforms over the half spectrum,
                          the pointwise update spread over threads by kz slab.
* ``Decomposition``, ``scatter``, ``gather``, ``exchange_fill``,
  ``exchange_sum``, ``step_local`` -- the domain-decomposed method of Sec. 3.2
                          (Fig. 2a and the three steps of Fig. 3): every
                          subdomain padded with guard cells, advanced as an
                          independent periodic box with its own local FFT, then
                          its guard cells replaced by the owning neighbour's
                          values.  The guard-current sum (deposited mode) is
                          standard PIC practice (Sec. 2, the deposition step of
                          the PIC loop); the paper does not spell it out.
* ``heat_step_global``, ``heat_run_local`` -- the same local-FFT method for
                          the diffusion equation (Sec. 5 names it among the
                          initial-value problems the method applies to): exact
                          propagator exp(-D |[k]|^2 dt) with the order-p [k].
* diagnostics: spectral div B, Gauss residual, field energy.

Conventions (readings of the paper, each listed in the design notes):
  * arrays are C-ordered [z][y][x]; vector fields carry a leading axis of
    length 3 holding the (x, y, z) components;
  * forward FFT exp(-i k.x), unnormalised; inverse carries 1/N;
  * d/dt B = -[curl] E,  d/dt E = c^2 [curl] B - J   (eps0 = 1, mu0 = 1/c^2);
  * Nyquist entries of the modified wavenumber are exactly 0;
  * where |[k]| = 0 the k -> 0 limits of the coefficients are used.

Parity: every function here is pinned by the CPU tests against closed forms,
brute force, a matrix exponential or textbook values.
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass
from fractions import Fraction
from functools import lru_cache

import numpy as np
import scipy.fft as sfft

# FFT worker threads: the CPUs this process may use, at most 16 (override with
# PSATD_ORACLE_WORKERS).
_WORKERS = int(os.environ.get("PSATD_ORACLE_WORKERS",
                              min(len(os.sched_getaffinity(0)) or 1, 16)))


# --------------------------------------------------------------------------
# Sec. 3.1: order-p modified wavenumbers
# --------------------------------------------------------------------------
@lru_cache(maxsize=None)
def fd_weights_exact(p: int) -> tuple:
    """Exact rational weights w_1..w_{p/2} of the order-p centred nodal first
    derivative  f'(x_i) ~ (1/du) sum_j w_j (f_{i+j} - f_{i-j})  (Sec. 3.1: "the
    coefficients of the finite-differenciation at order p").

    Definition: the stencil is exact for every polynomial of degree <= p, i.e.
    for f = x^(2l+1), l = 0..p/2-1:  sum_j 2 j^(2l+1) w_j = [l == 0].  (Even
    powers are annihilated by symmetry.)  Solved here by exact Gaussian
    elimination over the rationals.
    """
    if p < 2 or p % 2:
        raise ValueError("order p must be even and >= 2")
    M = p // 2
    rows = [[Fraction(2 * j ** (2 * l + 1)) for j in range(1, M + 1)]
            + [Fraction(1 if l == 0 else 0)] for l in range(M)]
    for col in range(M):
        piv = next(r for r in range(col, M) if rows[r][col] != 0)
        rows[col], rows[piv] = rows[piv], rows[col]
        pv = rows[col][col]
        rows[col] = [x / pv for x in rows[col]]
        for r in range(M):
            if r != col and rows[r][col] != 0:
                f = rows[r][col]
                rows[r] = [a - f * b for a, b in zip(rows[r], rows[col])]
    return tuple(rows[i][M] for i in range(M))


def fd_weights(p: int) -> np.ndarray:
    """FP64 copy of :func:`fd_weights_exact`."""
    return np.array([float(w) for w in fd_weights_exact(p)], dtype=np.float64)


def signed_index(N: int) -> np.ndarray:
    """Signed FFT index m~ for m = 0..N-1 (m for m < N/2, m - N above)."""
    m = np.arange(N)
    return np.where(m <= (N - 1) // 2, m, m - N)


def modified_k(N: int, du: float, p: int) -> np.ndarray:
    """Modified wavenumber [k]_u over the FFT index m = 0..N-1 (Sec. 3.1).

    k_m = 2 pi m~ / (N du).  Finite even p: [k] = sum_j w_j sin(j k_m du)/(du/2).
    p == 0 means infinite order: [k] = k_m.  For even N the Nyquist entry
    m = N/2 is set to exactly 0 (finite p gives sin(j pi) = 0 analytically;
    for infinite order this is the reading that keeps the update real-valued).
    """
    mt = signed_index(N).astype(np.float64)
    km = 2.0 * np.pi * mt / (N * du)
    if p == 0:
        kk = km.copy()
    else:
        w = fd_weights(p)
        kk = np.zeros(N)
        for j, wj in enumerate(w, start=1):
            kk += wj * np.sin(j * km * du) / (du / 2.0)
    if N % 2 == 0:
        kk[N // 2] = 0.0
    return kk


def k_grid(shape_zyx, d_xyz, p):
    """Broadcastable ([k]_x, [k]_y, [k]_z) for an array of shape (Nz, Ny, Nx)."""
    Nz, Ny, Nx = shape_zyx
    kx = modified_k(Nx, d_xyz[0], p)[None, None, :]
    ky = modified_k(Ny, d_xyz[1], p)[None, :, None]
    kz = modified_k(Nz, d_xyz[2], p)[:, None, None]
    return kx, ky, kz


# --------------------------------------------------------------------------
# Sec. 3.1: Eqs. PSATD_1 / PSATD_2
# --------------------------------------------------------------------------
def psatd_coefficients(k2, c, dt):
    """C, S/(c k), (1-C)/k^2 and (S/(c k) - dt)/k^2 at |[k]|^2 = k2 (Eq. PSATD,
    C = cos(c k dt), S = sin(c k dt)); the k -> 0 limits where k2 == 0."""
    k2 = np.asarray(k2, dtype=np.float64)
    k = np.sqrt(k2)
    zero = k2 == 0.0
    ks = np.where(zero, 1.0, k)
    th = c * ks * dt
    C = np.where(zero, 1.0, np.cos(th))
    S_ck = np.where(zero, dt, np.sin(th) / (c * ks))
    # 1 - cos(th) written as 2 sin^2(th/2): the same number without the
    # cancellation that would otherwise cost digits in i (X1/c^2) [k] x J at small k.
    X1 = np.where(zero, 0.5 * c * c * dt * dt, 2.0 * np.sin(0.5 * th) ** 2 / (ks * ks))
    X2 = np.where(zero, -(c * c * dt ** 3) / 6.0,
                  (np.sin(th) / (c * ks) - dt) / (ks * ks))
    return C, S_ck, X1, X2


def _cross(a, b):
    return (a[1] * b[2] - a[2] * b[1],
            a[2] * b[0] - a[0] * b[2],
            a[0] * b[1] - a[1] * b[0])


def psatd_update(Ek, Bk, Jk, kvec, c, dt):
    """Eqs. PSATD_1 / PSATD_2 for general c, on spectra (3, ...) with
    kvec = ([k]_x, [k]_y, [k]_z) broadcastable against them:

      E' = C E + i c^2 (S/ck) [k]xB - (S/ck) J + X1 [k]([k].E) + X2 [k]([k].J)
      B' = C B - i (S/ck) [k]xE + i (X1/c^2) [k]xJ

    with X1 = (1-C)/k^2, X2 = (S/ck - dt)/k^2.  At c = 1 this is the printed
    form: i S k^ x B, (1-C) k^(k^.E), k^(k^.J)(S/k - dt), i (1-C)/k k^ x J.
    """
    kx, ky, kz = kvec
    k2 = kx * kx + ky * ky + kz * kz
    C, S_ck, X1, X2 = psatd_coefficients(k2, c, dt)
    K = (kx, ky, kz)
    kE = kx * Ek[0] + ky * Ek[1] + kz * Ek[2]
    kJ = kx * Jk[0] + ky * Jk[1] + kz * Jk[2]
    kxB = _cross(K, Bk)
    kxE = _cross(K, Ek)
    kxJ = _cross(K, Jk)
    En = np.empty(np.broadcast_shapes(Ek.shape, np.shape(C)), dtype=np.complex128)
    Bn = np.empty_like(En)
    for a in range(3):
        En[a] = (C * Ek[a] + 1j * c * c * S_ck * kxB[a] - S_ck * Jk[a]
                 + X1 * K[a] * kE + X2 * K[a] * kJ)
        Bn[a] = C * Bk[a] - 1j * S_ck * kxE[a] + 1j * (X1 / (c * c)) * kxJ[a]
    return En, Bn


def fft3(f):
    """Unnormalised forward 3D FFT over the last three axes (library routine)."""
    return sfft.fftn(f, axes=(-3, -2, -1), workers=_WORKERS)


def ifft3(F):
    """Inverse 3D FFT over the last three axes, 1/N included (library routine)."""
    return sfft.ifftn(F, axes=(-3, -2, -1), workers=_WORKERS)


def rfft3(f):
    """Unnormalised forward 3D FFT of a real array over the last three axes,
    kept on the half spectrum kx = 0..Nx//2 (library routine; the other half is
    the complex conjugate of this one)."""
    return sfft.rfftn(f, axes=(-3, -2, -1), workers=_WORKERS)


def irfft3(F, shape_zyx):
    """Inverse of :func:`rfft3` onto a real (..., Nz, Ny, Nx) array, 1/N
    included (library routine)."""
    return sfft.irfftn(F, s=tuple(shape_zyx), axes=(-3, -2, -1), workers=_WORKERS)


def k_grid_half(shape_zyx, d_xyz, p):
    """:func:`k_grid` restricted to the half spectrum kx = 0..Nx//2 of rfft3."""
    kx, ky, kz = k_grid(shape_zyx, d_xyz, p)
    return kx[..., : shape_zyx[2] // 2 + 1], ky, kz


_POOL = None


def psatd_update_by_kz(Ek, Bk, Jk, kvec, c, dt):
    """:func:`psatd_update` applied to slabs of consecutive kz planes by a pool
    of threads.  The update acts on every k-point by itself (Eqs. PSATD_1 /
    PSATD_2 couple the fields at one k only), so each point gets exactly the
    arithmetic of one call on the whole spectrum; the slabs only bound the
    size of numpy's temporaries and let the threads share the work."""
    global _POOL
    if _POOL is None:
        from concurrent.futures import ThreadPoolExecutor
        _POOL = ThreadPoolExecutor(max_workers=_WORKERS)
    kx, ky, kz = kvec
    Nz = Ek.shape[-3]
    En = np.empty(np.broadcast_shapes(Ek.shape, Bk.shape, Jk.shape), dtype=np.complex128)
    Bn = np.empty_like(En)
    edges = np.linspace(0, Nz, min(Nz, 4 * _WORKERS) + 1).astype(int)

    def slab(i):
        z0, z1 = edges[i], edges[i + 1]
        e, b = psatd_update(Ek[..., z0:z1, :, :], Bk[..., z0:z1, :, :], Jk[..., z0:z1, :, :],
                            (kx, ky, kz[z0:z1]), c, dt)
        En[..., z0:z1, :, :] = e
        Bn[..., z0:z1, :, :] = b

    list(_POOL.map(slab, range(len(edges) - 1)))
    return En, Bn


def step_global(E, B, J, d, p, c, dt, return_residue=False):
    """One PSATD step on a periodic box (Sec. 3.1): FFT E, B, J; update; inverse
    FFT.  E, B, J are real (3, Nz, Ny, Nx) arrays; d = (dx, dy, dz).

    The fields are real, so the transforms are taken real-to-complex over the
    half spectrum kx = 0..Nx//2 (the update maps conjugate k-points to
    conjugate values because [k](-m) = -[k](m) and the Nyquist entries are 0;
    the other half adds nothing).  return_residue=True takes the full complex
    transforms instead and also returns the largest imaginary part left by the
    inverse, the check that the update keeps real fields real."""
    shape = E.shape[1:]
    if return_residue:
        kvec = k_grid(shape, d, p)
        En, Bn = psatd_update(fft3(E), fft3(B), fft3(J), kvec, c, dt)
        e = ifft3(En)
        b = ifft3(Bn)
        res = max(np.abs(e.imag).max(), np.abs(b.imag).max())
        return e.real.copy(), b.real.copy(), res
    kvec = k_grid_half(shape, d, p)
    En, Bn = psatd_update_by_kz(rfft3(E), rfft3(B), rfft3(J), kvec, c, dt)
    return irfft3(En, shape), irfft3(Bn, shape)


def run_global(E, B, J, d, p, c, dt, nsteps):
    for _ in range(nsteps):
        E, B = step_global(E, B, J, d, p, c, dt)
    return E, B


# --------------------------------------------------------------------------
# Sec. 3.2: domain decomposition with guard cells (Fig. 2a, Fig. 3)
# --------------------------------------------------------------------------
@dataclass
class Decomposition:
    """Global periodic grid N = (Nx, Ny, Nz) tiled by boxes; box s owns cells
    lo[s] .. lo[s]+n[s]-1 per axis and is padded by g[s] guard cells on both
    sides of each axis.  lo, n, g are (nsub, 3) integer arrays in (x, y, z)."""
    N: tuple
    lo: np.ndarray
    n: np.ndarray
    g: np.ndarray

    def __post_init__(self):
        self.N = tuple(int(v) for v in self.N)
        self.lo = np.asarray(self.lo, dtype=np.int64).reshape(-1, 3)
        self.n = np.asarray(self.n, dtype=np.int64).reshape(-1, 3)
        self.g = np.asarray(self.g, dtype=np.int64).reshape(-1, 3)

    @property
    def nsub(self):
        return self.lo.shape[0]

    def padded(self, s):
        """Padded extents (Nx_s, Ny_s, Nz_s) of box s."""
        return tuple(int(v) for v in self.n[s] + 2 * self.g[s])

    def global_index(self, s):
        """Per axis (x, y, z): global index (mod N) of every padded position."""
        return [(self.lo[s, u] - self.g[s, u] + np.arange(self.padded(s)[u])) % self.N[u]
                for u in range(3)]

    def owner_map(self):
        """Brute-force owner of every global cell, array [z][y][x]."""
        Nx, Ny, Nz = self.N
        own = -np.ones((Nz, Ny, Nx), dtype=np.int64)
        for s in range(self.nsub):
            x0, y0, z0 = self.lo[s]
            nx, ny, nz = self.n[s]
            if (own[z0:z0 + nz, y0:y0 + ny, x0:x0 + nx] != -1).any():
                raise ValueError("boxes overlap")
            own[z0:z0 + nz, y0:y0 + ny, x0:x0 + nx] = s
        if (own < 0).any():
            raise ValueError("boxes leave a gap")
        return own


def scatter(F, dec):
    """Global field(s) (..., Nz, Ny, Nx) -> list of padded boxes: every padded
    cell takes the value at its global index mod N (a consistent split,
    Fig. 3 step 1)."""
    out = []
    for s in range(dec.nsub):
        ix, iy, iz = dec.global_index(s)
        # padded cell (z, y, x) <- F[..., iz[z], iy[y], ix[x]]: one gather per axis
        out.append(F.take(iz, axis=-3).take(iy, axis=-2).take(ix, axis=-1))
    return out


def gather(boxes, dec):
    """Interiors of the padded boxes -> global field (each cell from its owner)."""
    first = boxes[0]
    Nx, Ny, Nz = dec.N
    G = np.zeros(first.shape[:-3] + (Nz, Ny, Nx), dtype=first.dtype)
    for s in range(dec.nsub):
        x0, y0, z0 = dec.lo[s]
        nx, ny, nz = dec.n[s]
        gx, gy, gz = dec.g[s]
        G[..., z0:z0 + nz, y0:y0 + ny, x0:x0 + nx] = \
            boxes[s][..., gz:gz + nz, gy:gy + ny, gx:gx + nx]
    return G


def exchange_fill(boxes, dec):
    """Fig. 3 step 3: every guard cell takes the value of the cell with the same
    global index in the box that owns it (faces, edges, corners, periodic wrap,
    guards wider than the neighbour)."""
    return scatter(gather(boxes, dec), dec)


def exchange_sum(boxes, dec):
    """Deposited-current mode: J_tot(X) = sum of J over every padded copy of the
    global cell X (all boxes, all positions), written back to every copy."""
    first = boxes[0]
    Nx, Ny, Nz = dec.N
    G = np.zeros(first.shape[:-3] + (Nz, Ny, Nx), dtype=first.dtype)
    for s in range(dec.nsub):
        ix, iy, iz = dec.global_index(s)
        Z, Y, X = np.meshgrid(iz, iy, ix, indexing="ij")
        for comp in np.ndindex(first.shape[:-3]):
            np.add.at(G[comp], (Z, Y, X), boxes[s][comp])
    return scatter(G, dec)


def step_local(Eb, Bb, Jb, dec, d, p, c, dt, jmode="replicated"):
    """One step of the decomposed method (Sec. 3.2, Fig. 3):
      1. currents made consistent (deposited: summed over copies; replicated:
         guard copies take the owner's value);
      2. each padded box advanced by step_global as if it were a periodic box
         of its own padded size (its own local FFT and its own modified k);
      3. guard cells of E and B replaced by the owners' values.
    Returns new (E boxes, B boxes, J boxes)."""
    if jmode == "deposited":
        Jb = exchange_sum(Jb, dec)
    elif jmode == "replicated":
        Jb = exchange_fill(Jb, dec)
    else:
        raise ValueError(jmode)
    En, Bn = [], []
    for s in range(dec.nsub):
        e, b = step_global(Eb[s], Bb[s], Jb[s], d, p, c, dt)
        En.append(e)
        Bn.append(b)
    return exchange_fill(En, dec), exchange_fill(Bn, dec), Jb


def run_local(Eb, Bb, Jb, dec, d, p, c, dt, nsteps, jmode="replicated"):
    """nsteps steps with J held fixed.  Deposited partial currents are summed
    once, at the first step; the summed (consistent) J is then held, i.e. the
    later steps use the replicated mode, which leaves a consistent J as is."""
    for i in range(nsteps):
        Eb, Bb, Jb = step_local(Eb, Bb, Jb, dec, d, p, c, dt, jmode if i == 0 else "replicated")
    return Eb, Bb, Jb


# --------------------------------------------------------------------------
# Sec. 5: the same local-FFT method for another initial-value problem, the
# diffusion (heat) equation du/dt = D lap u.  The Laplacian's symbol is
# -|[k]|^2 with the order-p modified wavenumbers of Sec. 3.1 (the symbol of the
# order-p first derivative applied twice, as in the curl-curl of the Maxwell
# update), and the step is its exact propagator.
# --------------------------------------------------------------------------
def heat_step_global(u, d, p, D, dt):
    """One step on a periodic box: u <- IFFT(exp(-D |[k]|^2 dt) FFT(u)); u is a
    real (Nz, Ny, Nx) array."""
    kx, ky, kz = k_grid(u.shape, d, p)
    g = np.exp(-D * (kx * kx + ky * ky + kz * kz) * dt)
    return np.fft.ifftn(g * np.fft.fftn(u)).real.copy()


def heat_run_local(ub, dec, d, p, D, dt, nsteps):
    """nsteps steps of the decomposed method (Sec. 3.2 / Fig. 3 applied to the
    heat equation): every padded box advanced by heat_step_global as its own
    periodic box, then its guard cells replaced by the owners' values."""
    for _ in range(nsteps):
        ub = exchange_fill([heat_step_global(ub[s], d, p, D, dt) for s in range(dec.nsub)], dec)
    return ub


# --------------------------------------------------------------------------
# Diagnostics
# --------------------------------------------------------------------------
def div_spectral(F, d, p):
    """i [k].F~ (spectral divergence with the same modified k)."""
    kx, ky, kz = k_grid(F.shape[1:], d, p)
    Fk = fft3(F)
    return 1j * (kx * Fk[0] + ky * Fk[1] + kz * Fk[2])


def energy(E, B, c):
    """W = 1/2 sum(|E|^2 + c^2 |B|^2) over the grid (eps0 = 1, mu0 = 1/c^2)."""
    return 0.5 * (np.sum(E * E) + c * c * np.sum(B * B))


def gauss_solution(rho, d, p):
    """Zero-mean E with i[k].E~ = rho~ and [k] x E~ = 0:  E~ = -i [k] rho~/|[k]|^2
    (rho must have zero mean; modes with |[k]| = 0 are set to 0)."""
    kx, ky, kz = k_grid(rho.shape, d, p)
    k2 = kx * kx + ky * ky + kz * kz
    rk = fft3(rho)
    safe = np.where(k2 == 0, 1.0, k2)
    f = np.where(k2 == 0, 0.0, -1j * rk / safe)
    return np.stack([ifft3(kx * f).real, ifft3(ky * f).real, ifft3(kz * f).real])


def project_transverse(a, kvec):
    """Component of vector a orthogonal to kvec (both length-3)."""
    kvec = np.asarray(kvec, dtype=np.float64)
    nk = kvec @ kvec
    if nk == 0:
        return np.asarray(a, dtype=np.float64)
    return a - (a @ kvec) / nk * kvec


def rel_l2(x, ref):
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    den = np.sqrt(np.sum(ref * ref))
    return float(np.sqrt(np.sum((x - ref) ** 2)) / (den if den > 0 else 1.0))
