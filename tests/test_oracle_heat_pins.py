"""Pins of the oracle's heat-equation step (Sec. 5: the local-FFT method applied
to the diffusion equation du/dt = D lap u) against the real-space semi-discrete
operator, closed forms and invariants.  CPU only."""
import numpy as np
import pytest
from scipy.linalg import expm

from oracle import psatd_oracle as O
from paper_1707_08500_amd import synth


def fd_matrix(N, du, p):
    """Circulant order-p centred first-derivative matrix on N periodic points:
    (D f)_i = (1/du) sum_j w_j (f_{i+j} - f_{i-j}) (the weights are pinned
    against the textbook table by the Maxwell oracle's P2)."""
    D = np.zeros((N, N))
    for j, wj in enumerate(O.fd_weights(p), start=1):
        for i in range(N):
            D[i, (i + j) % N] += wj / du
            D[i, (i - j) % N] -= wj / du
    return D


@pytest.mark.parametrize("p", [2, 4, 8])
def test_H1_step_is_the_semi_discrete_propagator(p):
    """expm(D dt L) with L = Dx^2 + Dy^2 + Dz^2 built from the real-space
    order-p first-derivative stencils, on an anisotropic 6 x 5 x 4 grid."""
    Nx, Ny, Nz = 6, 5, 4
    d = (0.7, 1.1, 1.3)
    Dc, dt = 0.37, 0.9
    r = np.random.default_rng(40 + p)
    u = r.normal(size=(Nz, Ny, Nx))
    Dx, Dy, Dz = (fd_matrix(Nx, d[0], p), fd_matrix(Ny, d[1], p), fd_matrix(Nz, d[2], p))
    Ix, Iy, Iz = np.eye(Nx), np.eye(Ny), np.eye(Nz)
    L = (np.kron(Dz @ Dz, np.kron(Iy, Ix)) + np.kron(Iz, np.kron(Dy @ Dy, Ix)) +
         np.kron(Iz, np.kron(Iy, Dx @ Dx)))
    ref = (expm(Dc * dt * L) @ u.ravel()).reshape(u.shape)
    got = O.heat_step_global(u, d, p, Dc, dt)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("p", [0, 8])
def test_H2_single_mode_decays_by_its_symbol(p):
    """cos(k.x + phi) decays as exp(-D |[k]|^2 t); at infinite order [k] = k,
    the continuum heat solution of a resolved mode."""
    N = (16, 12, 10)
    d = (1.0, 0.5, 2.0)
    m = (3, -2, 1)
    Dc, dt, n = 0.2, 0.3, 5
    x = [np.arange(N[u]) * d[u] for u in range(3)]
    Z, Y, X = np.meshgrid(x[2], x[1], x[0], indexing="ij")
    k = [2 * np.pi * m[u] / (N[u] * d[u]) for u in range(3)]
    u0 = np.cos(k[0] * X + k[1] * Y + k[2] * Z + 0.4)
    if p == 0:
        k2 = sum(kk * kk for kk in k)
    else:
        k2 = sum(O.modified_k(N[u], d[u], p)[m[u] % N[u]] ** 2 for u in range(3))
    u = u0
    for _ in range(n):
        u = O.heat_step_global(u, d, p, Dc, dt)
    assert np.abs(u - np.exp(-Dc * k2 * n * dt) * u0).max() <= 1e-13


def test_H3_invariants():
    """Mean conserved; semigroup (two steps of dt = one of 2 dt); D = 0 is the
    identity; the L2 norm does not grow."""
    r = np.random.default_rng(43)
    u = r.normal(size=(8, 6, 10))
    d, p, Dc, dt = (1.0, 1.0, 1.0), 16, 0.25, 0.5
    one = O.heat_step_global(u, d, p, Dc, dt)
    two = O.heat_step_global(one, d, p, Dc, dt)
    big = O.heat_step_global(u, d, p, Dc, 2 * dt)
    assert abs(one.mean() - u.mean()) <= 1e-15
    assert np.abs(two - big).max() <= 1e-14
    assert np.abs(O.heat_step_global(u, d, p, 0.0, dt) - u).max() <= 1e-14
    assert np.linalg.norm(one) < np.linalg.norm(u)


def test_H4_local_reductions_and_guard_trend():
    """One box without guards is the global step; boxes whose padded length is
    the grid length are cyclic shifts of it; on smooth data the local-vs-global
    difference falls with the guard width."""
    N = (24, 24, 24)
    d, p, Dc, dt, n = (1.0, 1.0, 1.0), 16, 0.3, 0.5, 3
    r = np.random.default_rng(44)
    u = r.normal(size=(N[2], N[1], N[0]))
    ref = u
    for _ in range(n):
        ref = O.heat_step_global(ref, d, p, Dc, dt)
    dec1 = O.Decomposition(N, [[0, 0, 0]], [list(N)], [[0, 0, 0]])
    got1 = O.gather(O.heat_run_local(O.scatter(u, dec1), dec1, d, p, Dc, dt, n), dec1)
    assert np.abs(got1 - ref).max() <= 1e-13
    lo, nn, g = synth.uniform_decomposition(N, (2, 2, 2), 6)
    dec2 = O.Decomposition(N, lo, nn, g)
    got2 = O.gather(O.heat_run_local(O.scatter(u, dec2), dec2, d, p, Dc, dt, n), dec2)
    assert np.abs(got2 - ref).max() <= 1e-12
    # smooth data, 3 x 3 x 3 boxes of 8: error falls with the guard width
    ms, amps, phases = synth.wave_parameters(case=44, count=3, mmax=2)
    s = sum(synth.plane_wave(N, m, a, ph)[0] for m, a, ph in zip(ms, amps, phases))
    s = s + 0.5 * synth.current_pulses(N, d, case=44, count=1, sigma=3.0)[0]
    sref = s
    for _ in range(n):
        sref = O.heat_step_global(sref, d, p, Dc, dt)
    errs = []
    for gw in (2, 4, 8):
        lo, nn, g = synth.uniform_decomposition(N, (3, 3, 3), gw)
        dec = O.Decomposition(N, lo, nn, g)
        got = O.gather(O.heat_run_local(O.scatter(s, dec), dec, d, p, Dc, dt, n), dec)
        errs.append(O.rel_l2(got, sref))
    assert errs[0] > errs[1] > errs[2]
