"""CPU: the truncation harness's inputs are vacuum eigenmodes of PSATD-global
(Sec. 3.1): at infinite order a forward pulse is translated by c dt exactly,
and the broadband waves are divergence-free for the order-p [k]."""
import numpy as np

from oracle import psatd_oracle as O
from paper_1707_08500_amd import truncation as T


def test_pulses_move_forward_by_c_dt_at_infinite_order():
    N, d, c, dt = (48, 40, 56), (1.0, 1.0, 1.0), 1.0, 3.0
    E, B, J = T.resolution_fields(N, 12.0, width=3.0, c=c)
    E1, B1 = O.run_global(E, B, J, d, 0, c, dt, 1)
    shift = int(round(c * dt))
    # atol: the Nyquist mode has [k] = 0 (static) under the reading of the
    # infinite order; a 12-cell carrier under a 3-cell envelope puts ~1e-13
    # there
    # the x pulse (E_y, B_z) moves along x, the y pulse (E_z, B_x) along y,
    # the z pulse (E_x, B_y) along z; arrays are [z][y][x]
    axis_of = {1: 2, 2: 1, 0: 0}
    for comp, ax in axis_of.items():
        np.testing.assert_allclose(E1[comp], np.roll(E[comp], shift, axis=ax), atol=1e-11)
    for comp, ax in {2: 2, 0: 1, 1: 0}.items():
        np.testing.assert_allclose(B1[comp], np.roll(B[comp], shift, axis=ax), atol=1e-11)


def test_broadband_waves_are_divergence_free_for_order_p():
    N, d, p = (24, 24, 24), (1.0, 1.0, 1.0), 16
    kmod = [O.modified_k(N[u], d[u], p) for u in range(3)]
    E, B, J = T.smooth_fields(N, kmod, d)
    for F in (E, B):
        div = O.div_spectral(F, d, p)
        # fft3 is unnormalised: compare with the transform's own scale
        assert np.max(np.abs(div)) <= 1e-14 * np.prod(N) * np.max(np.abs(F))
