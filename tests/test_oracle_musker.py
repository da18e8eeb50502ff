"""Pins of the Musker law of the wall (reading R21 of Sec. II.C, the alternative
the paper names to the Reichardt law) in the oracle, by the physics it must
reproduce: u+ = y+ in the viscous sublayer, the logarithmic law (kappa 0.41,
intercept near 5) in the log layer, agreement with the Reichardt law there,
the published explicit profile up to its additive constant, a derivative that
matches differences, and a Newton solve of Eq. (20) that inverts it."""
import numpy as np
import pytest

import oracle as O


def test_viscous_sublayer():
    assert O.uplus_musker(0.0) == 0.0
    for yp in (1e-8, 1e-4):
        assert abs(O.uplus_musker(yp) / yp - 1.0) < 1e-3
    for yp in (0.5, 1.0, 2.0):
        assert abs(O.uplus_musker(yp) / yp - 1.0) < 0.03


def test_log_layer():
    for yp in (100.0, 1e3, 1e4):
        assert abs(O.uplus_musker(yp) - (np.log(yp) / 0.41 + 5.0)) < 0.2
    # slope d u+ / d ln y+ -> 1 / kappa
    yp = 1e4
    s = (O.uplus_musker(yp * 1.001) - O.uplus_musker(yp / 1.001)) / (2 * np.log(1.001))
    assert abs(s * 0.41 - 1.0) < 0.01


def test_published_profile_up_to_its_constant():
    """The explicit profile as usually printed, with its rounded constant -3.52, differs
    from the oracle's by one constant (the oracle's constant gives u+(0) = 0)."""
    yp = np.array([0.0, 0.3, 3.0, 11.0, 21.25, 40.0, 400.0, 4e4])
    printed = 5.424 * np.arctan((2 * yp - 8.15) / 16.7) + np.log10((yp + 10.6) ** 9.6 / (yp * yp - 8.15 * yp + 86) ** 2) \
        - 3.52
    d = printed - np.array([O.uplus_musker(v) for v in yp])
    assert np.ptp(d) < 1e-12
    assert abs(d[0] + 0.00867) < 1e-4


def test_close_to_reichardt_in_the_log_layer():
    for yp in np.geomspace(30, 1e4, 12):
        assert abs(O.uplus_musker(yp) / O.uplus(yp) - 1) < 0.05


def test_derivative_matches_differences():
    for yp in np.geomspace(0.1, 1e4, 25):
        h = 1e-5 * max(1.0, yp)
        fd = (O.uplus_musker(yp + h) - O.uplus_musker(yp - h)) / (2 * h)
        assert abs(O.duplus_musker(yp) - fd) < 1e-7 * max(1.0, abs(fd))


@pytest.mark.parametrize("tau0", [0.5001, 0.505, 0.56])
def test_newton_inverts_the_musker_law(tau0):
    cfg = O.make_cfg(4, 4, 4, tau0=tau0, wall_law=1)
    nu = (tau0 - 0.5) / 3
    for ut in np.geomspace(1e-7, 2e-2, 12):
        ua = ut * O.uplus_musker(cfg.y_wall * ut / nu)
        st, got = O.utau(cfg, ua)
        assert st == O.OK and abs(got / ut - 1) < 1e-12


def test_planted_sign_error_fails():
    O.set_mutation(12)
    try:
        off = abs(O.uplus_musker(0.0))
    finally:
        O.set_mutation(0)
    assert off > 0.1
