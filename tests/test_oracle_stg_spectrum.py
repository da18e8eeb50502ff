"""Pins of the per-row modified von Karman spectrum of the STG (Sec. III.A,
Eq. (25); reading R22: the spectrum of the cited STG, built per inlet row from
RANS k, omega and the wall distance) in the oracle.

Each pin comes from a property of the spectrum rather than its formula: the
weights are a partition of unity; the von Karman shape peaks where k equals the
most energetic wavenumber 2 pi / l_e (a calculus fact of r^4 / (1 + 2.4 r^2)^(17/6)),
with l_e the smaller of twice the wall distance and three RANS length scales;
it falls as k^(-5/3) in the inertial range; above 0.9 k_cut and near the
Kolmogorov wavenumber it is damped by the stated cut-off factors; and with the
spectrum the generated fluctuations still have the covariance R on every row.
"""
import numpy as np
import pytest

import oracle as O
from paper_2304_04214_amd import synthetic as S

CMU = 0.09


def _stg(ny, kmag, k, om, seed=0, R=None):
    n = len(kmag)
    mt = S.mode_table(n, ny / 2, seed_offset=seed)
    R = S.reynolds_stress(ny, 1.0) if R is None else R
    ab, boy = S.amp_bins(ny)
    return O.StgInputs(mt["q"], mt["sigma"], np.asarray(kmag, float), mt["d"], mt["phi"], mt["omega"],
                       np.zeros((3, ny)), R, ab, boy, k_rans=k, omega_rans=om)


def _density(q, kmag):
    return q / np.gradient(kmag)


def test_weights_sum_to_one_on_every_row():
    ny = 16
    k, om = S.rans_k_omega(ny, 0.005)
    kmag = np.geomspace(*S.spectrum_k_range(ny / 2), 120)
    cfg = O.make_cfg(4, ny, 4, xbc=1, ywall=2, tau0=0.5005)
    stg = _stg(ny, kmag, k, om)
    for y in range(ny):
        st, q = O.stg_weights(cfg, stg, y)
        assert st == O.OK
        assert abs(q.sum() - 1) < 1e-13 and (q > 0).all()


@pytest.mark.parametrize("y", [40, 100, 250, 350, 399, 759])
def test_peak_at_the_most_energetic_wavenumber(y):
    """Rows near the wall take l_e = 2 d_w, rows further out 3 l_t (omega chosen so both occur)."""
    ny = 800
    d_w = np.minimum(np.arange(ny) + 0.5, ny - np.arange(ny) - 0.5)
    k = np.full(ny, 1e-4)
    om = np.full(ny, np.sqrt(1e-4) / (CMU * 200.0))  # l_t = 200, 3 l_t = 600: the wall branch up to d_w = 300
    kmag = np.geomspace(1e-3, 0.3, 3000)  # well below 0.9 k_cut and k_eta
    cfg = O.make_cfg(4, ny, 4, xbc=1, ywall=2, tau0=0.5 + 3e-5)
    st, q = O.stg_weights(cfg, _stg(ny, kmag, k, om), y)
    assert st == O.OK
    l_e = min(2 * d_w[y], 600.0)
    k_peak = kmag[np.argmax(_density(q, kmag))]
    assert abs(np.log(k_peak / (2 * np.pi / l_e))) < 2 * np.log(kmag[1] / kmag[0])


def test_inertial_range_slope():
    ny = 400
    k = np.full(ny, 1e-4)
    om = np.full(ny, np.sqrt(1e-4) / (CMU * 200.0))
    kmag = np.geomspace(0.5, 2.5, 200)
    cfg = O.make_cfg(4, ny, 4, xbc=1, ywall=2, tau0=0.5 + 3e-6)
    st, q = O.stg_weights(cfg, _stg(ny, kmag, k, om), ny // 2)  # l_e = 400: k / k_e ~ 30 .. 160
    assert st == O.OK
    e = _density(q, kmag)
    slope = np.polyfit(np.log(kmag[5:-5]), np.log(e[5:-5]), 1)[0]
    assert abs(slope + 5 / 3) < 2e-3


def test_cut_off_damping_above_0_9_k_cut():
    """On the unit lattice l_cut = 2, k_cut = pi: above 0.9 pi the -5/3 law is damped
    by exp(-(4 (k - 0.9 pi) / pi)^3)."""
    ny = 400
    k = np.full(ny, 1e-4)
    om = np.full(ny, np.sqrt(1e-4) / (CMU * 200.0))
    kmag = np.geomspace(2.0, 4.5, 400)
    cfg = O.make_cfg(4, ny, 4, xbc=1, ywall=2, tau0=0.5 + 3e-6)
    st, q = O.stg_weights(cfg, _stg(ny, kmag, k, om), ny // 2)
    assert st == O.OK
    e = _density(q, kmag)
    i0 = np.searchsorted(kmag, 2.5)
    for i in np.searchsorted(kmag, [3.0, 3.3, 3.8, 4.3]):
        damp = e[i] / (e[i0] * (kmag[i] / kmag[i0]) ** (-5 / 3))
        ref = np.exp(-(4 * (kmag[i] - 0.9 * np.pi) / np.pi) ** 3)
        assert abs(damp / ref - 1) < 5e-3, (kmag[i], damp, ref)


def test_kolmogorov_damping():
    """With eta = (nu^3 / eps)^(1/4), eps = C_mu k omega, of order one cell, the -5/3 law
    below the cut-off is damped by exp(-(12 k / k_eta)^2), k_eta = 2 pi / eta."""
    ny = 400
    nu = 1.7e-3  # eta ~ 1
    k = np.full(ny, 1e-4)
    om = np.full(ny, np.sqrt(1e-4) / (CMU * 200.0))
    kmag = np.geomspace(0.25, 0.6, 400)
    cfg = O.make_cfg(4, ny, 4, xbc=1, ywall=2, tau0=0.5 + 3 * nu)
    st, q = O.stg_weights(cfg, _stg(ny, kmag, k, om), ny // 2)
    assert st == O.OK
    e = _density(q, kmag)
    eta = (nu ** 3 / (CMU * 1e-4 * om[0])) ** 0.25
    k_eta = 2 * np.pi / eta
    i0 = 0
    assert 0.5 < 12 * 0.5 / k_eta < 2  # the damping matters in this range
    for i in np.searchsorted(kmag, [0.35, 0.45, 0.55]):
        damp = e[i] / (e[i0] * (kmag[i] / kmag[i0]) ** (-5 / 3))
        ref = np.exp(-(12 * kmag[i] / k_eta) ** 2) / np.exp(-(12 * kmag[i0] / k_eta) ** 2)
        assert abs(damp / ref - 1) < 2e-2, (kmag[i], damp, ref)


def test_covariance_is_R_with_the_row_spectrum():
    """Sum_n q^n(y) = 1 keeps E[u' u'^T] = R on every row (as for one table)."""
    ny, nz = 8, 1
    cfg = O.make_cfg(4, ny, nz, xbc=1, ywall=2, tau0=0.5005)
    R = S.reynolds_stress(ny, 1.0)
    k, om = S.rans_k_omega(ny, 1.0)
    kmag = np.geomspace(*S.spectrum_k_range(ny / 2), 50)
    samples = []
    for seed in range(400):
        st, uin = O.stg_plane(cfg, _stg(ny, kmag, k, om, seed=seed, R=R), 0.0)
        assert st in (O.OK, O.ERR_MACH)
        samples.append(uin[:, :, 0])
    X = np.array(samples)
    n = X.shape[0]
    for y in (0, 3, 7):
        u = X[:, :, y]
        cov = (u.T @ u) / n
        Rm = np.array([[R[0, y], R[1, y], R[3, y]], [R[1, y], R[2, y], R[4, y]], [R[3, y], R[4, y], R[5, y]]])
        for a in range(3):
            for b in range(3):
                se = np.sqrt(np.var(u[:, a] * u[:, b]) / n)
                assert abs(cov[a, b] - Rm[a, b]) < 4 * se + 1e-12


def test_rows_differ_and_invalid_inputs_are_rejected():
    ny = 12
    cfg = O.make_cfg(4, ny, 4, xbc=1, ywall=2, tau0=0.5005)
    k, om = S.rans_k_omega(ny, 0.005)
    kmag = np.geomspace(*S.spectrum_k_range(ny / 2), 64)
    _, q0 = O.stg_weights(cfg, _stg(ny, kmag, k, om), 0)
    _, q5 = O.stg_weights(cfg, _stg(ny, kmag, k, om), 5)
    assert np.abs(q0 - q5).max() > 1e-3  # the near-wall row has smaller eddies
    bad = kmag.copy()
    bad[[10, 11]] = bad[[11, 10]]
    assert O.stg_weights(cfg, _stg(ny, bad, k, om), 0)[0] == O.ERR_ARG
    k2 = k.copy()
    k2[3] = 0.0
    assert O.stg_weights(cfg, _stg(ny, kmag, k2, om), 3)[0] == O.ERR_ARG
    cfgp = O.make_cfg(4, ny, 4, xbc=1, ywall=0, tau0=0.5005)
    assert O.stg_weights(cfgp, _stg(ny, kmag, k, om), 0)[0] == O.ERR_ARG


@pytest.mark.parametrize("mutation,test", [(13, test_inertial_range_slope), (14, lambda: test_peak_at_the_most_energetic_wavenumber(399))])
def test_planted_mistakes_fail(mutation, test):
    O.set_mutation(mutation)
    try:
        with pytest.raises(AssertionError):
            test()
    finally:
        O.set_mutation(0)
