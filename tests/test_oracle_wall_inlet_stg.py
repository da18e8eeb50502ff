"""Pins of the oracle's wall model (Sec. II.C), regularised STG inlet and mode
sum (Sec. III.A), against limits, identities and the paper's printed values."""
import os

import numpy as np
import pytest

import oracle as O
from paper_2304_04214_amd import synthetic as S

CS2 = 1.0 / 3.0
KAPPA, B = 0.41, 7.8
GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
RNG = np.random.default_rng(11)


# ---------------- Reichardt law, Eq. (16) ----------------

def test_reichardt_viscous_limit():
    """u+ = y+ + O(y+^2) at the wall: slope 1 at y+ = 0 (viscous sublayer)."""
    assert O.uplus(0.0) == 0.0
    assert O.duplus(0.0) == pytest.approx(1.0, abs=1e-15)
    assert O.uplus(1e-4) == pytest.approx(1e-4, rel=1e-4)


def test_reichardt_pin_catches_printed_form(mutation):
    mutation(5)
    assert O.uplus(1e-4) != pytest.approx(1e-4, rel=1e-2)


def test_reichardt_values_match_closed_form():
    """u+ at y+ = 1, 50, 260 against the closed form of Eq. (16) (reading R6) evaluated by
    hand (tests/golden/reichardt_uplus.txt, six significant digits)."""
    rows = np.loadtxt(os.path.join(GOLDEN, "reichardt_uplus.txt"))
    for yp, up in rows:
        assert O.uplus(yp) == pytest.approx(up, rel=1e-5), yp


@pytest.mark.parametrize("k", [17, 18])
def test_reichardt_value_pin_catches_buffer_layer_misreadings(mutation, k):
    """Misreadings of the buffer-layer term, planted in u+ and du+ alike (17: e^(-y+/2) for
    e^(-y+/3); 18: y+/10 for y+/11), fail the value pin.  Mutation 17 keeps the viscous
    slope, the log-law limit and the derivative check, so only the value pin sees it."""
    mutation(k)
    rows = np.loadtxt(os.path.join(GOLDEN, "reichardt_uplus.txt"))
    assert any(O.uplus(yp) != pytest.approx(up, rel=1e-5) for yp, up in rows)
    if k == 17:
        assert O.duplus(0.0) == pytest.approx(1.0, abs=1e-15)
        for yp in (0.3, 11.0, 50.0):
            h = 1e-5 * max(yp, 1.0)
            assert O.duplus(yp) == pytest.approx((O.uplus(yp + h) - O.uplus(yp - h)) / (2 * h), rel=1e-8)


def test_reichardt_log_law_limit():
    """u+ -> ln(y+)/kappa + ln(kappa)/kappa + B for y+ -> infinity."""
    C = np.log(KAPPA) / KAPPA + B
    for yp in (1e5, 1e6):
        assert O.uplus(yp) == pytest.approx(np.log(yp) / KAPPA + C, abs=2e-4 * 1e5 / yp + 1e-5)
    assert O.duplus(1e6) * 1e6 == pytest.approx(1 / KAPPA, rel=1e-5)


def test_reichardt_derivative_matches_central_differences():
    for yp in (0.3, 2.0, 11.0, 50.0, 260.0, 5000.0):
        h = 1e-5 * max(yp, 1.0)
        fd = (O.uplus(yp + h) - O.uplus(yp - h)) / (2 * h)
        assert O.duplus(yp) == pytest.approx(fd, rel=1e-8)


def test_first_cell_yplus_matches_paper():
    """Sec. IV.B prints first-cell y+ for three Re_tau and three resolutions;
    they follow from y_perp = 1/2 (halfway walls) and delta = H/2."""
    rows = np.loadtxt(os.path.join(GOLDEN, "first_cell_yplus.txt"))
    cfg = O.make_cfg(4, 4, 4)
    for re_tau, H, yp_printed in rows:
        delta = H / 2
        yp = cfg.y_wall * re_tau / delta  # y+ = y u_tau / nu, nu = u_tau delta / Re_tau
        assert yp == pytest.approx(yp_printed, rel=5e-3)


@pytest.mark.parametrize("tau0,uhat", [(0.5004270558446486, 0.06), (0.5001393543659287, 0.055),
                                       (0.5002787087318575, 0.05), (0.52, 0.03), (0.52, 1e-5),
                                       (0.8, 0.2), (0.5001, 1e-3), (0.52, 1e-9), (0.52, 1e-12)])
def test_newton_solves_wall_law(tau0, uhat):
    cfg = O.make_cfg(4, 4, 4, tau0=tau0)
    nu = (tau0 - 0.5) / 3
    st, ut = O.utau(cfg, uhat)
    assert st == O.OK
    assert ut * O.uplus(cfg.y_wall * ut / nu) == pytest.approx(uhat, rel=1e-13)
    if uhat < 1e-6:  # viscous sublayer: u_tau^2 y / nu = u_hat to leading order
        assert ut == pytest.approx(np.sqrt(nu * uhat / cfg.y_wall), rel=1e-5)


def test_newton_round_trip():
    cfg = O.make_cfg(4, 4, 4, tau0=0.5004)
    nu = 0.0004 / 3
    for ut_star in (1e-4, 1e-3, 4.45e-3, 2e-2):
        uhat = ut_star * O.uplus(0.5 * ut_star / nu)
        st, ut = O.utau(cfg, uhat)
        assert st == O.OK and ut == pytest.approx(ut_star, rel=1e-12)


# ---------------- wall force, Eq. (18)-(21) ----------------

def test_wall_force_direction_and_magnitude():
    cfg = O.make_cfg(4, 4, 4, tau0=0.5004)
    nu = 0.0004 / 3
    for top in (0, 1):
        for _ in range(10):
            uw = np.array([0.05, 0.01, 0.02]) * RNG.uniform(0.2, 1.0, 3) * np.sign(RNG.uniform(-1, 1, 3))
            u2 = uw * RNG.uniform(0.9, 1.5, 3)
            rho = 1 + 0.02 * RNG.uniform(-1, 1)
            st, F, ut = O.wall_force(cfg, rho, uw, u2, top)
            assert st == O.OK
            t = np.array([u2[0], 0.0, u2[2]])
            e = t / np.linalg.norm(t)
            uhat = uw @ e
            # friction opposes the projected flow, magnitude rho u_tau^2, wall-parallel
            assert F[1] == 0.0
            assert np.linalg.norm(F) == pytest.approx(rho * ut * ut, rel=1e-14)
            assert F @ e == pytest.approx(-np.sign(uhat) * rho * ut * ut, rel=1e-14)
            assert ut * O.uplus(0.5 * ut / nu) == pytest.approx(abs(uhat), rel=1e-12)


def test_wall_force_zero_cases():
    cfg = O.make_cfg(4, 4, 4)
    st, F, _ = O.wall_force(cfg, 1.0, np.array([0.05, 0, 0]), np.array([0.0, 0.03, 0.0]), 0)
    assert st == O.OK and np.all(F == 0)
    st, F, _ = O.wall_force(cfg, 1.0, np.array([0.0, 0.01, 0.05]), np.array([0.05, 0.0, 0.0]), 0)
    assert st == O.OK and np.all(F == 0)


# ---------------- regularised inlet, Eq. (26)-(31) ----------------

def _Q():
    c = O.tables()["c"].astype(float)
    return c, np.einsum("ia,ib->iab", c, c) - CS2 * np.eye(3)


def test_inlet_moments():
    c, Q = _Q()
    for _ in range(20):
        rho = 1 + 0.05 * RNG.uniform(-1, 1)
        u = 0.05 * RNG.uniform(-1, 1, 3)
        f = O.feq(rho, u) + 0.02 * O.tables()["w"] * RNG.uniform(-1, 1, 19)
        uin = np.array([0.1, 0.0, 0.0]) + 0.01 * RNG.uniform(-1, 1, 3)
        out, rin = O.inlet_node(f, uin)
        assert out.sum() == pytest.approx(rin, rel=1e-15)
        assert np.abs(out @ c - rin * uin).max() < 1e-16


def _zou_he_ok():
    for _ in range(20):
        rho = 1 + 0.05 * RNG.uniform(-1, 1)
        uin = np.array([0.1, 0.01, -0.02]) * RNG.uniform(0.5, 1.5, 3)
        f = O.feq(rho, uin)
        _, rin = O.inlet_node(f, uin)
        if abs(rin - rho) > 1e-15:
            return False
    return True


def test_zou_he_density_recovers_equilibrium_density():
    """Known populations at equilibrium with the prescribed velocity give rho_in = rho exactly."""
    assert _zou_he_ok()


def test_zou_he_pin_catches_printed_labels(mutation):
    mutation(6)
    assert not _zou_he_ok()


def _regularised_fixed_point_ok():
    c, Q = _Q()
    w = O.tables()["w"]
    for _ in range(20):
        rho = 1 + 0.05 * RNG.uniform(-1, 1)
        uin = np.array([0.1, 0.0, 0.0]) + 0.01 * RNG.uniform(-1, 1, 3)
        A = 1e-3 * RNG.uniform(-1, 1, (3, 3))
        P = A + A.T
        f = O.feq(rho, uin) + w / (2 * CS2 ** 2) * np.einsum("iab,ab->i", Q, P)
        out, rin = O.inlet_node(f, uin)
        if np.abs(out - f).max() > 1e-15 or abs(rin - rho) > 1e-15:
            return False
    return True


def test_regularised_state_is_a_fixed_point_of_the_inlet():
    """A state f_eq + w/(2cs^4) Q:P is rebuilt exactly from its c_x <= 0 part (reading R7)."""
    assert _regularised_fixed_point_ok()


def test_regularised_pin_catches_printed_factor(mutation):
    mutation(7)
    assert not _regularised_fixed_point_ok()


# ---------------- STG, Eq. (22)-(25) ----------------

def test_cholesky_reproduces_R():
    for y in range(16):
        R = S.reynolds_stress(16, 1.0)[:, y]
        a = O.cholesky(R)
        L = np.array([[a[0], 0, 0], [a[1], a[2], 0], [a[3], a[4], a[5]]])
        Rm = np.array([[R[0], R[1], R[3]], [R[1], R[2], R[4]], [R[3], R[4], R[5]]])
        assert np.abs(L @ L.T - Rm).max() < 1e-14
    R = np.array([2.0, 0.3, 1.5, -0.4, 0.2, 1.1])
    a = O.cholesky(R)
    L = np.array([[a[0], 0, 0], [a[1], a[2], 0], [a[3], a[4], a[5]]])
    assert np.abs(L @ L.T - np.array([[2, .3, -.4], [.3, 1.5, .2], [-.4, .2, 1.1]])).max() < 1e-14


def _stg(ny, n_modes, seed, u_rans=None, R=None):
    mt = S.mode_table(n_modes, ny / 2, seed_offset=seed)
    if u_rans is None:
        u_rans = np.zeros((3, ny))
    if R is None:
        R = S.reynolds_stress(ny, 1.0)
    ab, boy = S.amp_bins(ny)
    return O.StgInputs(mt["q"], mt["sigma"], mt["kmag"], mt["d"], mt["phi"], mt["omega"], u_rans, R, ab, boy)


def test_stg_single_mode_is_the_closed_form():
    """Eq. (22)-(25) with one mode (q = 1): u_in(y, z, t) = U(y) + s_b a(y) sqrt(6) sigma
    cos(k (d_y y_c + d_z z) + omega t + phi), y_c = iy + 1/2 and z = iz (lattice units), a the
    lower Cholesky factor of R(y) (numpy's), with a full R (R31, R32 != 0) and per-row s_b."""
    ny, nz, t = 8, 6, 37.0
    cfg = O.make_cfg(4, ny, nz, ywall=2, xbc=1, tau0=0.52)
    d = np.array([0.48, -0.6, 0.64])
    d /= np.linalg.norm(d)
    sigma = np.cross(d, [0.0, 0.0, 1.0])
    sigma /= np.linalg.norm(sigma)
    k, phi, omega = 0.7, 1.3, 0.021
    eta = (np.arange(ny) + 0.5) / (ny / 2) - 1
    R = np.stack([1.0 + 3 * eta ** 2, eta, 0.5 + 0.5 * eta ** 2, 0.2 * eta, -0.1 + 0.05 * eta, 0.7 + 0.8 * eta ** 2])
    R *= 1e-4
    U = np.zeros((3, ny))
    U[0] = 0.05 + 0.01 * eta ** 2
    amp_bin = np.array([1.0, 0.5, 2.0])
    bin_of_y = np.array([0, 0, 1, 1, 2, 2, 0, 1], dtype=np.int32)
    stg = O.StgInputs([1.0], sigma[:, None], [k], d[:, None], [phi], [omega], U, R, amp_bin, bin_of_y)
    st, uin = O.stg_plane(cfg, stg, t)
    assert st == O.OK
    ref = np.zeros((3, ny, nz))
    for y in range(ny):
        Ry = np.array([[R[0, y], R[1, y], R[3, y]], [R[1, y], R[2, y], R[4, y]], [R[3, y], R[4, y], R[5, y]]])
        a = np.linalg.cholesky(Ry)
        for z in range(nz):
            v = np.sqrt(6.0) * sigma * np.cos(k * (d[1] * (y + 0.5) + d[2] * z) + omega * t + phi)
            ref[:, y, z] = U[:, y] + amp_bin[bin_of_y[y]] * (a @ v)
    assert np.abs(uin - ref).max() <= 1e-14


def test_stg_ensemble_covariance_converges_to_R():
    """Eq. (25): with |sigma| = 1, sigma . d = 0, sum q = 1 and random phases the
    fluctuation has E[v v^T] = I, so E[u' u'^T] = a a^T = R (reading R12)."""
    ny, nz = 8, 1
    cfg = O.make_cfg(4, ny, nz, xbc=1)
    R = S.reynolds_stress(ny, 1.0)
    samples = []
    for seed in range(400):
        stg = _stg(ny, 50, seed, R=R)
        st, uin = O.stg_plane(cfg, stg, 0.0)  # unit-scale R trips the Mach flag; values are still set
        assert st in (O.OK, O.ERR_MACH)
        samples.append(uin[:, :, 0])
    X = np.array(samples)  # [n, 3, ny]
    n = X.shape[0]
    for y in (0, 3, 7):
        u = X[:, :, y]
        mean = u.mean(0)
        cov = (u.T @ u) / n
        Rm = np.array([[R[0, y], R[1, y], R[3, y]], [R[1, y], R[2, y], R[4, y]], [R[3, y], R[4, y], R[5, y]]])
        # standard errors of second moments from the samples themselves
        for a in range(3):
            se_m = np.sqrt(np.var(u[:, a]) / n)
            assert abs(mean[a]) < 4 * se_m + 1e-12
            for b in range(3):
                se = np.sqrt(np.var(u[:, a] * u[:, b]) / n)
                assert abs(cov[a, b] - Rm[a, b]) < 4 * se + 1e-12


def test_stg_time_mean_is_zero_and_mean_inflow_added():
    ny, nz = 6, 4
    cfg = O.make_cfg(4, ny, nz, xbc=1)
    U = np.zeros((3, ny))
    U[0] = 0.1
    stg = _stg(ny, 40, 3, u_rans=U, R=S.reynolds_stress(ny, 1e-4))
    acc = np.zeros((3, ny, nz))
    T = 3000
    for t in range(0, T):
        st, uin = O.stg_plane(cfg, stg, float(t))
        assert st == O.OK
        acc += uin
    m = acc / T
    assert np.abs(m[0] - 0.1).max() < 2e-3
    assert np.abs(m[1:]).max() < 2e-3


def test_stg_mach_guard():
    ny, nz = 4, 2
    cfg = O.make_cfg(4, ny, nz, xbc=1)
    U = np.zeros((3, ny))
    U[0] = 0.2  # above 0.3 c_s = 0.1732
    st, _ = O.stg_plane(cfg, _stg(ny, 10, 1, u_rans=U, R=S.reynolds_stress(ny, 1e-8)), 0.0)
    assert st == O.ERR_MACH
