"""Pins of the oracle's equilibrium, forcing and collision (Sec. II.A-II.B).

Each test checks the oracle against an identity fixed by the mathematics, not
against a retyped copy of the oracle's own formula.  Tests with the
``mutation`` fixture plant a plausible mistake in the oracle and check that the
pin catches it.
"""
import numpy as np
import pytest

import oracle as O

CS2 = 1.0 / 3.0
RNG = np.random.default_rng(7)


def _rand_state(rng, amp=0.05):
    t = O.tables()
    rho = 1 + 0.05 * rng.uniform(-1, 1)
    u = 0.08 * rng.uniform(-1, 1, 3)
    f = O.feq(rho, u) + amp * t["w"] * rng.uniform(-1, 1, 19)
    return f


def _meq_projection_ok():
    t = O.tables()
    for _ in range(20):
        rho = 1 + 0.1 * RNG.uniform(-1, 1)
        u = 0.1 * RNG.uniform(-1, 1, 3)
        if np.abs(O.meq(rho, u) - t["M"] @ O.feq(rho, u)).max() > 1e-14:
            return False
    return True


def test_moment_equilibrium_is_projection_of_equilibrium():
    """Eq. (8) with readings R1, R2 equals M f_eq exactly (Eq. (7), (27))."""
    assert _meq_projection_ok()


@pytest.mark.parametrize("k", [1, 2])
def test_meq_pin_catches_printed_typos(mutation, k):
    mutation(k)  # 1: printed m2_eq, 2: printed m4,6,8_eq = -3/2 rho u
    assert not _meq_projection_ok()


def _guo_moments_ok():
    t = O.tables()
    c = t["c"].astype(float)
    for _ in range(10):
        u = 0.1 * RNG.uniform(-1, 1, 3)
        F = 1e-3 * RNG.uniform(-1, 1, 3)
        Fb = O.guo(u, F)
        if abs(Fb.sum()) > 1e-17:
            return False
        if np.abs(Fb @ c - F).max() > 1e-17:
            return False
        if np.abs(np.einsum("i,ia,ib->ab", Fb, c, c) - (np.outer(u, F) + np.outer(F, u))).max() > 1e-17:
            return False
    return True


def test_guo_forcing_moments():
    """Eq. (9): zeroth moment 0, first F, second u F + F u (Guo et al. 2002)."""
    assert _guo_moments_ok()


def test_guo_pin_catches_dropped_velocity(mutation):
    mutation(3)
    assert not _guo_moments_ok()


def test_rest_state_is_fixed_point():
    t = O.tables()
    cfg = O.make_cfg(4, 4, 4, tau0=0.52, cs_smag=0.1)
    for rho in (0.9, 1.0, 1.1):
        out, tau, _ = O.collide_node(cfg, rho * t["w"], np.zeros(3))
        assert np.abs(out - rho * t["w"]).max() < 1e-15
        assert tau == pytest.approx(0.52, abs=1e-15)


def _conservation_ok(cfg):
    t = O.tables()
    c = t["c"].astype(float)
    for _ in range(20):
        f = _rand_state(RNG)
        F = 1e-4 * RNG.uniform(-1, 1, 3)
        out, _, _ = O.collide_node(cfg, f, F)
        if abs(out.sum() - f.sum()) > 1e-15:
            return False
        if np.abs(out @ c - (f @ c + F)).max() > 1e-15:
            return False
    return True


def test_collision_conserves_mass_and_adds_force_to_momentum():
    assert _conservation_ok(O.make_cfg(4, 4, 4, tau0=0.52, cs_smag=0.1))
    assert _conservation_ok(O.make_cfg(4, 4, 4, tau0=0.8, cs_smag=0.0))


def test_conserved_rates_do_not_matter():
    """Under moment-space forcing m*_j = m_j + F for any s_0, s_3, s_5, s_7 (reading R4)."""
    f = _rand_state(RNG)
    F = np.array([2e-4, -1e-4, 5e-5])
    base = O.collide_node(O.make_cfg(4, 4, 4), f, F)[0]
    rates = list(O.PAPER_RATES)
    for k in (0, 3, 5, 7):
        rates[k] = 1.7
    other = O.collide_node(O.make_cfg(4, 4, 4, rates=rates), f, F)[0]
    assert np.abs(base - other).max() < 1e-16


def test_bgk_limit():
    """Sec. II.A: with all rates equal the MRT operator is BGK (with Guo forcing)."""
    t = O.tables()
    c = t["c"].astype(float)
    tau = 0.73
    cfg = O.make_cfg(4, 4, 4, tau0=tau, cs_smag=0.0, rates=[1 / tau] * 19)
    for _ in range(10):
        f = _rand_state(RNG)
        F = 1e-4 * RNG.uniform(-1, 1, 3)
        rho = f.sum()
        u = (f @ c + F / 2) / rho
        bgk = f - (f - O.feq(rho, u)) / tau + (1 - 1 / (2 * tau)) * O.guo(u, F)
        out = O.collide_node(cfg, f, F)[0]
        assert np.abs(out - bgk).max() < 2e-16


def _regularised(rho, u, P):
    """f = f_eq + w/(2 cs^4) Q:P, whose non-equilibrium stress is exactly P."""
    t = O.tables()
    c = t["c"].astype(float)
    Q = np.einsum("ia,ib->iab", c, c) - CS2 * np.eye(3)
    return O.feq(rho, u) + t["w"] / (2 * CS2 ** 2) * np.einsum("iab,ab->i", Q, P)


def test_smagorinsky_relaxation_time_matches_printed_strain_rate():
    """tau_eff = tau0 + 3 C_smag |S| with |S| from the printed strain-rate root
    (Sec. II.B, Eq. (13), (14), (5)), evaluated on states with known Pi_neq."""
    for tau0, cs in ((0.52, 0.1), (0.5004, 0.1), (0.8, 0.3)):
        cfg = O.make_cfg(4, 4, 4, tau0=tau0, cs_smag=cs)
        C = cs * cs
        for _ in range(10):
            rho = 1 + 0.05 * RNG.uniform(-1, 1)
            u = 0.05 * RNG.uniform(-1, 1, 3)
            A = 1e-3 * RNG.uniform(-1, 1, (3, 3))
            P = A + A.T
            f = _regularised(rho, u, P)
            _, tau, _ = O.collide_node(cfg, f, np.zeros(3))
            Qh = np.sqrt((P * P).sum())
            S = (-tau0 * rho + np.sqrt((tau0 * rho) ** 2 + 18 * np.sqrt(2) * rho * C * Qh)) / (6 * rho * C)
            assert tau == pytest.approx(tau0 + 3 * C * S, rel=1e-13)


def test_smagorinsky_off_gives_molecular_tau():
    f = _rand_state(RNG)
    _, tau, _ = O.collide_node(O.make_cfg(4, 4, 4, tau0=0.61, cs_smag=0.0), f, np.zeros(3))
    assert tau == pytest.approx(0.61, abs=1e-15)


def test_bgk_pin_catches_missing_half_force_shift(mutation):
    """Eq. (11): the velocity of the equilibrium carries F/2; dropping it breaks the BGK limit."""
    mutation(4)
    with pytest.raises(AssertionError):
        test_bgk_limit()
