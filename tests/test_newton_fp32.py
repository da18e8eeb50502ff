"""The device's default of 4 Newton steps for u_tau (Sec. II.C, Eq. (20)).

The kernels run a fixed number of FP32 Newton steps from the viscous-sublayer
estimate.  This checks, with the same iteration in numpy float32, that 4 steps
reach the FP64 oracle's converged root to FP32 rounding over a range of nu0
and |u_hat| wider than that of the channel workloads (nu0 1e-5 .. 2e-2,
|u_hat| 1e-6 .. 0.3; the workloads use 4.6e-5 .. 6.7e-3 and up to 0.2), and
that 2 steps do not (3 reach rounding level; the fourth is the margin).
"""
import numpy as np

import oracle as O


def newton_fp32(nu, ua, steps, kappa=0.41, B=7.8, y=0.5):
    f = np.float32
    kappa, B, y, nu, ua = f(kappa), f(B), f(y), f(nu), f(ua)
    ut = np.sqrt(nu * ua / y).astype(f)
    for _ in range(steps):
        yp = y * ut / nu
        e1, e3 = np.exp(-yp / f(11)), np.exp(-yp / f(3))
        up = np.log1p(kappa * yp) / kappa - B * (np.expm1(-yp / f(11)) + yp / f(11) * e3)
        dup = f(1) / (f(1) + kappa * yp) + B * ((e1 - e3) / f(11) + yp / f(33) * e3)
        ut = (ut - (ut * up - ua) / (up + yp * dup)).astype(f)
    return float(ut)


def test_four_fp32_newton_steps_reach_the_root():
    worst = {2: 0.0, 4: 0.0}
    for nu in np.geomspace(1e-5, 2e-2, 16):
        cfg = O.make_cfg(4, 4, 4, tau0=0.5 + 3 * nu)
        for ua in np.geomspace(1e-6, 0.3, 20):
            st, ref = O.utau(cfg, ua)
            assert st == O.OK
            for k in worst:
                worst[k] = max(worst[k], abs(newton_fp32(nu, ua, k) - ref) / ref)
    assert worst[4] < 1e-6, worst
    assert worst[2] > 1e-5, worst


def newton_fp32_musker(nu, ua, steps, y=0.5):
    """The kernels' FP32 form of the Musker profile (differences from y+ = 0)."""
    f = np.float32
    nu, ua, y = f(nu), f(ua), f(y)
    t0 = f(-8.15 / 16.7)
    ut = np.sqrt(nu * ua / y).astype(f)
    for _ in range(steps):
        yp = y * ut / nu
        t = (f(2) * yp - f(8.15)) / f(16.7)
        up = f(5.424) * np.arctan2(yp * f(2 / 16.7), f(1) + t * t0) + \
            (f(9.6) * np.log1p(yp / f(10.6)) - f(2) * np.log1p(yp * (yp - f(8.15)) / f(86))) * f(0.4342944819)
        q = yp * yp - f(8.15) * yp + f(86)
        dup = f(5.424) * (f(2) / f(16.7)) / (f(1) + t * t) + f(0.4342944819) * (f(9.6) / (yp + f(10.6)) - f(2) * (f(2) * yp - f(8.15)) / q)
        ut = (ut - (ut * up - ua) / (up + yp * dup)).astype(f)
    return float(ut)


def test_four_fp32_newton_steps_reach_the_musker_root():
    """The same for the Musker law over first-cell y+ 0.01 .. 3000."""
    worst = {2: 0.0, 4: 0.0}
    for nu in np.geomspace(1e-5, 2e-2, 12):
        for yp in np.geomspace(0.01, 3000.0, 20):
            ut = yp * nu / 0.5
            ua = ut * O.uplus_musker(yp)
            cfg = O.make_cfg(4, 4, 4, tau0=0.5 + 3 * nu, wall_law=1)
            st, ref = O.utau(cfg, ua)
            assert st == O.OK
            for k in worst:
                worst[k] = max(worst[k], abs(newton_fp32_musker(nu, ua, k) - ref) / ref)
    assert worst[4] < 1e-6, worst
    assert worst[2] > 1e-5, worst
