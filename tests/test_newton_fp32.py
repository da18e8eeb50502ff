"""The device's default of 4 Newton steps for u_tau (Sec. II.C, Eq. (20)).

The kernels run a fixed number of FP32 Newton steps from the viscous-sublayer
estimate, the Reichardt law evaluated from base-2 transcendentals.  This checks,
with the same evaluation and iteration in numpy float32, that 4 steps
reach the FP64 oracle's converged root to FP32 rounding over a range of nu0
and |u_hat| wider than that of the channel workloads (nu0 1e-5 .. 2e-2,
|u_hat| 1e-6 .. 0.3; the workloads use 4.6e-5 .. 6.7e-3 and up to 0.2), and
that 2 steps do not (3 reach rounding level; the fourth is the margin).
"""
import numpy as np

import oracle as O


def reichardt_fp32(yp, kappa, B):
    """The kernels' FP32 evaluation of the Reichardt law: e^x as 2^(x log2 e), log(1 + x) from
    log2 with Goldberg's correction x log(u) / (u - 1), u = fl(1 + x), and e^t - 1 by its Taylor
    series to t^6 for |t| = y+/11 < 0.3 (numpy's exp2 / log2 round correctly; the hardware's are
    within about 1 ulp)."""
    f = np.float32
    t = yp * f(-1 / 11)
    e1 = np.exp2(t * f(1.44269504088896341)).astype(f)
    e3 = np.exp2(yp * f(-1 / 3) * f(1.44269504088896341)).astype(f)
    series = t * (f(1) + t * (f(0.5) + t * (f(1 / 6) + t * (f(1 / 24) + t * (f(1 / 120) + t * f(1 / 720))))))
    em1 = series if t > f(-0.3) else e1 - f(1)
    x = kappa * yp
    u = f(1) + x
    d = u - f(1)
    l1p = x if d == 0 else (np.log2(u).astype(f) * f(0.693147180559945309)) * (x * (f(1) / d))
    up = l1p * (f(1) / kappa) - B * (em1 + yp * f(1 / 11) * e3)
    dup = f(1) / (f(1) + x) + B * ((e1 - e3) * f(1 / 11) + yp * f(1 / 33) * e3)
    return f(up), f(dup)


def newton_fp32(nu, ua, steps, kappa=0.41, B=7.8, y=0.5):
    f = np.float32
    kappa, B, y, nu, ua = f(kappa), f(B), f(y), f(nu), f(ua)
    ut = np.sqrt(nu * ua * (f(1) / y)).astype(f)
    inv_nu = f(1) / nu
    for _ in range(steps):
        yp = f(y * ut * inv_nu)
        up, dup = reichardt_fp32(yp, kappa, B)
        ut = (ut - (ut * up - ua) * (f(1) / (up + yp * dup))).astype(f)
    return float(ut)


def test_fp32_reichardt_evaluation_against_the_law():
    """The kernels' evaluation of u+ and du+/dy+ against the FP64 oracle's law (Eq. (16)) for
    y+ from 1e-4 to 1e4: within 5e-7 relative (the library functions it replaces give
    about 1e-7)."""
    f = np.float32
    worst_u = worst_d = 0.0
    for yp in np.geomspace(1e-4, 1e4, 4001):
        up, dup = reichardt_fp32(f(yp), f(0.41), f(7.8))
        ref, dref = O.uplus(float(f(yp))), O.duplus(float(f(yp)))
        worst_u = max(worst_u, abs(up - ref) / ref)
        worst_d = max(worst_d, abs(dup - dref) / abs(dref))
    assert worst_u < 5e-7 and worst_d < 5e-7, (worst_u, worst_d)


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
