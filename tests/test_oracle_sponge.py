"""Pins of the outlet sponge (reading R19 of Sec. IV.A): over the last L planes
the molecular viscosity rises as nu(x) = nu0 + (nu_s - nu0) r^2.

* nu_s = nu0 is the plain step, bit for bit.
* Physics: a shear wave u_x = A sin(2 pi y / ny) decays at each plane with the
  local viscosity, A(t) ~ exp(-nu(x) k^2 t); its decay rate measured at planes
  inside the sponge (away from the inlet and outlet by more than the number of
  steps, so neither has reached them) gives nu(x) within 2%.  The sponge is
  long (L = 192): the x-variation of nu adds a correction that falls as 1/L^2
  (5% at L = 48, 1.6% at 96, 0.7-1% at 192; uniform nu: 0.4%).  A planted
  linear ramp fails.
"""
import numpy as np
import pytest

import oracle as O


def still_inlet(ny):
    """STG inputs whose inlet velocity is zero (zero mean, zero amplitude)."""
    R = np.zeros((6, ny))
    R[0] = R[2] = R[5] = 1e-6
    return O.StgInputs([1.0], [[0.0], [0.0], [1.0]], [1.0], [[1.0], [0.0], [0.0]], [0.0], [0.0],
                       np.zeros((3, ny)), R, [0.0], np.zeros(ny, np.int32))


def shear_wave(cfg, A=1e-3):
    nx, ny, nz = cfg.nx, cfg.ny, cfg.nz
    u = np.zeros((3, nx, ny, nz))
    u[0] = A * np.sin(2 * np.pi * np.arange(ny) / ny)[None, :, None]
    return O.init(cfg, u)


def amplitude(cfg, f):
    _, u = O.macro(cfg, f)
    s = np.sin(2 * np.pi * np.arange(cfg.ny) / cfg.ny)
    return 2.0 / cfg.ny * np.einsum("xyz,y->x", u[0], s) / cfg.nz


def test_sponge_with_molecular_viscosity_is_the_plain_step():
    base = dict(ywall=2, xbc=1, wall_model=1, tau0=0.52)
    nx, ny, nz = 8, 6, 8
    plain = O.make_cfg(nx, ny, nz, **base)
    nu0 = (0.52 - 0.5) / 3
    sp = O.make_cfg(nx, ny, nz, sponge_cells=5, sponge_nu=nu0, **base)
    f, h = shear_wave(plain, A=0.02)
    stg = still_inlet(ny)
    a = O.run(plain, f, h, 0, 3, stg=stg)
    b = O.run(sp, f, h, 0, 3, stg=stg)
    assert a[0] == O.OK and b[0] == O.OK
    assert np.array_equal(a[1], b[1]) and np.array_equal(a[2], b[2])


def measured_viscosity(mutation=0):
    nx, ny, nz, L = 384, 32, 2, 192
    tau0, nu_s = 0.8, 0.3
    cfg = O.make_cfg(nx, ny, nz, ywall=0, xbc=1, wall_model=0, tau0=tau0, cs_smag=0.0, sponge_cells=L,
                     sponge_nu=nu_s)
    stg = still_inlet(ny)
    f, h = shear_wave(cfg)
    O.set_mutation(mutation)
    try:
        st, f4, h4 = O.run(cfg, f, h, 0, 4, stg=stg)
        st2, f16, _ = O.run(cfg, f4, h4, 4, 12, stg=stg)
    finally:
        O.set_mutation(0)
    assert st == O.OK and st2 == O.OK
    k = 2 * np.pi / ny
    xs = np.arange(nx - L + 20, nx - 20, 4)
    rate = np.log(amplitude(cfg, f4)[xs] / amplitude(cfg, f16)[xs]) / 12
    nu0 = (tau0 - 0.5) / 3
    r = (xs - (nx - L) + 1) / L
    return rate / k ** 2, nu0 + (nu_s - nu0) * r ** 2


def test_shear_wave_decays_with_the_sponge_viscosity():
    meas, expect = measured_viscosity()
    err = np.abs(meas / expect - 1).max()
    assert err < 0.02, (meas, expect)


def test_planted_linear_ramp_fails():
    meas, expect = measured_viscosity(mutation=11)
    assert np.abs(meas / expect - 1).max() > 0.1
