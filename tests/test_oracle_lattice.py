"""Lattice-level pins of the oracle: streaming index map, closed-form flows
(shear-wave decay, Poiseuille), conservation, uniform-flow preservation with
all boundaries, and the statistics accumulators."""
import numpy as np
import pytest

import oracle as O
from paper_2304_04214_amd import synthetic as S

RNG = np.random.default_rng(5)


def _coded(cfg):
    """Integer-coded populations: every (i, node) holds a distinct integer."""
    n = 19 * cfg.nx * cfg.ny * cfg.nz
    return np.arange(n, dtype=np.float64).reshape(19, cfg.nx, cfg.ny, cfg.nz)


def test_periodic_streaming_is_a_roll():
    """Eq. (3) streaming in a periodic box: f_i(x + c_i) = f_i(x)."""
    cfg = O.make_cfg(5, 4, 7)
    f = _coded(cfg)
    out = O.stream_only(cfg, f)
    c = O.tables()["c"]
    for i in range(19):
        assert np.array_equal(out[i], np.roll(f[i], shift=tuple(c[i]), axis=(0, 1, 2)))


def _brute_stream(cfg, f):
    """Brute-force pull with the wall rules written out case by case."""
    t = O.tables()
    c, opp, refl = t["c"], t["opp"], t["refl"]
    nx, ny, nz = cfg.nx, cfg.ny, cfg.nz
    out = np.full_like(f, -1.0)
    for i in range(19):
        for x in range(nx):
            for y in range(ny):
                for z in range(nz):
                    xs, ys, zs = x - c[i][0], y - c[i][1], (z - c[i][2]) % nz
                    if cfg.xbc == 0:
                        xs %= nx
                    if 0 <= ys < ny:
                        if 0 <= xs < nx:
                            out[i, x, y, z] = f[i, xs, ys, zs]
                    elif cfg.ywall == 1:
                        out[i, x, y, z] = f[opp[i], x, y, z]
                    elif cfg.ywall == 2:
                        if 0 <= xs < nx:
                            out[i, x, y, z] = f[refl[i], xs, y, zs]
    return out


@pytest.mark.parametrize("ywall,xbc", [(1, 0), (2, 0), (1, 1), (2, 1)])
def test_wall_streaming_matches_brute_force(ywall, xbc):
    cfg = O.make_cfg(5, 4, 3, ywall=ywall, xbc=xbc)
    f = _coded(cfg)
    assert np.array_equal(O.stream_only(cfg, f), _brute_stream(cfg, f))


@pytest.mark.parametrize("ywall", [1, 2])
def test_closed_box_streaming_is_a_permutation(ywall):
    cfg = O.make_cfg(4, 5, 3, ywall=ywall)
    f = _coded(cfg)
    out = O.stream_only(cfg, f)
    assert np.array_equal(np.sort(out.ravel()), np.sort(f.ravel()))


def _shear_wave_nu(N, tau, U=1e-4, t1=40, t2=None):
    cfg = O.make_cfg(1, N, 1, tau0=tau, cs_smag=0.0)
    y = np.arange(N)
    k = 2 * np.pi / N
    u = np.zeros((3, 1, N, 1))
    u[0, 0, :, 0] = U * np.sin(k * y)
    f, _ = O.init(cfg, u)
    t2 = t2 or int(1.0 / ((tau - 0.5) / 3 * k * k))

    def amp(f):
        _, uu = O.macro(cfg, f)
        return 2.0 / N * (uu[0, 0, :, 0] @ np.sin(k * y))

    _, f1, _ = O.run(cfg, f, None, 0, t1)
    _, f2, _ = O.run(cfg, f1, None, t1, t2 - t1)
    return -np.log(amp(f2) / amp(f1)) / (k * k * (t2 - t1))


def test_shear_wave_decays_at_lattice_viscosity():
    """Sec. II.A, Eq. (5): a shear wave decays as exp(-nu k^2 t), nu = cs^2 (tau - 1/2)."""
    for tau in (0.6, 0.8, 1.1):
        nu = (tau - 0.5) / 3
        e32 = abs(_shear_wave_nu(32, tau) / nu - 1)
        e64 = abs(_shear_wave_nu(64, tau) / nu - 1)
        assert e32 < 1e-2
        assert e64 < e32 / 3 or e64 < 1e-6  # second-order convergence in the wavenumber


def _poiseuille(tau, rates, ny=16, g=1e-6, steps=12000):
    cfg = O.make_cfg(1, ny, 1, ywall=1, tau0=tau, cs_smag=0.0, rates=rates, g=(g, 0.0, 0.0))
    f, _ = O.init(cfg, np.zeros((3, 1, ny, 1)))
    _, f, _ = O.run(cfg, f, None, 0, steps)
    rho, u = O.macro(cfg, f)
    # the stored state is post-collision (j* = j + F), so the velocity of
    # Eq. (11), (j + F/2)/rho, is j*/rho - g/2
    return u[0, 0, :, 0] - g / 2, cfg


def test_poiseuille_trt_magic_parameter_is_exact():
    """Halfway bounce-back with a TRT rate set (Lambda = 3/16) through the MRT
    path: the steady profile is the exact parabola u = g/(2 nu) (y+1/2)(ny-1/2-y)."""
    tau, ny, g = 0.8, 16, 1e-6
    sp = 1 / tau
    sm = 1 / (0.5 + (3.0 / 16.0) / (1 / sp - 0.5))
    rates = [1.0] * 19
    for k in (1, 2, 9, 10, 11, 12, 13, 14, 15):
        rates[k] = sp
    for k in (4, 6, 8, 16, 17, 18):
        rates[k] = sm
    u, _ = _poiseuille(tau, rates, ny, g)
    nu = (tau - 0.5) / 3
    y = np.arange(ny)
    exact = g / (2 * nu) * (y + 0.5) * (ny - 0.5 - y)
    assert np.abs(u - exact).max() < 1e-10 * exact.max()


def test_poiseuille_paper_rates_bulk_curvature_and_symmetry():
    tau, ny, g = 0.8, 16, 1e-6
    u, _ = _poiseuille(tau, O.PAPER_RATES, ny, g)
    nu = (tau - 0.5) / 3
    assert np.abs(u - u[::-1]).max() < 1e-12 * u.max()
    d2 = u[2:] - 2 * u[1:-1] + u[:-2]
    assert np.abs(d2 + g / nu).max() < 1e-9 * g / nu
    y = np.arange(ny)
    exact = g / (2 * nu) * (y + 0.5) * (ny - 0.5 - y)
    assert np.abs(u - exact).max() < 1e-2 * exact.max()


def _random_state(cfg, seed):
    du, dp = S.perturbations(cfg.nx, cfg.ny, cfg.nz, seed_offset=seed)
    u = 0.02 * du
    u[0] += 0.05
    return O.init(cfg, u, rho=1 + 0.01 * du[0], pert=dp, eps=0.05)


@pytest.mark.parametrize("ywall,wm", [(0, 0), (1, 0), (2, 0), (1, 1), (2, 1)])
def test_closed_box_conserves_mass(ywall, wm):
    cfg = O.make_cfg(6, 8, 5, ywall=ywall, wall_model=wm, tau0=0.52, cs_smag=0.1, g=(1e-5, 0, 0))
    f, _ = _random_state(cfg, 1)
    m0 = f.sum()
    st, f2, _ = O.run(cfg, f, None, 0, 10)
    assert st == O.OK
    assert abs(f2.sum() - m0) < 1e-12 * m0


def test_periodic_momentum_gain_equals_body_force():
    g = np.array([1e-5, -2e-6, 3e-6])
    cfg = O.make_cfg(6, 8, 5, tau0=0.52, cs_smag=0.1, g=tuple(g))
    f, _ = _random_state(cfg, 2)
    c = O.tables()["c"].astype(float)
    p0 = np.einsum("ixyz,ia->a", f, c)
    mass = f.sum()
    st, f2, _ = O.run(cfg, f, None, 0, 5)
    p1 = np.einsum("ixyz,ia->a", f2, c)
    assert np.abs(p1 - p0 - 5 * g * mass).max() < 1e-13 * mass


def _uniform_channel(ywall, nx=6, ny=6, nz=4, U=0.08, outlet=0):
    cfg = O.make_cfg(nx, ny, nz, ywall=ywall, xbc=1, wall_model=0, tau0=0.52, cs_smag=0.1, u_conv=U, outlet=outlet)
    u_rans = np.zeros((3, ny))
    u_rans[0] = U
    mt = S.mode_table(8, ny / 2)
    ab, boy = S.amp_bins(ny)
    stg = O.StgInputs(mt["q"], mt["sigma"], mt["kmag"], mt["d"], mt["phi"], mt["omega"], u_rans,
                      S.reynolds_stress(ny, 1e-3), 0 * ab, boy)
    u = np.zeros((3, nx, ny, nz))
    u[0] = U
    f, hist = O.init(cfg, u)
    return cfg, stg, f, hist


def test_uniform_flow_is_preserved_by_slip_walls_inlet_and_outlet():
    cfg, stg, f, hist = _uniform_channel(2)
    st, f2, h2 = O.run(cfg, f, hist, 0, 10, stg=stg)
    assert st == O.OK
    assert np.abs(f2 - f).max() < 1e-15
    assert np.abs(h2 - hist).max() < 1e-15


def test_uniform_flow_is_preserved_by_the_zero_gradient_outlet():
    cfg, stg, f, hist = _uniform_channel(2, outlet=1)
    st, f2, _ = O.run(cfg, f, hist, 0, 10, stg=stg)
    assert st == O.OK
    assert np.abs(f2 - f).max() < 1e-15


def test_zero_gradient_outlet_is_the_fast_convection_limit():
    """f_i = f_i(x-1) is the limit U_c -> infinity of (f_i^prev + U_c f_i(x-1)) / (1 + U_c)."""
    cfg0, stg, f, hist = _uniform_channel(2, nx=7, outlet=1)
    du, dp = S.perturbations(7, 6, 4, seed_offset=5)
    f, hist = O.init(cfg0, 0.08 * np.array([1.0, 0, 0])[:, None, None, None] + 1e-2 * du, pert=dp, eps=0.05)
    zg = O.run(cfg0, f, hist, 0, 6, stg=stg)[1]
    fast = O.make_cfg(7, 6, 4, ywall=2, xbc=1, wall_model=0, tau0=0.52, cs_smag=0.1, u_conv=1e9)
    conv = O.run(fast, f, hist, 0, 6, stg=stg)[1]
    slow = O.make_cfg(7, 6, 4, ywall=2, xbc=1, wall_model=0, tau0=0.52, cs_smag=0.1, u_conv=0.1)
    other = O.run(slow, f, hist, 0, 6, stg=stg)[1]
    assert np.abs(conv - zg).max() < 1e-9
    assert np.abs(other - zg).max() > 1e-5  # the rules do differ


def test_statistics_of_a_uniform_flow():
    cfg, stg, f, hist = _uniform_channel(2)
    planes = [1, 3]
    acc = np.zeros((2, cfg.ny, 9))
    st, _, _ = O.run(cfg, f, hist, 0, 4, stg=stg, planes=planes, acc=acc)
    mean = acc / (4 * cfg.nz)
    assert np.allclose(mean[:, :, 0], 0.08, atol=1e-15)
    assert np.abs(mean[:, :, 1:3]).max() < 1e-15
    var_u = mean[:, :, 3] - mean[:, :, 0] ** 2
    assert np.abs(var_u).max() < 1e-15
    assert np.abs(mean[:, :, 6] - mean[:, :, 0] * mean[:, :, 1]).max() < 1e-15


def test_step_nodes_matches_full_step():
    ny = 8
    cfg = O.make_cfg(7, ny, 5, ywall=2, xbc=1, wall_model=1, tau0=0.5004, cs_smag=0.1, u_conv=0.1)
    u_tau = 0.0045
    u_rans = O.reichardt_inflow(cfg, u_tau)
    mt = S.mode_table(20, ny / 2)
    ab, boy = S.amp_bins(ny)
    stg = O.StgInputs(mt["q"], mt["sigma"], mt["kmag"], mt["d"], mt["phi"], mt["omega"], u_rans,
                      S.reynolds_stress(ny, u_tau), ab, boy)
    du, dp = S.perturbations(cfg.nx, ny, cfg.nz)
    u = np.broadcast_to(u_rans[:, None, :, None], (3, cfg.nx, ny, cfg.nz)) + 1e-3 * du
    f, hist = O.init(cfg, u, pert=dp, eps=0.01)
    st, full, _ = O.step(cfg, f, hist, 1.0, stg=stg)
    assert st == O.OK
    nodes = RNG.choice(cfg.nx * ny * cfg.nz, 40, replace=False)
    st, out, _ = O.step_nodes(cfg, f, hist, 1.0, nodes, stg=stg)
    assert st == O.OK
    assert np.array_equal(out, full.reshape(19, -1)[:, nodes])


def test_wall_statistics_of_a_uniform_flow():
    """One step from a uniform state: every first off-wall cell sees u_w = u_2 = U, so
    the wall statistics hold nz u_tau(U) at every x for both walls."""
    nx, ny, nz, U = 6, 6, 4, 0.08
    cfg, stg, f, hist = _uniform_channel(2, nx=nx, ny=ny, nz=nz, U=U)
    cfg.wall_model = 1
    wall = np.zeros((2, nx))
    st, _, _ = O.step(cfg, f, hist, 1.0, stg=stg, wall_acc=wall)
    assert st == O.OK
    st, ut = O.utau(cfg, U)
    assert np.allclose(wall, nz * ut, rtol=1e-14, atol=0)
