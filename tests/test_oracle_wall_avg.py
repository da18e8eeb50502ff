"""Pins of the line-averaged friction velocity (reading R23 of Sec. II.C: the
plane-averaged u_tau of the works the paper cites, averaged over the
homogeneous direction z of each wall line) in the oracle.

* A state that does not vary in z has u_hat equal along every line, so the
  averaged model is the local model exactly (any wrong averaging weight or a
  changed force law breaks this).
* The line's u_tau solves Eq. (20) for |mean over z of u_hat| (checked with the
  oracle's scalar Newton solve of the local model) and carries the sign of the mean.
* The wall statistics of a step report the line's u_tau at every cell.
* With u_hat varying along z the two models differ.
The adjoint of the averaged model is pinned by the dot-product tests of
tests/test_oracle_adjoint.py.
"""
import numpy as np
import pytest

import oracle as O
from paper_2304_04214_amd import synthetic as S


def _z_uniform_state(cfg, seed=4):
    g = np.random.default_rng(seed)
    u = np.zeros((3, cfg.nx, cfg.ny, 1))
    u[0] = 0.05 + 0.02 * g.uniform(-1, 1, (cfg.nx, cfg.ny, 1))
    u[1] = 0.005 * g.uniform(-1, 1, (cfg.nx, cfg.ny, 1))
    u[2] = 0.01 * g.uniform(-1, 1, (cfg.nx, cfg.ny, 1))
    u = np.broadcast_to(u, (3, cfg.nx, cfg.ny, cfg.nz)).copy()
    f, hist = O.init(cfg, u)
    return f


@pytest.mark.parametrize("ywall", [1, 2])
def test_z_uniform_state_reduces_to_the_local_model(ywall):
    kw = dict(ywall=ywall, xbc=0, wall_model=1, tau0=0.51, g=(3e-6, 0.0, 0.0))
    loc = O.make_cfg(6, 7, 5, **kw)
    avg = O.make_cfg(6, 7, 5, wall_avg=1, **kw)
    f = _z_uniform_state(loc)
    st, fl, _ = O.run(loc, f, None, 0, 4)
    assert st == O.OK
    st, fa, _ = O.run(avg, f, None, 0, 4)
    assert st == O.OK
    assert np.abs(fa - fl).max() < 1e-15
    # the wall force acted: the result differs from a run without the wall model
    st, fn, _ = O.run(O.make_cfg(6, 7, 5, **dict(kw, wall_model=0)), f, None, 0, 4)
    assert np.abs(fn - fl).max() > 1e-7


def _inflow_case(seed=2):
    nx, ny, nz = 5, 8, 9
    cfg = O.make_cfg(nx, ny, nz, ywall=2, xbc=1, wall_model=1, tau0=0.505, wall_avg=1)
    U = O.reichardt_inflow(cfg, 0.006)
    du, dp = S.perturbations(nx, ny, nz, seed_offset=seed)
    f, hist = O.init(cfg, U[:, None, :, None] + 5e-3 * du, pert=dp, eps=0.05)
    mt = S.mode_table(20, ny / 2, seed_offset=seed)
    ab, boy = S.amp_bins(ny)
    stg = O.StgInputs(mt["q"], mt["sigma"], mt["kmag"], mt["d"], mt["phi"], mt["omega"], U,
                      S.reynolds_stress(ny, 0.006), ab, boy)
    return cfg, f, hist, stg


def test_line_utau_solves_eq20_for_the_mean_u_hat():
    cfg, f, hist, stg = _inflow_case()
    st, line, uhat = O.wall_lines(cfg, f, hist, 3.0, stg=stg)
    assert st == O.OK
    assert np.abs(uhat.std(axis=2)).min() > 1e-5  # u_hat does vary along the lines
    loc = O.make_cfg(cfg.nx, cfg.ny, cfg.nz, ywall=2, xbc=1, wall_model=1, tau0=cfg.tau0)
    for w in range(2):
        for x in range(cfg.nx):
            m = uhat[w, x].mean()
            st, ut = O.utau(loc, abs(m))
            assert st == O.OK
            assert abs(line[w, x] - np.sign(m) * ut) <= 1e-15 * ut


def test_wall_statistics_report_the_line_utau():
    cfg, f, hist, stg = _inflow_case()
    st, line, _ = O.wall_lines(cfg, f, hist, 1.0, stg=stg)
    acc = np.zeros((2, cfg.nx))
    st2, _, _ = O.step(cfg, f, hist, 1.0, stg=stg, wall_acc=acc)
    assert st == O.OK and st2 == O.OK
    assert np.abs(acc / cfg.nz - np.abs(line)).max() < 1e-15


def test_models_differ_when_u_hat_varies_along_z():
    cfg, f, hist, stg = _inflow_case()
    loc = O.make_cfg(cfg.nx, cfg.ny, cfg.nz, ywall=2, xbc=1, wall_model=1, tau0=cfg.tau0)
    _, fa, _ = O.step(cfg, f, hist, 1.0, stg=stg)
    _, fl, _ = O.step(loc, f, hist, 1.0, stg=stg)
    d = np.abs(fa - fl).max(axis=(0, 1, 3))  # per y row
    assert d[0] > 1e-8 and d[-1] > 1e-8
    assert d[2:-2].max() == 0.0  # rows away from the wall cells are untouched in one step


def test_planted_averaging_weight_fails():
    O.set_mutation(15)
    try:
        with pytest.raises(AssertionError):
            test_z_uniform_state_reduces_to_the_local_model(2)
    finally:
        O.set_mutation(0)
