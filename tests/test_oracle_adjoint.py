"""Pins of the FP64 oracle's discrete adjoint step.

The adjoint of a step is fixed by a definition that does not involve its own
code: for any directions (ds, dh, du_in, dC_s), the inner product of the
adjoint outputs with them equals the directional derivative of
J = <lam, s_{n+1}> + <eta, hist_{n+1}> + sum coef * stats, which central
finite differences of the (separately pinned) forward step give to ~1e-9.
Planted mistakes in the adjoint (a dropped wall-neighbour term, outlet
history term or outlet upstream term) must fail it.
"""
import numpy as np
import pytest

import oracle as O
from paper_2304_04214_amd import synthetic as S

NY, NZ = 6, 8
TOL = 2e-6  # central differences with h = 1e-4 on O(1e-2) directions: truncation ~1e-9, rounding ~1e-11


def setup(nx=5, ny=NY, nz=NZ, ywall=2, xbc=1, wm=1, g=(2e-6, 0.0, 0.0), seed=3, n_bins=3, cs=0.1, sponge=0,
          outlet=0, law=0, spectrum=False, avg=0):
    cfg = O.make_cfg(nx, ny, nz, ywall=ywall, xbc=xbc, wall_model=wm, tau0=0.52, cs_smag=cs, g=g,
                     sponge_cells=sponge, sponge_nu=0.02 if sponge else 0.0, outlet=outlet, wall_law=law, wall_avg=avg)
    U = O.reichardt_inflow(cfg, 0.0084)
    du, dp = S.perturbations(nx, ny, nz, seed_offset=seed)
    u = U[:, None, :, None] + 3e-3 * du
    f, hist = O.init(cfg, u, pert=dp, eps=0.05)
    mt = S.mode_table(12, ny / 2, seed_offset=seed, k_range=S.spectrum_k_range(ny / 2) if spectrum else None)
    R = S.reynolds_stress(ny, 0.0084)
    ab, boy = S.amp_bins(ny, n_bins)
    k_om = S.rans_k_omega(ny, 0.0084) if spectrum else (None, None)
    stg = O.StgInputs(mt["q"], mt["sigma"], mt["kmag"], mt["d"], mt["phi"], mt["omega"], U, R, ab, boy,
                      k_rans=k_om[0], omega_rans=k_om[1])
    return cfg, f, hist, stg


def with_cs(cfg, cs):
    c = O.make_cfg(cfg.nx, cfg.ny, cfg.nz, ywall=cfg.ywall, xbc=cfg.xbc, wall_model=cfg.wall_model,
                   tau0=cfg.tau0, cs_smag=cs, g=tuple(cfg.g), rates=list(cfg.s), sponge_cells=cfg.sponge_cells,
                   sponge_nu=cfg.sponge_nu, outlet=cfg.outlet, wall_law=cfg.wall_law, wall_avg=cfg.wall_avg)
    return c


CASES = {
    "slip_inflow_wallmodel": dict(ywall=2, xbc=1, wm=1),
    "bounceback_inflow_wallmodel": dict(ywall=1, xbc=1, wm=1),
    "bounceback_inflow": dict(ywall=1, xbc=1, wm=0),
    "slip_periodic_x_wallmodel": dict(ywall=2, xbc=0, wm=1, g=(4e-6, 0.0, 0.0)),
    "periodic_all": dict(ywall=0, xbc=0, wm=0, g=(4e-6, 1e-6, 0.0)),
    "slip_inflow_wallmodel_sponge": dict(ywall=2, xbc=1, wm=1, nx=8, sponge=4),
    "slip_inflow_zero_gradient_outlet": dict(ywall=2, xbc=1, wm=1, outlet=1),
    "slip_inflow_musker_wall_law": dict(ywall=2, xbc=1, wm=1, law=1),
    "slip_inflow_row_spectrum": dict(ywall=2, xbc=1, wm=1, spectrum=True),
    "slip_inflow_line_averaged_utau": dict(ywall=2, xbc=1, wm=1, avg=1),
    "bounceback_periodic_x_line_averaged_utau": dict(ywall=1, xbc=0, wm=1, g=(4e-6, 0.0, 0.0), avg=1),
    "bounceback_inflow_musker_wall_law": dict(ywall=1, xbc=1, wm=1, law=1),
}


def dot_test(cfg, f, hist, stg, seed=5, t_next=7.0):
    g = np.random.default_rng(seed)
    open_ = cfg.xbc == 1
    uin = O.stg_plane(cfg, stg, t_next)[1] if open_ else None
    lam = g.normal(size=f.shape)
    eta = g.normal(size=(5, cfg.ny, cfg.nz)) if open_ else None
    planes = [1, 3]
    coef = g.normal(size=(2, cfg.ny, 9))
    adj = O.adjoint_step(cfg, f, hist if open_ else None, t_next, lam, eta, uin=uin, planes=planes, coef=coef)
    assert adj["status"] == O.OK

    def J(fv, hv, uv, cs):
        acc = np.zeros((2, cfg.ny, 9))
        st, fo, ho = O.step_uin(with_cs(cfg, cs), fv, hv, uv, planes=planes, acc=acc)
        assert st == O.OK
        r = (lam * fo).sum() + (coef * acc).sum()
        return r + ((eta * ho).sum() if open_ else 0.0)

    ds = g.normal(size=f.shape) * 1e-2
    dh = g.normal(size=(5, cfg.ny, cfg.nz)) * 1e-2
    du = g.normal(size=(3, cfg.ny, cfg.nz)) * 1e-2
    dc = 0.05
    cs0 = cfg.cs_smag
    h0 = hist if open_ else None
    parts = {
        "s": (lambda e: (f + e * ds, h0, uin, cs0), lambda: (adj["lam"] * ds).sum()),
        "cs": (lambda e: (f, h0, uin, cs0 + e * dc), lambda: adj["g_cs"] * dc),
    }
    if open_:
        parts["hist"] = (lambda e: (f, hist + e * dh, uin, cs0), lambda: (adj["eta"] * dh).sum())
        parts["uin"] = (lambda e: (f, hist, uin + e * du, cs0), lambda: (adj["g_uin"] * du).sum())
    errs = {}
    eps = 1e-4
    for name, (arg, ad) in parts.items():
        fd = (J(*arg(eps)) - J(*arg(-eps))) / (2 * eps)
        a = ad()
        errs[name] = (abs(fd - a) / max(abs(fd), 1e-30), fd, a)
    return errs


@pytest.mark.parametrize("name", sorted(CASES))
def test_adjoint_dot_product_matches_fd(name):
    cfg, f, hist, stg = setup(**CASES[name])
    errs = dot_test(cfg, f, hist, stg)
    cfg = setup(**CASES[name])[0]
    for k, (e, fd, a) in errs.items():
        if k == "hist" and cfg.outlet == 1:  # the zero-gradient outlet does not read the history
            assert fd == 0.0 and a == 0.0, (fd, a)
            continue
        assert abs(fd) > 1e-8, (k, fd)  # the direction actually moves J
        assert e < TOL, (name, k, e, fd, a)


@pytest.mark.parametrize("mutation,part,avg", [(8, "s", 0), (9, "hist", 0), (10, "s", 0), (16, "s", 1)])
def test_planted_adjoint_mistakes_fail(mutation, part, avg):
    """8: wall-neighbour term dropped; 9: outlet history sensitivity dropped;
    10: outlet upstream term dropped; 16: the line average's second-cell term dropped."""
    cfg, f, hist, stg = setup(avg=avg)
    O.set_mutation(mutation)
    try:
        errs = dot_test(cfg, f, hist, stg)
    finally:
        O.set_mutation(0)
    assert errs[part][0] > 10 * TOL, errs


@pytest.mark.parametrize("spectrum", [False, True])
def test_amp_bin_gradient_matches_fd(spectrum):
    """dL/ds_b = sum over the bin's inlet rows of g_uin . (a v'), checked through the STG
    (one spectral table, or per-row spectra)."""
    cfg, f, hist, stg = setup(n_bins=3, spectrum=spectrum)
    g = np.random.default_rng(11)
    lam = g.normal(size=f.shape)
    eta = g.normal(size=(5, cfg.ny, cfg.nz))
    adj = O.adjoint_step(cfg, f, hist, 9.0, lam, eta, stg=stg, want_amp=True)
    assert adj["status"] == O.OK

    def J(amp):
        st2 = O.StgInputs(stg.q, stg.sigma, stg.kmag, stg.d, stg.phi, stg.omega, stg.u_rans, stg.R, amp,
                          stg.bin_of_y, k_rans=stg.k_rans, omega_rans=stg.omega_rans)
        st, fo, ho = O.step(cfg, f, hist, 9.0, stg=st2)
        assert st == O.OK
        return (lam * fo).sum() + (eta * ho).sum()

    for b in range(3):
        e = np.zeros(3)
        e[b] = 1e-3
        fd = (J(stg.amp_bin + e) - J(stg.amp_bin - e)) / 2e-3
        assert abs(fd - adj["g_amp"][b]) <= 1e-6 * abs(fd), (b, fd, adj["g_amp"][b])


def loss_and_coef(acc, nz, T, U_target, R12_target):
    """Mean-profile loss of the statistics sums and its derivative dL/dacc (plain numpy)."""
    m = acc / (nz * T)
    U, V, UV = m[..., 0], m[..., 1], m[..., 6]
    uv = UV - U * V
    a = U - U_target
    b = uv - R12_target
    L = (a ** 2).sum() / (U_target ** 2).sum() + (b ** 2).sum() / (R12_target ** 2).sum()
    dU = 2 * a / (U_target ** 2).sum()
    db = 2 * b / (R12_target ** 2).sum()
    dm = np.zeros_like(m)
    dm[..., 0] = dU - db * V
    dm[..., 1] = -db * U
    dm[..., 6] = db
    return L, dm / (nz * T)


def test_multistep_loss_gradient_matches_fd():
    """Gradient of a statistics loss over 4 steps w.r.t. every s_b and C_s."""
    cfg, f, hist, stg = setup(nx=6, n_bins=3)
    T, planes = 4, [2, 4]
    U_t = stg.u_rans[0] * 1.01
    R12_t = stg.R[1]

    def forward(amp, cs):
        st2 = O.StgInputs(stg.q, stg.sigma, stg.kmag, stg.d, stg.phi, stg.omega, stg.u_rans, stg.R, amp,
                          stg.bin_of_y)
        acc = np.zeros((2, cfg.ny, 9))
        st, _, _ = O.run(with_cs(cfg, cs), f, hist, 0.0, T, stg=st2, planes=planes, acc=acc)
        assert st == O.OK
        return acc

    acc = forward(stg.amp_bin, cfg.cs_smag)
    L, coef = loss_and_coef(acc, cfg.nz, T, U_t, R12_t)
    r = O.gradient_run(cfg, stg, f, hist, 0.0, T, planes, coef)
    assert np.allclose(r["acc"], acc, rtol=0, atol=1e-15)
    h = 1e-4
    fd = []
    for b in range(3):
        e = np.zeros(3)
        e[b] = h
        Lp = loss_and_coef(forward(stg.amp_bin + e, cfg.cs_smag), cfg.nz, T, U_t, R12_t)[0]
        Lm = loss_and_coef(forward(stg.amp_bin - e, cfg.cs_smag), cfg.nz, T, U_t, R12_t)[0]
        fd.append((Lp - Lm) / (2 * h))
    Lp = loss_and_coef(forward(stg.amp_bin, cfg.cs_smag + h), cfg.nz, T, U_t, R12_t)[0]
    Lm = loss_and_coef(forward(stg.amp_bin, cfg.cs_smag - h), cfg.nz, T, U_t, R12_t)[0]
    fd.append((Lp - Lm) / (2 * h))
    fd = np.array(fd)
    ad = np.append(r["g_amp"], r["g_cs"])
    assert np.abs(fd).max() > 0
    err = np.abs(ad - fd).max() / np.abs(fd).max()
    assert err < 1e-6, (ad, fd, err)
