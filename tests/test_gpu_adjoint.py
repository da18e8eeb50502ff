"""Parity of the HIP adjoint step with the FP64 oracle's adjoint (GPU tests).

Both sides receive the same state s_n (the oracle's seeded equilibrium state,
rounded to the storage type: the HIP side imports it, the oracle takes the
rounded values in FP64), the same random lam_{n+1}, eta_{n+1} and statistics
weights.  Each side computes its own inlet plane.  The HIP side computes in
FP32, so the bound is relative to the largest value of each output:
  lam_n, eta_n, g_uin   5e-6 (FP32 arithmetic, O(100) operations on O(1)
                        values: a few 1e-7; measured 1.3e-7 .. 3.7e-7)
  dL/ds_b, dL/dC_s      3e-4 (sums over a plane / the lattice of products whose
                        FP32 factors carry relative errors up to ~1e-5: the
                        Smagorinsky path differentiates |Pi_neq|, which FP32
                        forms from populations with ~1e-3 cancellation;
                        measured up to 3e-5 for dL/dC_s)
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2304_04214_amd import synthetic as S
from paper_2304_04214_amd.adjoint import StatsGradient
from parity_cases import Case, rel_linf

pytestmark = pytest.mark.gpu

TOL_FIELD = 5e-6
TOL_PARAM = 3e-4


def storage_round(f, storage, ref=None):
    """Values the HIP side holds after importing f (float32, or half deviations from the
    weights plus the optional per-row reference offsets ref [19, ny])."""
    w = O.tables()["w"].astype(np.float32)[:, None, None, None]
    f32 = np.asarray(f, dtype=np.float32)
    if storage == "f32":
        return f32.astype(np.float64)
    r = np.zeros((1, 1, 1, 1), np.float32) if ref is None else np.asarray(ref, np.float32)[:, None, :, None]
    h = ((f32 - w) - r).astype(np.float16)
    return ((w + r) + h.astype(np.float32)).astype(np.float64)


def to_numpy(t):
    return t.detach().cpu().numpy().astype(np.float64)


def single_step(case, storage="f32", seed=7, planes=(1, 3), t_next=5.0):
    ch = case.ch
    nx, ny, nz = case.nx, case.ny, case.nz
    open_ = case.xbc == "inflow"
    g = np.random.default_rng(seed)
    s = storage_round(case.f_or, storage, case.dref)
    hist = np.asarray(case.hist_or, dtype=np.float32).astype(np.float64)
    lam = g.normal(size=(19, nx, ny, nz)).astype(np.float32).astype(np.float64)
    eta = g.normal(size=(5, ny, nz)).astype(np.float32).astype(np.float64)
    coef = g.normal(size=(len(planes), ny, 9)).astype(np.float32).astype(np.float64)
    # ---- oracle ----
    ref = O.adjoint_step(case.ocfg, s, hist if open_ else None, t_next, lam, eta if open_ else None,
                         stg=case.stg_or if open_ else None, planes=list(planes), coef=coef, want_amp=open_)
    assert ref["status"] == O.OK
    # ---- HIP ----
    ch.load_populations(torch.as_tensor(case.f_or, dtype=torch.float32))
    f_cur, h_cur = ch.state()
    h_cur.copy_(torch.as_tensor(hist, dtype=torch.float32))
    ch.stats_attach(list(planes))
    lam_n = ch.field_import(torch.as_tensor(lam, dtype=torch.float32))
    lam_p = ch.new_field()
    eta_n = torch.as_tensor(eta, dtype=torch.float32, device="cuda")
    eta_p = torch.zeros_like(eta_n)
    g_uin = torch.zeros((3, ny, nz), dtype=torch.float32, device="cuda")
    n_bins = len(case.ab) if open_ else 0
    grad = torch.zeros(n_bins + 1, dtype=torch.float64, device="cuda")
    ch.adjoint_step(f_cur, h_cur, t_next, lam_n, lam_p, eta_n, eta_p,
                    coef=torch.as_tensor(coef, dtype=torch.float32), g_uin=g_uin, grad=grad)
    ch.sync()
    out = dict(lam=to_numpy(ch.field_export(lam_p)), eta=to_numpy(eta_p), g_uin=to_numpy(g_uin),
               grad=to_numpy(grad))
    return ref, out


def check_single(ref, out, open_, label):
    errs = {"lam": rel_linf(out["lam"], ref["lam"])}
    if open_:
        errs["eta"] = rel_linf(out["eta"], ref["eta"])
        errs["g_uin"] = rel_linf(out["g_uin"], ref["g_uin"])
        errs["g_amp"] = rel_linf(out["grad"][:-1], ref["g_amp"])
    errs["g_cs"] = abs(out["grad"][-1] - ref["g_cs"]) / max(abs(ref["g_cs"]), 1e-300)
    print(label, {k: "%.2e" % v for k, v in errs.items()}, "g_cs", out["grad"][-1], ref["g_cs"], flush=True)
    for k in ("lam", "eta", "g_uin"):
        if k in errs:
            assert errs[k] < TOL_FIELD, (label, k, errs)
    for k in ("g_amp", "g_cs"):
        if k in errs:
            assert errs[k] < TOL_PARAM, (label, k, errs)
    return errs


CASES = {
    # name: (Case kwargs, storage)
    "slip_inflow_wallmodel_6x8x70": (dict(nx=6, ny=8, nz=70, ywall="slip", xbc="inflow", wall_model=True,
                                          g=(2e-6, 0.0, 0.0)), "f32"),
    "slip_inflow_wallmodel_ragged_ny5": (dict(nx=5, ny=5, nz=20, ywall="slip", xbc="inflow", wall_model=True), "f32"),
    "slip_inflow_wallmodel_ragged_ny9": (dict(nx=5, ny=9, nz=66, ywall="slip", xbc="inflow", wall_model=True), "f32"),
    "bounceback_inflow_wallmodel": (dict(nx=6, ny=6, nz=16, ywall="bounceback", xbc="inflow", wall_model=True), "f32"),
    "bounceback_inflow": (dict(nx=6, ny=7, nz=16, ywall="bounceback", xbc="inflow", wall_model=False), "f32"),
    "slip_periodic_x_wallmodel": (dict(nx=6, ny=8, nz=12, ywall="slip", xbc="periodic", wall_model=True,
                                       g=(4e-6, 0.0, 0.0)), "f32"),
    "periodic_all_force": (dict(nx=5, ny=4, nz=9, ywall="periodic", xbc="periodic", wall_model=False,
                                g=(4e-6, 1e-6, 0.0)), "f32"),
    "f16_slip_inflow_wallmodel": (dict(nx=6, ny=8, nz=70, ywall="slip", xbc="inflow", wall_model=True), "f16dev"),
    "slip_inflow_wallmodel_sponge": (dict(nx=9, ny=8, nz=20, ywall="slip", xbc="inflow", wall_model=True,
                                          sponge_cells=5, sponge_nu=0.02), "f32"),
    "slip_inflow_zero_gradient_outlet": (dict(nx=6, ny=8, nz=20, ywall="slip", xbc="inflow", wall_model=True,
                                              outlet="zero-gradient"), "f32"),
    "slip_inflow_musker_wall_law": (dict(nx=6, ny=8, nz=20, ywall="slip", xbc="inflow", wall_model=True,
                                         wall_law="musker"), "f32"),
    "slip_inflow_row_spectrum": (dict(nx=6, ny=8, nz=20, ywall="slip", xbc="inflow", wall_model=True,
                                      spectrum=True), "f32"),
    "slip_inflow_line_averaged_utau": (dict(nx=6, ny=8, nz=70, ywall="slip", xbc="inflow", wall_model=True,
                                            wall_avg="line"), "f32"),
    "bounceback_periodic_line_averaged_utau_ragged_ny9": (dict(nx=5, ny=9, nz=66, ywall="bounceback",
                                                               xbc="periodic", wall_model=True, g=(4e-6, 0.0, 0.0),
                                                               wall_avg="line"), "f32"),
    "f16_slip_inflow_line_averaged_utau": (dict(nx=6, ny=8, nz=70, ywall="slip", xbc="inflow", wall_model=True,
                                                wall_avg="line"), "f16dev"),
    "f16ref_slip_inflow_wallmodel": (dict(nx=6, ny=8, nz=70, ywall="slip", xbc="inflow", wall_model=True,
                                          reference=True), "f16dev"),
    "f16ref_bounceback_periodic_force": (dict(nx=5, ny=9, nz=66, ywall="bounceback", xbc="periodic",
                                              wall_model=True, g=(4e-6, 0.0, 0.0), reference=True), "f16dev"),
    "f16ref_slip_inflow_line_averaged_utau": (dict(nx=6, ny=8, nz=70, ywall="slip", xbc="inflow", wall_model=True,
                                                   wall_avg="line", reference=True), "f16dev"),
    "f16_bounceback_periodic_line_averaged_utau": (dict(nx=5, ny=9, nz=66, ywall="bounceback", xbc="periodic",
                                                        wall_model=True, g=(4e-6, 0.0, 0.0), wall_avg="line"),
                                                   "f16dev"),
    "f16_slip_inflow_musker_wall_law": (dict(nx=6, ny=8, nz=70, ywall="slip", xbc="inflow", wall_model=True,
                                             wall_law="musker"), "f16dev"),
    # dispatch list: no bulk columns at all (nx = 3), and many columns of both classes over the
    # 8 XCDs with padding (ragged nz, 3 y-groups of which 2 hold a wall row)
    "slip_inflow_wallmodel_nx3": (dict(nx=3, ny=8, nz=20, ywall="slip", xbc="inflow", wall_model=True), "f32"),
    "bounceback_inflow_wallmodel_23x12x130": (dict(nx=23, ny=12, nz=130, ywall="bounceback", xbc="inflow",
                                                   wall_model=True), "f32"),
    "f16_slip_inflow_wallmodel_23x12x130": (dict(nx=23, ny=12, nz=130, ywall="slip", xbc="inflow",
                                                 wall_model=True), "f16dev"),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_adjoint_step_matches_oracle(name):
    kw, storage = CASES[name]
    print("case", name, flush=True)
    case = Case(**kw, storage=storage)
    planes = (1, 3) if kw["nx"] > 3 else (1,)
    ref, out = single_step(case, storage=storage, planes=planes)
    check_single(ref, out, kw["xbc"] == "inflow", name)


def test_adjoint_rejects_bad_arguments():
    from paper_2304_04214_amd import _abi as A
    case = Case(6, 8, 16)
    ch = case.ch
    f_cur, h_cur = ch.state()
    lam = ch.new_field()
    eta = torch.zeros((5, 8, 16), dtype=torch.float32, device="cuda")
    with pytest.raises(A.LbmError):  # lam_prev aliases lam_next
        ch.adjoint_step(f_cur, h_cur, 1.0, lam, lam, eta, torch.zeros_like(eta))
    with pytest.raises(A.LbmError):  # coef without statistics planes
        ch.adjoint_step(f_cur, h_cur, 1.0, lam, ch.new_field(), eta, torch.zeros_like(eta),
                        coef=torch.zeros((1, 8, 9)))
    with pytest.raises(A.LbmError):  # open channel without eta buffers
        ch.adjoint_step(f_cur, h_cur, 1.0, lam, ch.new_field())
    ch.sync()



def test_multistep_statistics_gradient_matches_oracle():
    """dL/ds_b and dL/dC_s of a mean-profile loss over 6 steps with checkpoint
    segments of 4 (recompute included), HIP vs oracle; each side runs its own
    forward from the same initial state."""
    nx, ny, nz, T = 8, 8, 24, 6
    case = Case(nx, ny, nz, ywall="slip", xbc="inflow", wall_model=True, n_modes=16, seed=2)
    planes = [3, 6]
    # identical initial state on both sides (float32 values)
    f0 = storage_round(case.f_or, "f32")
    h0 = np.asarray(case.hist_or, dtype=np.float32).astype(np.float64)
    case.ch.load_populations(torch.as_tensor(f0, dtype=torch.float32))
    case.ch.state()[1].copy_(torch.as_tensor(h0, dtype=torch.float32))
    U_t = case.U_or[0] * 1.02
    R12_t = case.R[1]
    # oracle
    acc = np.zeros((2, ny, 9))
    st, _, _ = O.run(case.ocfg, f0, h0, 0.0, T, stg=case.stg_or, planes=planes, acc=acc)
    assert st == O.OK
    dmeans = loss_grad(acc / (nz * T), U_t, R12_t)
    ref = O.gradient_run(case.ocfg, case.stg_or, f0, h0, 0.0, T, planes, dmeans / (nz * T))
    # HIP
    run = StatsGradient(case.ch, planes, T, segment=4)
    means = run.forward()
    assert rel_linf(means, acc / (nz * T)) < 1e-5
    dmeans_g = loss_grad(means, U_t, R12_t)
    g = run.backward(dmeans_g)
    e_amp = rel_linf(g[:-1], ref["g_amp"])
    e_cs = abs(g[-1] - ref["g_cs"]) / abs(ref["g_cs"])
    print("multistep g_amp err %.2e g_cs err %.2e" % (e_amp, e_cs), g[-1], ref["g_cs"], flush=True)
    assert e_amp < TOL_PARAM and e_cs < TOL_PARAM


def test_autograd_function_gradient_matches_oracle():
    """plane_statistics (the torch.autograd.Function over the adjoint sweep): a torch loss of its
    output back-propagates to the amplitude scalings and C_s; the gradients equal the FP64
    oracle's adjoint gradient of the same loss (6 steps, checkpoint segments of 4)."""
    from paper_2304_04214_amd.adjoint import mean_profile_loss, plane_statistics
    nx, ny, nz, T = 8, 8, 24, 6
    case = Case(nx, ny, nz, ywall="slip", xbc="inflow", wall_model=True, n_modes=16, seed=4)
    planes = [3, 6]
    f0 = storage_round(case.f_or, "f32")
    h0 = np.asarray(case.hist_or, dtype=np.float32).astype(np.float64)
    case.ch.load_populations(torch.as_tensor(f0, dtype=torch.float32))
    case.ch.state()[1].copy_(torch.as_tensor(h0, dtype=torch.float32))
    U_t = case.U_or[0] * 1.02
    R12_t = case.R[1]
    run = StatsGradient(case.ch, planes, T, segment=4)
    amp = torch.tensor(np.asarray(case.ab, dtype=np.float64), requires_grad=True)
    cs = torch.tensor(0.1, dtype=torch.float64, requires_grad=True)
    means = plane_statistics(run, amp, cs)
    loss = sum(mean_profile_loss(means[p], U_t, R12_t) for p in range(len(planes)))
    loss.backward()
    # oracle: the same loss of its own statistics, and its adjoint gradient
    acc = np.zeros((len(planes), ny, 9))
    st, _, _ = O.run(case.ocfg, f0, h0, 0.0, T, stg=case.stg_or, planes=planes, acc=acc)
    assert st == O.OK
    assert rel_linf(means.detach().numpy(), acc / (nz * T)) < 1e-5
    dmeans = loss_grad(acc / (nz * T), U_t, R12_t)
    ref = O.gradient_run(case.ocfg, case.stg_or, f0, h0, 0.0, T, planes, dmeans / (nz * T))
    e_amp = rel_linf(amp.grad.numpy(), ref["g_amp"])
    e_cs = abs(float(cs.grad) - ref["g_cs"]) / abs(ref["g_cs"])
    print("autograd g_amp err %.2e g_cs err %.2e" % (e_amp, e_cs), flush=True)
    assert e_amp < TOL_PARAM and e_cs < TOL_PARAM


def loss_grad(m, U_t, R12_t):
    """dL/dmeans of the mean-profile loss (summed over planes), plain numpy."""
    U, V, UV = m[..., 0], m[..., 1], m[..., 6]
    b = UV - U * V - R12_t
    dU = 2 * (U - U_t) / (U_t ** 2).sum()
    db = 2 * b / (R12_t ** 2).sum()
    d = np.zeros_like(m)
    d[..., 0] = dU - db * V
    d[..., 1] = -db * U
    d[..., 6] = db
    return d


@pytest.mark.parametrize("storage,avg,ref,n,keep,stats", [
    ("f32", "local", False, 3, True, False), ("f16dev", "local", False, 3, True, False),
    ("f32", "line", False, 3, True, False), ("f16dev", "line", False, 3, True, False),
    ("f16dev", "local", True, 3, True, False),
    ("f32", "local", False, 35, True, False), ("f16dev", "local", False, 5, False, False),
    ("f16dev", "local", False, 4, True, True), ("f16dev", "local", True, 4, True, True)])
def test_step_record_matches_step(storage, avg, ref, n, keep, stats):
    """The recompute entry point reproduces lbm_step bit for bit (same kernels,
    caller buffers) and keeps the inlet plane of every step (planes of up to 32
    steps from one launch: n = 35 spans two; keep=False: planes not kept).
    stats: the forward steps accumulate statistics at two planes while the recompute
    runs with them detached, as in a gradient sweep (with FP16 storage the sampled
    planes keep their kernel, whose rounding differs from the bulk kernel's)."""
    case = Case(8, 8, 70, ywall="slip", xbc="inflow", wall_model=True, storage=storage, g=(2e-6, 0.0, 0.0),
                wall_avg=avg, reference=ref)
    ch = case.ch
    if stats:
        ch.stats_attach([2, 5])
        ch.stats_detach()
    f0, h0 = [t.clone() for t in ch.state()]
    t0 = ch.time
    ring_f = [torch.empty_like(f0) for _ in range(n)]
    ring_h = [torch.empty_like(h0) for _ in range(n)]
    ring_u = [torch.empty((3, 8, 70), dtype=torch.float32, device="cuda") for _ in range(n)] if keep else None
    ring_fl = [torch.empty((3, 8, 70), dtype=torch.float32, device="cuda") for _ in range(n)] if keep else None
    ch.step_record(f0, h0, t0, ring_f, ring_h, ring_u, ring_fl)
    if stats:
        ch.stats_attach([2, 5])
    valid = torch.ones_like(f0, dtype=torch.bool)  # bricks (x, zc, y, i, z%64): padding nodes z >= nz are unwritten
    valid[:, -1, :, :, 70 - 64:] = False
    for k in range(n):
        ch.step(1)
        f, h = ch.state()
        assert torch.equal(f[valid], ring_f[k][valid]), k
        assert torch.equal(h, ring_h[k]), k
        if keep:
            assert torch.equal(ch.u_in, ring_u[k]), k
            assert torch.equal(ch.fluct, ring_fl[k]), k
    ch.sync()


def test_gradient_matches_fp64_finite_differences():
    """GPU adjoint gradient of the mean-profile loss against central differences
    (h = 1e-4) of the FP64 oracle's forward run, on the 64 x 32 x 32 channel of the
    oracle configuration over 30 steps with the loss at x = 8: 7 amplitude bins and C_s.
    Bound 1e-4 relative to the largest FD component (the gradient target)."""
    nx, ny, nz, T = 64, 32, 32, 30
    case = Case(nx, ny, nz, ywall="slip", xbc="inflow", wall_model=True, tau0=0.52, n_modes=100, seed=1)
    planes = [8]
    f0 = storage_round(case.f_or, "f32")
    h0 = np.asarray(case.hist_or, dtype=np.float32).astype(np.float64)
    case.ch.load_populations(torch.as_tensor(f0, dtype=torch.float32))
    case.ch.state()[1].copy_(torch.as_tensor(h0, dtype=torch.float32))
    U_t = case.U_or[0] * 1.02
    R12_t = case.R[1]
    stg = case.stg_or

    def loss_of(amp, cs):
        cfg = O.make_cfg(nx, ny, nz, ywall=2, xbc=1, wall_model=1, tau0=0.52, cs_smag=cs)
        s2 = O.StgInputs(stg.q, stg.sigma, stg.kmag, stg.d, stg.phi, stg.omega, stg.u_rans, stg.R, amp, stg.bin_of_y)
        acc = np.zeros((1, ny, 9))
        st, _, _ = O.run(cfg, f0, h0, 0.0, T, stg=s2, planes=planes, acc=acc)
        assert st == O.OK
        m = acc / (nz * T)
        U, V, UV = m[0, :, 0], m[0, :, 1], m[0, :, 6]
        return ((U - U_t) ** 2).sum() / (U_t ** 2).sum() + ((UV - U * V - R12_t) ** 2).sum() / (R12_t ** 2).sum()

    run = StatsGradient(case.ch, planes, T, segment=6)
    means = run.forward()
    g = run.backward(loss_grad(means, U_t, R12_t))
    bins = [1, 5, 10, 15, 21, 26, 30]
    h = 1e-4
    amp0 = stg.amp_bin.copy()
    fd = []
    for b in bins:
        e = np.zeros_like(amp0)
        e[b] = h
        fd.append((loss_of(amp0 + e, 0.1) - loss_of(amp0 - e, 0.1)) / (2 * h))
    fd.append((loss_of(amp0, 0.1 + h) - loss_of(amp0, 0.1 - h)) / (2 * h))
    fd = np.array(fd)
    ad = np.append(g[bins], g[-1])
    err = np.abs(ad - fd).max() / np.abs(fd).max()
    print("FD", fd, "\nadjoint", ad, "\nrel err %.2e" % err, flush=True)
    assert np.abs(fd).max() > 0
    assert err < 1e-4
