"""Parity of the HIP path with the FP64 oracle on the same seeded inputs.

Sizes span several 64-wide z tiles with a ragged tail, y groups with a ragged
tail, and every boundary combination.  Tolerances:
  * streaming index map: bit-exact (integer-coded FP32 populations < 2^24);
  * FP32 fields over 20 steps: 1e-5 relative L-inf;
  * FP16-deviation storage over 20 steps: 2e-4 relative L-inf (half-ulp
    rounding of deviations |h| < 2^-6 is <= 2^-18 per step, about 20 such
    roundings accumulate, against max f = 1/3).
"""
import numpy as np
import pytest
import torch

import oracle as O
from paper_2304_04214_amd import _abi as A
from paper_2304_04214_amd import synthetic as S
from paper_2304_04214_amd.channel import Channel
from parity_cases import Case, reference_offsets, rel_linf
from test_gpu_adjoint import storage_round

pytestmark = [pytest.mark.gpu,
              pytest.mark.skipif(not torch.cuda.is_available(), reason="needs a GPU")]

TOL32 = 1e-5
TOL16 = 2e-4
# FP32 error relative to the largest deviation from the weights max |f - w| and to the
# largest velocity max |u| (density and momentum of the populations): the absolute
# rounding error of the O(1/3) populations, ~1e-7 after 20 steps, against flows with
# max |u| down to ~1e-2 (measured 0.9-2.8e-5 of max |f - w| and 1.6-4.2e-6 of max |u|)
TOL_DEV = 1e-4
TOL_U = 2e-5


def macro(cfg, f):
    """Density and velocity j / rho of populations [19, nx, ny, nz] (oracle's moments, FP64)."""
    return O.macro(cfg, f)


def _say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("ywall,xbc,shape", [
    ("periodic", "periodic", (5, 6, 70)),
    ("bounceback", "periodic", (5, 10, 70)),
    ("slip", "periodic", (4, 9, 3)),
    ("bounceback", "inflow", (5, 6, 130)),
    ("slip", "inflow", (6, 10, 65)),
    ("slip", "inflow", (3, 4, 1)),
])
def test_stream_index_map_bit_exact(ywall, xbc, shape):
    nx, ny, nz = shape
    _say("stream map", ywall, xbc, shape)
    ch = Channel(nx, ny, nz, tau0=0.6, ywall=ywall, xbc=xbc, wall_model=False)
    codes = np.arange(19 * nx * ny * nz, dtype=np.float64).reshape(19, nx, ny, nz)
    assert codes.max() < 2 ** 24
    ch.load_populations(codes)
    ch.stream_only()
    ch.sync()
    gpu = ch.populations().cpu().numpy().astype(np.float64)
    ocfg = O.make_cfg(nx, ny, nz, ywall={"periodic": 0, "bounceback": 1, "slip": 2}[ywall],
                      xbc={"periodic": 0, "inflow": 1}[xbc])
    ref = O.stream_only(ocfg, codes)
    assert np.array_equal(gpu, ref)


PARITY_CASES = {
    "periodic-smag-force": dict(shape=(6, 9, 70), kw=dict(ywall="periodic", xbc="periodic", wall_model=False,
                                                         g=(2e-5, -1e-5, 5e-6), tau0=0.53)),
    "bounceback-wallmodel": dict(shape=(5, 10, 70), kw=dict(ywall="bounceback", xbc="periodic", wall_model=True,
                                                           g=(1e-5, 0.0, 0.0))),
    "slip-wallmodel": dict(shape=(4, 6, 67), kw=dict(ywall="slip", xbc="periodic", wall_model=True)),
    "slip-inflow-wallmodel": dict(shape=(7, 10, 70), kw=dict(ywall="slip", xbc="inflow", wall_model=True,
                                                            n_modes=40)),
    "bounceback-inflow-ny4": dict(shape=(5, 4, 66), kw=dict(ywall="bounceback", xbc="inflow", wall_model=True)),
    "slip-inflow-nz1": dict(shape=(3, 5, 1), kw=dict(ywall="slip", xbc="inflow", wall_model=True)),
    "slip-inflow-wallmodel-sponge": dict(shape=(12, 10, 70), kw=dict(ywall="slip", xbc="inflow", wall_model=True,
                                                                    sponge_cells=6, sponge_nu=0.02)),
    "slip-inflow-zero-gradient-outlet": dict(shape=(7, 10, 70), kw=dict(ywall="slip", xbc="inflow", wall_model=True,
                                                                       outlet="zero-gradient")),
    "slip-inflow-musker-wall-law": dict(shape=(6, 10, 70), kw=dict(ywall="slip", xbc="inflow", wall_model=True,
                                                                  wall_law="musker")),
    "bounceback-inflow-musker-wall-law": dict(shape=(6, 9, 66), kw=dict(ywall="bounceback", xbc="inflow",
                                                                       wall_model=True, wall_law="musker")),
    "slip-inflow-row-spectrum": dict(shape=(7, 10, 70), kw=dict(ywall="slip", xbc="inflow", wall_model=True,
                                                               n_modes=120, spectrum=True)),
    "slip-inflow-line-averaged-utau": dict(shape=(7, 10, 70), kw=dict(ywall="slip", xbc="inflow", wall_model=True,
                                                                     wall_avg="line")),
    "bounceback-periodic-line-averaged-utau": dict(shape=(5, 9, 66), kw=dict(ywall="bounceback", xbc="periodic",
                                                                            wall_model=True, g=(1e-5, 0.0, 0.0),
                                                                            wall_avg="line")),
    "re1000-like": dict(shape=(8, 12, 64), kw=dict(ywall="slip", xbc="inflow", wall_model=True,
                                                  tau0=0.5004270558446486, u_tau=0.004448498381757104,
                                                  n_modes=50)),
}


@pytest.mark.parametrize("name", list(PARITY_CASES))
def test_fp32_fields_match_oracle_over_20_steps(name):
    spec = PARITY_CASES[name]
    _say("parity", name, spec["shape"])
    c = Case(*spec["shape"], **spec["kw"])
    c.ch.step(20)
    c.ch.sync()
    st, f_or, hist_or, _ = c.run_oracle(20)
    assert st == O.OK
    f_g, hist_g = c.gpu_state()
    err = rel_linf(f_g, f_or)
    dev = np.abs(f_g - f_or).max() / np.abs(f_or - O.tables()["w"][:, None, None, None]).max()
    rho_g, u_g = macro(c.ocfg, f_g)
    rho_or, u_or = macro(c.ocfg, f_or)
    e_rho = rel_linf(rho_g, rho_or)
    e_u = np.abs(u_g - u_or).max() / np.abs(u_or).max()
    _say("  rel Linf %.3e   (vs max |f - w|: %.3e; rho %.3e, u vs max |u| %.3e)" % (err, dev, e_rho, e_u))
    assert err <= TOL32
    # the deviations from the weights carry the flow: FP32 rounding of O(1/3) populations
    # (absolute ~1e-7 after 20 steps) against max |f - w| and max |u| of the case
    assert dev <= TOL_DEV and e_rho <= TOL32 and e_u <= TOL_U
    if c.xbc == "inflow":
        assert rel_linf(hist_g, hist_or) <= TOL32


def test_c1_oracle_config_50_steps():
    """The 64x32x32 FP64-oracle configuration (bounce-back walls, wall model, STG N=100,
    tau 0.52, C_s 0.1) in FP32 on the GPU: fields after 20 and 50 steps."""
    _say("c1 config")
    c = Case(64, 32, 32, ywall="bounceback", xbc="inflow", wall_model=True, tau0=0.52, cs_smag=0.1,
             n_modes=100, seed=1)
    c.ch.step(20)
    c.ch.sync()
    st, f20, h20, _ = c.run_oracle(20)
    assert st == O.OK
    f_g, _ = c.gpu_state()
    e20 = rel_linf(f_g, f20)
    c.ch.step(30)
    c.ch.sync()
    st, f50, _ = O.run(c.ocfg, f20, h20, 20, 30, stg=c.stg_or)
    f_g, _ = c.gpu_state()
    e50 = rel_linf(f_g, f50)
    _say("  rel Linf 20 steps %.3e, 50 steps %.3e" % (e20, e50))
    assert e20 <= TOL32
    assert e50 <= 5 * TOL32


@pytest.mark.parametrize("wall_avg", ["local", "line"])
def test_fp32_x_range_dispatches_full_field(wall_avg):
    """A lattice of 96,000 blocks (12000 x 32 x 8: every z-chunk holds 8 of its 64 lanes), whose
    FP32 step goes out as three dispatches of 4000 x-planes: every node and the statistics of
    the planes on both sides of the two dispatch boundaries after 5 steps, against the oracle;
    the local and the line-averaged wall model (the line kernel runs once per step, before the
    dispatches)."""
    _say("x-range dispatches 12000x32x8", wall_avg)
    c = Case(12000, 32, 8, ywall="slip", xbc="inflow", wall_model=True, n_modes=24, seed=7, wall_avg=wall_avg)
    assert c.ch.collide_dispatches() == (3, 4000)
    planes = [3999, 4000, 7999, 8000]
    c.ch.stats_attach(planes)
    c.ch.step(5)
    means, n = c.ch.stats_read()
    assert n == 5
    st, f_or, hist_or, acc = c.run_oracle(5, planes=planes)
    assert st == O.OK
    f_g, hist_g = c.gpu_state()
    err = rel_linf(f_g, f_or)
    e_s = np.abs(means - acc / (5 * c.nz)).max() / np.abs(acc / (5 * c.nz)).max()
    _say("  rel Linf %.3e, outlet history %.3e, statistics %.3e" % (err, rel_linf(hist_g, hist_or), e_s))
    assert err <= TOL32 and rel_linf(hist_g, hist_or) <= TOL32 and e_s <= TOL32


@pytest.mark.parametrize("storage", ["f32", "f16dev", "f16ref"])
def test_fp64_initial_equilibrium_matches_oracle(storage):
    """lbm_init_equilibrium_f64 (Eq. (27) from FP64 fields, with a perturbation): the stored
    state is the oracle's FP64 state rounded once to the storage.  FP32: at most one unit in
    the last place (the two FP64 evaluations differ in operation order only); FP16: the
    deviations within one half-precision rounding of the oracle's.  The outlet history is the
    state's outlet plane."""
    nx, ny, nz = 8, 10, 70
    cfg = O.make_cfg(nx, ny, nz, ywall=2, xbc=1, wall_model=1, tau0=0.52, cs_smag=0.1, u_conv=0.1)
    U = O.reichardt_inflow(cfg, 0.008369396673286735)
    du, dp = S.perturbations(nx, ny, nz, seed_offset=3)
    u = U[:, None, :, None] + 1e-3 * du
    f_or, h_or = O.init(cfg, u, pert=dp, eps=0.05)
    ch = Channel(nx, ny, nz, tau0=0.52, storage="f16dev" if storage == "f16ref" else storage, ywall="slip",
                 xbc="inflow", wall_model=True, u_conv=0.1)
    dref = None
    if storage == "f16ref":
        U_g = ch.inflow_reichardt(0.008369396673286735)
        ch.set_reference(U_g)
        dref = reference_offsets(U_g.cpu().numpy())
    ch.init(u, pert=dp, eps=0.05)
    ch.sync()
    f_g, h_g = ch.populations().cpu().numpy().astype(np.float64), ch.state()[1].cpu().numpy().astype(np.float64)
    ch.close()
    if storage == "f32":
        ulp = np.abs(f_g - f_or.astype(np.float32)) / np.spacing(np.abs(f_or).astype(np.float32))
        _say("  FP32: max %.1f ulp, %.2e of the values differ" % (ulp.max(), np.mean(ulp > 0)))
        assert ulp.max() <= 1.0
    else:
        w = O.tables()["w"][:, None, None, None]
        r = 0.0 if dref is None else dref.astype(np.float64)[:, None, :, None]
        h_exact = f_or - w - r
        h_got = f_g - w - r
        bound = np.spacing(np.abs(h_exact).astype(np.float16)).astype(np.float64) + 1e-12
        _say("  FP16: max |h - h_oracle| / half ulp %.2f" % (np.abs(h_got - h_exact) / bound).max())
        assert np.all(np.abs(h_got - h_exact) <= bound)
    assert np.abs(h_g - h_or.astype(np.float32)).max() <= np.spacing(np.float32(1.0))


def test_copy_probe_copies_bit_exactly():
    """The bandwidth reference kernel (non-temporal loads and stores) copies every byte, also
    for a size that ends inside a block of threads."""
    from paper_2304_04214_amd.channel import copy_probe
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    for n in (1 << 20, (1 << 20) + 4 * 37):  # floats: whole blocks, and a ragged tail of 37 float4
        src = torch.rand(n, generator=g, device="cuda")
        dst = torch.zeros_like(src)
        copy_probe(src, dst)
        torch.cuda.synchronize()
        assert torch.equal(src, dst)


def test_statistics_match_oracle():
    c = Case(8, 10, 70, ywall="slip", xbc="inflow", wall_model=True, n_modes=30)
    planes = [1, 4, 7]
    c.ch.step(3)
    c.ch.stats_attach(planes)
    c.ch.step(10)
    means, n = c.ch.stats_read()
    assert n == 10
    _, f3, h3, _ = c.run_oracle(3)
    acc = np.zeros((3, c.ny, 9))
    O.run(c.ocfg, f3, h3, 3, 10, stg=c.stg_or, planes=planes, acc=acc)
    ref = acc / (10 * c.nz)
    err = np.abs(means - ref).max() / np.abs(ref).max()
    _say("stats rel err %.3e" % err)
    assert err <= TOL32


@pytest.mark.parametrize("storage,law,avg", [("f32", "reichardt", "local"), ("f16dev", "reichardt", "local"),
                                            ("f32", "musker", "local"), ("f32", "reichardt", "line"),
                                            ("f16dev", "reichardt", "line")])
def test_wall_statistics_match_oracle(storage, law, avg):
    """Mean over z and steps of the wall law's u_tau at every x, both walls."""
    c = Case(9, 10, 70, ywall="slip", xbc="inflow", wall_model=True, n_modes=30, storage=storage, wall_law=law,
             wall_avg=avg)
    c.ch.stats_attach([4])
    c.ch.step(12)
    wall, n = c.ch.stats_read_wall()
    assert n == 12
    acc = np.zeros((2, c.nx))
    st, _, _ = O.run(c.ocfg, c.f_or, c.hist_or, 0, 12, stg=c.stg_or, wall_acc=acc)
    assert st == O.OK
    ref = acc / (12 * c.nz)
    err = np.abs(wall - ref).max() / np.abs(ref).max()
    _say("wall stats (%s) rel err %.3e" % (storage, err))
    assert err <= (1e-5 if storage == "f32" else 2e-3)


@pytest.mark.parametrize("t,spectrum", [(0.0, False), (1.0, False), (137.0, False), (5000.0, False), (3.0, True),
                                        (4321.0, True)])
def test_stg_plane_matches_oracle(t, spectrum):
    # amplitudes raised to exercise the FP32 mode sum, below the inlet Mach guard
    c = Case(4, 10, 70, ywall="slip", xbc="inflow", wall_model=True, n_modes=300, amp_scale=2.0 if spectrum else 3.0,
             spectrum=spectrum)
    u = c.ch.stg_fill(t).cpu().numpy()
    st, ref, fl = O.stg_plane(c.ocfg, c.stg_or, t, want_fluct=True)
    assert st == O.OK
    err = np.abs(u - ref).max() / np.abs(ref).max()
    errf = np.abs(c.ch.fluct.cpu().numpy() - fl).max() / np.abs(fl).max()
    _say("stg t=%g rel err %.3e fluct %.3e" % (t, err, errf))
    assert err <= TOL32 and errf <= 1e-5 * 50


def test_reichardt_inflow_matches_oracle_fp64():
    c = Case(4, 64, 8, ywall="slip", xbc="inflow", wall_model=True, tau0=0.5004270558446486,
             u_tau=0.004448498381757104)
    assert np.abs(c.U_g.cpu().numpy() - c.U_or).max() <= 1e-13 * np.abs(c.U_or).max()


def test_lattice_tables_match_oracle_tables():
    from paper_2304_04214_amd.channel import lattice_tables
    a, b = lattice_tables(), O.tables()
    assert np.array_equal(a["c"], b["c"]) and np.array_equal(a["opp"], b["opp"])
    assert np.array_equal(a["refl"], b["refl"]) and np.array_equal(a["w"], b["w"])


def test_invalid_row_spectrum_is_reported():
    """Non-ascending wavenumbers with the per-row spectrum: LBM_ERR_ARG at the next sync;
    a wall-free lattice refuses the spectrum when it is bound."""
    c = Case(4, 6, 8, ywall="slip", xbc="inflow", wall_model=False, n_modes=16, spectrum=True)
    c.ch.sync()
    mt = dict(c.mt)
    mt["kmag"] = mt["kmag"][::-1].copy()
    c.ch.set_stg(mt, c.U_g, c.R, c.ab, c.boy, k_rans=c.k_om[0], omega_rans=c.k_om[1])
    c.ch.stg_fill(1.0)
    with pytest.raises(A.LbmError) as e:
        c.ch.sync()
    assert e.value.status == A.LBM_ERR_ARG
    c.ch.sync()
    p = Channel(4, 6, 8, tau0=0.52, ywall="periodic", xbc="inflow", wall_model=False)
    p.set_stg(c.mt, c.U_g, c.R, c.ab, c.boy, k_rans=c.k_om[0], omega_rans=c.k_om[1])
    with pytest.raises(A.LbmError) as e:
        p.stg_fill(1.0)
    assert e.value.status == A.LBM_ERR_ARG


def test_non_spd_reynolds_stress_is_reported():
    """A Reynolds-stress row that is not positive definite (R22 < R21^2 / R11, so the
    Cholesky factor of Eq. (24) does not exist): LBM_ERR_ARG at the next sync, and that row
    takes a zero factor (its inlet velocity is the mean inflow), the other rows are
    unchanged."""
    c = Case(4, 6, 8, ywall="slip", xbc="inflow", wall_model=False, n_modes=16)
    c.ch.stg_fill(3.0)
    c.ch.sync()
    good = c.ch.u_in.clone()
    R = c.R.copy()
    R[2, 2] = 0.5 * R[1, 2] ** 2 / R[0, 2]  # row 2: R22 - a21^2 < 0
    c.ch.set_stg(c.mt, c.U_g, R, c.ab, c.boy)
    c.ch.stg_fill(3.0)
    with pytest.raises(A.LbmError) as e:
        c.ch.sync()
    assert e.value.status == A.LBM_ERR_ARG
    c.ch.sync()  # cleared once reported
    U = c.U_g.float()
    assert torch.equal(c.ch.u_in[:, 2, :], U[:, 2, None].expand(3, c.nz))
    rows = [y for y in range(c.ny) if y != 2]
    assert torch.equal(c.ch.u_in[:, rows, :], good[:, rows, :])


@pytest.mark.parametrize("storage", ["f32", "f16dev"])
def test_wall_model_degenerate_branches(storage):
    """The wall model's degenerate branches (Sec. II.C, Eq. (18)-(21)): a lattice uniform in x
    and z whose populations are dyadic numbers (every moment exact in FP32 and FP64), at rest
    except for an x momentum in row 1 (bottom: u_2 tangential, u_w = 0, so u_hat = 0) and in
    row ny-1 (top: u_w tangential, u_2 = 0, so the base vector e_x of Eq. (18) is undefined).
    Both give F_w = 0: one step equals the step without the wall model bit for bit, the wall
    statistics report u_tau = 0 exactly (FP32; with FP16 storage no plane is sampled, so
    every block takes the bulk kernel, which sums the exactly representable deviations),
    and the oracle agrees."""
    nx, ny, nz = 4, 8, 70
    f = np.full((19, nx, ny, nz), 1.0 / 32.0)
    f[9] = 1.0 - 18.0 / 32.0  # rho = 1
    for y in (1, ny - 1):  # c = (-1,0,0) is i = 8, (1,0,0) is i = 10
        f[10, :, y, :] += 1.0 / 64.0
        f[8, :, y, :] -= 1.0 / 64.0
    out = {}
    for wm in (True, False):
        ch = Channel(nx, ny, nz, tau0=0.52, storage=storage, ywall="slip", xbc="periodic", wall_model=wm,
                     cs_smag=0.1)
        ch.load_populations(torch.as_tensor(f, dtype=torch.float32))
        stats = wm and storage == "f32"
        if stats:
            ch.stats_attach([1])
        ch.step(1)
        ch.sync()
        out[wm] = ch.populations()
        if stats:
            wall, n = ch.stats_read_wall()
            assert n == 1 and not wall.any(), wall
        ch.close()
    assert torch.equal(out[True], out[False])
    cfg = O.make_cfg(nx, ny, nz, ywall=2, xbc=0, wall_model=1, tau0=0.52, cs_smag=0.1)
    f0 = storage_round(f, storage)
    wall_acc = np.zeros((2, nx))
    st, f1, _ = O.step(cfg, f0, None, 1.0, wall_acc=wall_acc)
    assert st == O.OK and not wall_acc.any()
    err = rel_linf(out[True].cpu().numpy(), f1)
    _say("degenerate wall model (%s): rel Linf vs oracle %.3e" % (storage, err))
    assert err <= (TOL32 if storage == "f32" else TOL16)


def test_mach_guard_is_reported():
    c = Case(4, 6, 8, ywall="slip", xbc="inflow", wall_model=False, n_modes=4)
    c.ch.sync()
    c.ch._stg_tensors["u_rans"][0].fill_(0.2)
    c.ch._stg_dirty = True
    c.ch.stg_fill(1.0)
    with pytest.raises(A.LbmError) as e:
        c.ch.sync()
    assert e.value.status == A.LBM_ERR_MACH
    c.ch.sync()  # the error is cleared once reported


def test_nonfinite_density_is_reported():
    c = Case(4, 6, 8, ywall="slip", xbc="periodic", wall_model=False)
    c.ch.sync()
    f = c.ch.populations()
    f[3, 1, 2, 5] = float("nan")
    c.ch.load_populations(f)
    c.ch.step(1)
    with pytest.raises(A.LbmError) as e:
        c.ch.sync()
    assert e.value.status == A.LBM_ERR_NONFINITE


@pytest.mark.parametrize("storage", ["f32", "f16dev"])
def test_degenerate_calls(storage):
    """Calls whose result is fixed without the oracle: zero steps change nothing; with every
    amplitude scaling s_b = 0 the inlet plane is the mean inflow exactly (Eq. (22)); the adjoint
    of lam = eta = 0 without a statistics source is zero everywhere, gradients included
    (the step's transpose is linear)."""
    c = Case(6, 8, 70, ywall="slip", xbc="inflow", wall_model=True, storage=storage)
    ch = c.ch
    p0, h0 = ch.populations().clone(), ch.state()[1].clone()  # the nodes (the bricks' padding is never written)
    t0 = ch.time
    ch.step(0)
    assert ch.time == t0 and torch.equal(p0, ch.populations()) and torch.equal(h0, ch.state()[1])
    ch.set_amp_bin(np.zeros(len(c.ab)))
    ch.stg_fill(7.0)
    ch.sync()
    U = c.U_g.float()[:, :, None].expand(3, c.ny, c.nz)
    assert torch.equal(ch.u_in, U)
    ch.set_amp_bin(np.ones(len(c.ab)))
    lam_n, lam_p = ch.new_field(), ch.new_field()
    lam_n.zero_()
    lam_p.fill_(1.0)
    eta_n = torch.zeros((5, c.ny, c.nz), dtype=torch.float32, device="cuda")
    eta_p = torch.ones_like(eta_n)
    g_uin = torch.ones((3, c.ny, c.nz), dtype=torch.float32, device="cuda")
    grad = torch.zeros(len(c.ab) + 1, dtype=torch.float64, device="cuda")
    f_cur, h_cur = ch.state()
    ch.adjoint_step(f_cur, h_cur, t0 + 1.0, lam_n, lam_p, eta_n, eta_p, g_uin=g_uin, grad=grad)
    ch.sync()
    assert not ch.field_export(lam_p).any()
    assert not eta_p.any() and not g_uin.any() and not grad.any()


@pytest.mark.parametrize("storage,ref,avg", [("f32", False, "local"), ("f16dev", False, "local"),
                                             ("f16dev", True, "local"), ("f32", False, "line")])
def test_checkpoint_resume_is_bit_exact(storage, ref, avg):
    """A run resumed from a checkpoint (the populations, their outlet history and the step index,
    restored with lbm_set_state) continues bit for bit like the uninterrupted run: populations,
    outlet history and the last inlet plane, also when the resumed calls split the steps (and so
    the batches of inlet planes) differently."""
    c = Case(7, 10, 70, ywall="slip", xbc="inflow", wall_model=True, storage=storage, reference=ref,
             wall_avg=avg, n_modes=40)
    ch = c.ch
    ch.stats_attach([2, 4])
    ch.step(5)
    f_k, h_k = [t.clone() for t in ch.state()]
    t_k = ch.time
    ch.step(40)
    p_ref, h_ref, u_ref = ch.populations().clone(), ch.state()[1].clone(), ch.u_in.clone()
    ch.set_state(f_k, h_k, t_k)
    ch.step(13)
    ch.step(27)
    ch.sync()
    assert ch.time == t_k + 40
    assert torch.equal(ch.populations(), p_ref)
    assert torch.equal(ch.state()[1], h_ref)
    assert torch.equal(ch.u_in, u_ref)


@pytest.mark.parametrize("name", ["slip-inflow-wallmodel", "periodic-smag-force", "slip-inflow-wallmodel-sponge",
                                  "slip-inflow-musker-wall-law", "slip-inflow-line-averaged-utau",
                                  "bounceback-wallmodel", "bounceback-inflow-ny4", "slip-inflow-nz1",
                                  "bounceback-periodic-line-averaged-utau"])
def test_fp16_deviation_storage_matches_oracle(name):
    spec = PARITY_CASES[name]
    _say("fp16 parity", name)
    c = Case(*spec["shape"], storage="f16dev", **spec["kw"])
    c.ch.step(20)
    c.ch.sync()
    st, f_or, _, _ = c.run_oracle(20)
    f_g, _ = c.gpu_state()
    err = rel_linf(f_g, f_or)
    _say("  fp16 rel Linf %.3e" % err)
    assert err <= TOL16


@pytest.mark.parametrize("name", ["slip-inflow-wallmodel", "bounceback-wallmodel", "periodic-smag-force",
                                  "slip-inflow-zero-gradient-outlet", "slip-inflow-line-averaged-utau"])
def test_fp16_reference_storage_matches_oracle(name):
    """FP16 deviations from the equilibrium at the mean inflow profile (lbm_set_reference):
    20 steps against the oracle, with a smaller error than deviations from the weights
    (here the 5% population perturbation of the initial state, not the mean flow,
    dominates the stored deviations, so the gain is modest)."""
    spec = PARITY_CASES[name]
    errs = {}
    for ref in (False, True):
        c = Case(*spec["shape"], storage="f16dev", reference=ref, **spec["kw"])
        c.ch.step(20)
        c.ch.sync()
        st, f_or, _, _ = c.run_oracle(20)
        assert st == O.OK
        f_g, _ = c.gpu_state()
        errs[ref] = rel_linf(f_g, f_or)
    _say("fp16 %s: rel Linf, weights %.3e, reference profile %.3e" % (name, errs[False], errs[True]))
    assert errs[True] <= TOL16
    assert errs[True] < errs[False]


def test_reference_storage_recode_and_roundtrip():
    """Changing the reference re-encodes the state (it moves only by the rounding of the new
    deviations); import / export round trips stay within that rounding."""
    c = Case(6, 10, 70, ywall="slip", xbc="inflow", wall_model=True, storage="f16dev")
    f0 = c.ch.populations().clone()
    c.ch.set_reference(c.U_g)
    f1 = c.ch.populations().clone()
    d1 = (f1 - f0).abs().max().item()
    c.ch.load_populations(f0)
    d2 = (c.ch.populations() - f0).abs().max().item()
    c.ch.set_reference(None)
    d3 = (c.ch.populations() - f0).abs().max().item()
    c.ch.sync()
    _say("recode %.2e, round trip %.2e, back %.2e" % (d1, d2, d3))
    assert 0 < d1 <= 1e-5 and d2 <= 1e-5 and d3 <= 2e-5


def test_bad_arguments_rejected():
    with pytest.raises(A.LbmError) as e:
        Channel(4, 3, 8, tau0=0.6)  # ny < 4
    assert e.value.status == A.LBM_ERR_SHAPE
    with pytest.raises(A.LbmError) as e:
        Channel(4, 8, 8, tau0=0.5)
    assert e.value.status == A.LBM_ERR_ARG
    ch = Channel(4, 8, 8, tau0=0.6, xbc="inflow", ywall="slip")
    with pytest.raises(A.LbmError) as e:
        ch.step(1)  # no STG bound
    assert e.value.status == A.LBM_ERR_STATE


def test_fp16_mean_profiles_long_horizon():
    """Mean profiles U(y) and <u'v'>(y) over steps 501-1000 at x = 16 and 32 of
    the 64 x 32 x 32 channel (slip walls, wall model, STG inlet): FP16-deviation
    and FP32 storage against the FP64 oracle.  U error relative to max U; the
    stress error relative to the prescribed stress scale max |R12|.  Bound for
    FP16 storage 1e-3 (the mean-profile target); FP32 1e-4."""
    nx, ny, nz = 64, 32, 32
    planes = [16, 32]
    res = {}
    for storage in ("f32", "f16dev"):
        c = Case(nx, ny, nz, ywall="slip", xbc="inflow", wall_model=True, tau0=0.52, n_modes=100, seed=3,
                 storage=storage)
        c.ch.step(500)
        c.ch.stats_attach(planes)
        c.ch.step(500)
        means, n = c.ch.stats_read()
        assert n == 500
        res[storage] = means
    st, f5, h5, _ = c.run_oracle(500)
    assert st == O.OK
    acc = np.zeros((2, ny, 9))
    st, _, _ = O.run(c.ocfg, f5, h5, 500, 500, stg=c.stg_or, planes=planes, acc=acc)
    assert st == O.OK
    ref = acc / (500 * nz)
    U_ref = ref[..., 0]
    uv_ref = ref[..., 6] - ref[..., 0] * ref[..., 1]
    scale = np.abs(c.R[1]).max()
    for storage, bound in (("f32", 1e-4), ("f16dev", 1e-3)):
        m = res[storage]
        eU = np.abs(m[..., 0] - U_ref).max() / np.abs(U_ref).max()
        euv = np.abs(m[..., 6] - m[..., 0] * m[..., 1] - uv_ref).max() / scale
        _say("%s: U profile err %.3e, <u'v'> err %.3e (of max|R12|)" % (storage, eU, euv))
        assert eU <= bound and euv <= bound


def test_recovery_run_executes():
    """The inflow-recovery driver on the H = 20 channel for one domain-through time
    (statistics from the start): finite results, u_tau / u_theory near 1; with FP16 storage
    relative to the mean inflow the friction-velocity ratio stays within 2e-3 of FP32's."""
    from paper_2304_04214_amd import recovery
    r = recovery.run(1000.0, 20, periods=1, stats_from=0)
    ratio = np.asarray(r["u_tau_ratio"])
    _say("recovery: u_tau ratio range %.3f .. %.3f" % (ratio.min(), ratio.max()))
    assert np.all(np.isfinite(ratio)) and np.abs(ratio - 1).max() < 0.2
    assert all(np.isfinite(p["uv_plus_err_l2"]) for p in r["planes"])
    r16 = recovery.run(1000.0, 20, periods=1, stats_from=0, storage="f16ref")
    d = np.abs(np.asarray(r16["u_tau_ratio"]) - ratio).max()
    _say("recovery: FP16 (reference storage) u_tau ratio differs from FP32 by %.2e" % d)
    assert d < 2e-3
