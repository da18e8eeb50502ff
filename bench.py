"""Throughput of the STG wall-modelled MRT-LBM channel step on one MI355X.

One step = one pass of the whole hot path over the lattice: STG inlet plane
(mode sum, Cholesky scaling) + fused pull-stream / slip walls / convective
outlet / regularised inlet / Reichardt wall model / MRT-Smagorinsky collision
+ FP64 plane statistics on four sampled x-planes.

Workload of the headline line: the Re_tau = 5200 channel shape
1536 x 128 x 384 (x, y, z; 75.5 M nodes), FP32 populations, N = 300 STG
modes, synthetic inputs.  Also timed: the same lattice with FP16 storage
(deviations from the equilibrium at the mean inflow, the FP16 line of record,
and deviations from the weights), the Re_tau = 1000 shape 768 x 64 x 192 in
every storage and with the outlet sponge, the 1536 x 256 x 384 lattice in FP32
over its 5000 steps, and the discrete adjoint on 256 x 64 x 64 (gradient of a
mean-profile loss over 400 steps, checkpoints every 20) and 512 x 64 x 128
(FP16 states in both storages, 2000 steps).  Every leg is timed REPEATS times (windows of
--steps steps; at least 200 on the 768 x 64 x 192 lattice, whose steps take 0.14-0.25 ms); the
line reports the median with the min and max.

Prints ONE JSON line.
"""
import argparse
import json
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS & HBM GB/s (FP32 vs FP16-store) + adjoint-step MLUPS at stated error"
HBM_PEAK_GBS = 8000.0
BYTES_PER_NODE = {"f32": 152, "f16dev": 76, "f16ref": 76}  # 19 populations read + 19 written
REPEATS = 5
C5_STEPS = 5000  # the 151 M-node workload's horizon (REPEATS windows of C5_STEPS / REPEATS steps)
C2_MIN_STEPS = 200  # shortest timed window on the 9-19 M-node lattices (768 x 64 x 192, the 8-GPU slab)
SPONGE_NU = 0.1  # viscosity at the outlet plane of the 1-delta sponge (the paper gives no value)
PROFILES_FILE = os.path.join(ROOT, "tests", "golden", "c4_profiles.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_channel(name, storage, device, sponge=False, planes=None, seed=None, shard=0, f64_init=False):
    """storage: "f32", "f16dev" (half deviations from the weights) or "f16ref" (half
    deviations from the equilibrium at the mean inflow profile).  shard = n > 0: the x-slab
    one of n GPUs would own in the middle of the channel (nx / n planes, x-periodic in place of
    the halo exchange with its neighbours; no inlet, outlet or statistics planes)."""
    import torch
    from paper_2304_04214_amd import synthetic as S
    from paper_2304_04214_amd.channel import Channel
    w = S.WORKLOADS[name]
    nx, ny, nz = w["nx"], w["ny"], w["nz"]
    if shard:
        nx //= shard
        planes = []
    delta = ny / 2
    ch = Channel(nx, ny, nz, tau0=w["tau0"], storage="f16dev" if storage == "f16ref" else storage, ywall="slip",
                 xbc="periodic" if shard else "inflow", wall_model=True, cs_smag=S.CS_SMAG, u_conv=S.U_C,
                 device=device, sponge_cells=int(delta) if sponge else 0, sponge_nu=SPONGE_NU if sponge else 0.0)
    U = ch.inflow_reichardt(w["u_tau"])
    if storage == "f16ref":
        ch.set_reference(U)
    k = int(name[1])
    if not shard:
        mt = S.mode_table(w["n_modes"], delta, seed_offset=k)
        ab, boy = S.amp_bins(ny)
        ch.set_stg(mt, U, S.reynolds_stress(ny, w["u_tau"]), ab, boy)
    if seed is None:
        g = torch.Generator(device=device)
        g.manual_seed(S.SEED_BASE + k)
        u = U.float()[:, None, :, None].expand(3, nx, ny, nz).contiguous()
        u += 1e-3 * (2 * torch.rand((3, nx, ny, nz), generator=g, device=device) - 1)
    elif f64_init:  # the reference computations' initial state: FP64 fields, f_eq formed in FP64
        du, _ = S.perturbations(nx, ny, nz, seed_offset=seed)
        u = U[:, None, :, None] + 1e-3 * torch.as_tensor(du, device=device)
        del du
    else:  # the seeded host perturbation of the reference computations
        du, _ = S.perturbations(nx, ny, nz, seed_offset=seed, dtype=np.float32)
        u = U.float()[:, None, :, None] + 1e-3 * torch.as_tensor(du, device=device)
        del du
    ch.init(u)
    del u
    if planes is None:
        planes = [p for p in (int(delta), int(2 * delta), int(4 * delta), int(8 * delta)) if p < nx]
    if planes:
        ch.stats_attach(planes)
    return ch, (nx, ny, nz)


def _spread(vals):
    return dict(median=statistics.median(vals), min=min(vals), max=max(vals))


def time_channel(name, storage, steps, warmup, device, sponge=False, repeats=REPEATS, shard=0):
    """REPEATS timed windows of `steps` steps after `warmup` untimed steps; per window the
    wall time between two device synchronisations and the HIP-event time of the dominant
    collide launches."""
    import torch
    ch, (nx, ny, nz) = make_channel(name, storage, device, sponge=sponge, shard=shard)
    N = nx * ny * nz
    n_disp, disp_planes = ch.collide_dispatches()
    ch.step(warmup)
    ch.sync()
    if not shard:
        ch.stats_reset()
    wall, kern = [], []
    k_nodes = 0
    for _ in range(repeats):
        ch.kernel_timing(2)  # reset and enable the per-launch HIP events
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ch.step(steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        k_ms, k_n, k_nodes = ch.kernel_timing(0)
        wall.append((t1 - t0) * 1e3 / steps)
        kern.append(k_ms / max(k_n, 1))
    status = "ok"
    try:
        ch.sync()
    except Exception as e:  # a latched device error is reported, not hidden
        status = str(e)
    w, k = _spread(wall), _spread(kern)
    bpn = BYTES_PER_NODE[storage]
    res = dict(workload=name, storage=storage, shape=[nx, ny, nz], nodes=N, steps=steps, repeats=repeats,
               ms_per_step=w["median"], ms_per_step_min=w["min"], ms_per_step_max=w["max"],
               mlups=N / (w["median"] * 1e-3) / 1e6, mlups_min=N / (w["max"] * 1e-3) / 1e6,
               mlups_max=N / (w["min"] * 1e-3) / 1e6,
               step_frac=bpn * N / (w["median"] * 1e-3) / 1e9 / HBM_PEAK_GBS,
               kernel_ms=k["median"], kernel_ms_min=k["min"], kernel_ms_max=k["max"], kernel_nodes=k_nodes,
               kernel_gbs=bpn * k_nodes / (k["median"] * 1e-3) / 1e9, status=status,
               dispatches_per_step=n_disp if storage == "f32" else 1, planes_per_dispatch=disp_planes)
    res["kernel_frac"] = res["kernel_gbs"] / HBM_PEAK_GBS
    ch.close()
    del ch
    torch.cuda.empty_cache()
    return res


def brief(r, keys=("mlups", "mlups_min", "mlups_max", "ms_per_step", "kernel_ms", "kernel_gbs", "kernel_frac",
                   "step_frac", "dispatches_per_step", "status")):
    return {k: (round(r[k], 5) if isinstance(r[k], float) else r[k]) for k in keys}


ADJ_BYTES_PER_NODE = 228  # s_n read + lam_{n+1} read + lam_n written, 19 floats each


def time_adjoint(device, name="c4", storage="f32", steps=400, segment=20, warmup=20, repeats=REPEATS):
    """Gradient of the mean-profile loss at x = 4 delta over `steps` steps w.r.t. the
    amplitude scalings (one bin per row) and C_s: forward with checkpoints, then the
    checkpointed adjoint sweep (recompute included), REPEATS times.  Workloads: the
    256 x 64 x 64 channel (FP32, 400 steps, checkpoints every 20) and the 512 x 64 x 128
    channel (FP16-deviation storage, 2000 steps, checkpoints every 45 ~ sqrt(2000))."""
    import torch
    from paper_2304_04214_amd.adjoint import StatsGradient, mean_profile_loss
    from paper_2304_04214_amd import synthetic as S
    ch, (nx, ny, nz) = make_channel(name, storage, device)
    w = S.WORKLOADS[name]
    N = nx * ny * nz
    x_obs = int(4 * ny / 2)
    ch.stats_detach()
    ch.step(warmup)
    ch.sync()
    # forward step time alone (same lattice, statistics on at x_obs)
    ch.stats_attach([x_obs])
    fwd, fwd_k = [], []
    for _ in range(repeats):
        ch.kernel_timing(2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ch.step(steps)
        torch.cuda.synchronize()
        fwd.append((time.perf_counter() - t0) * 1e3 / steps)
        k_ms, k_n, _ = ch.kernel_timing(0)
        fwd_k.append(k_ms / max(k_n, 1))
    run = StatsGradient(ch, [x_obs], steps, segment=segment)
    U_t = torch.as_tensor(ch._stg_tensors["u_rans"][0].cpu())
    R12_t = torch.as_tensor(S.reynolds_stress(ny, w["u_tau"])[1])
    gf, gb, adj = [], [], []
    for _ in range(repeats):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        means = run.forward()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        m = torch.tensor(means, dtype=torch.float64, requires_grad=True)
        loss = mean_profile_loss(m[0], U_t, R12_t)
        loss.backward()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        g, adj_ms_total = run.backward(m.grad.numpy(), time_kernel=True)
        torch.cuda.synchronize()
        t3 = time.perf_counter()
        gf.append((t1 - t0) * 1e3)
        gb.append((t3 - t2) * 1e3)
        adj.append(adj_ms_total / steps)
    status = "ok"
    try:
        ch.sync()
    except Exception as e:
        status = str(e)
    adj_ms = statistics.median(adj)
    fwd_ms = statistics.median(fwd)
    bpn = ADJ_BYTES_PER_NODE if storage == "f32" else ADJ_BYTES_PER_NODE - 38  # s_n in half deviations
    achieved = bpn * N / (adj_ms * 1e-3) / 1e9
    label = {"f32": "FP32", "f16dev": "FP16 storage, deviations from the weights",
             "f16ref": "FP16 storage, deviations from the mean-inflow equilibrium"}[storage]
    res = dict(workload="%dx%dx%d channel (%s), loss at x=%d over %d steps, checkpoint every %d" % (
        nx, ny, nz, label, x_obs, steps, segment),
        nodes=N, repeats=repeats, forward_ms_per_step=round(fwd_ms, 5),
        forward_kernel_ms=round(statistics.median(fwd_k), 5), adjoint_step_ms=round(adj_ms, 5),
        adjoint_step_ms_min=round(min(adj), 5), adjoint_step_ms_max=round(max(adj), 5),
        adjoint_mlups=round(N / (adj_ms * 1e-3) / 1e6, 1),
        adjoint_vs_forward=round(adj_ms / fwd_ms, 3),
        roofline={"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": round(achieved / HBM_PEAK_GBS, 4),
                  "traffic": (measured_traffic("adjoint_traffic_256x64x64.json", "c4:adjoint") if name == "c4" else
                              measured_traffic("adjoint_traffic_512x64x128.json", "c5a:adjoint:" + storage)),
                  "kernel": "adjoint_kernel<%s> (one launch per adjoint step; time per step includes the "
                            "line-model probe when configured)" % storage,
                  "bytes_per_node": bpn},
        gradient_forward_ms=round(statistics.median(gf), 3), gradient_backward_ms=round(statistics.median(gb), 3),
        backward_vs_forward_end_to_end=round(statistics.median(gb) / statistics.median(gf), 3),
        loss=float(loss.detach()), grad_cs=float(g[-1]), grad_amp_linf=float(np.abs(g[:-1]).max()), status=status)
    ch.close()
    del ch, run
    torch.cuda.empty_cache()
    return res


def read_fd_fixture():
    """(parameter names, central differences, L0) of tests/golden/c4_fd_gradient.txt."""
    names, fd, L0 = [], [], None
    for line in open(os.path.join(ROOT, "tests", "golden", "c4_fd_gradient.txt")):
        if line.startswith("# L0"):
            L0 = float(line.split()[2])
        if line.startswith("#") or not line.strip():
            continue
        t = line.split()
        names.append(t[0])
        fd.append(float(t[3]))
    return names, np.array(fd), L0


def fd_gradient_error(device):
    """The 256 x 64 x 64 adjoint workload's gradient against the FP64 oracle's central
    differences stored in tests/golden/c4_fd_gradient.txt (mean-profile loss at x = 128 over
    400 steps, h = 1e-4, the amplitude scalings of seven rows and C_s), the HIP side started
    from the same seeded state (the library's FP64 initial equilibrium of the same FP64 fields,
    rounded to FP32 as the fixture's state is) with checkpoints every 20 steps.
    Error = max |g_adjoint - g_FD| / max |g_FD| over the eight parameters."""
    import torch
    from paper_2304_04214_amd.adjoint import StatsGradient, mean_profile_loss
    from paper_2304_04214_amd import synthetic as S
    names, fd, L0 = read_fd_fixture()
    ch, (nx, ny, nz) = make_channel("c4", "f32", device, planes=[], seed=4, f64_init=True)
    x_obs = int(4 * ny / 2)
    run = StatsGradient(ch, [x_obs], 400, segment=20)
    U_t = torch.as_tensor(ch._stg_tensors["u_rans"][0].cpu())
    R12_t = torch.as_tensor(S.reynolds_stress(ny, S.WORKLOADS["c4"]["u_tau"])[1])
    means = run.forward()
    m = torch.tensor(means, dtype=torch.float64, requires_grad=True)
    loss = mean_profile_loss(m[0], U_t, R12_t)
    loss.backward()
    g = run.backward(m.grad.numpy())
    ad = np.array([g[int(n[1:])] if n != "cs" else g[-1] for n in names])
    ch.close()
    del ch, run
    torch.cuda.empty_cache()
    return {"grad_rel_err": float(np.abs(ad - fd).max() / np.abs(fd).max()),
            "per_parameter": {n: float(abs(x - y) / np.abs(fd).max()) for n, x, y in zip(names, ad, fd)},
            "loss_rel_err": abs(float(loss.detach()) - L0) / abs(L0), "parameters": names,
            "reference": "FP64 oracle central differences, tests/golden/c4_fd_gradient.txt"}


def fp16_gradient_error(device, name="c5a", steps=2000, segment=45):
    """Error of the FP16-state gradients of the large adjoint workload (512 x 64 x 128,
    mean-profile loss at x = 128 over 2000 steps, checkpoints every 45): each FP16 storage
    against the FP32-state gradient from the same seeded initial state."""
    import torch
    from paper_2304_04214_amd.adjoint import StatsGradient, mean_profile_loss
    from paper_2304_04214_amd import synthetic as S
    res = {}
    for storage in ("f32", "f16ref", "f16dev"):
        ch, (nx, ny, nz) = make_channel(name, storage, device, planes=[2 * S.WORKLOADS[name]["ny"]], seed=5)
        x_obs = 2 * ny
        run = StatsGradient(ch, [x_obs], steps, segment=segment)
        means = run.forward()
        U_t = torch.as_tensor(ch._stg_tensors["u_rans"][0].cpu())
        R12_t = torch.as_tensor(S.reynolds_stress(ny, S.WORKLOADS[name]["u_tau"])[1])
        m = torch.tensor(means, dtype=torch.float64, requires_grad=True)
        loss = mean_profile_loss(m[0], U_t, R12_t)
        loss.backward()
        res[storage] = (float(loss.detach()), run.backward(m.grad.numpy()))
        ch.close()
        del ch, run
        torch.cuda.empty_cache()
    L32, g32 = res["f32"]
    out = dict(workload="512x64x128, loss at x=128 over %d steps, checkpoint every %d" % (steps, segment),
               reference="FP32-state gradient from the same initial state")
    for k in ("f16ref", "f16dev"):
        L, g = res[k]
        out[k] = dict(grad_rel_linf=float(np.abs(g - g32).max() / np.abs(g32).max()),
                      amp_rel_linf=float(np.abs(g[:-1] - g32[:-1]).max() / np.abs(g32[:-1]).max()),
                      cs_rel=float(abs(g[-1] - g32[-1]) / abs(g32[-1])), loss_rel=abs(L - L32) / abs(L32))
    return out


def fp16_oracle_profile_error(device):
    """Mean-profile error of every storage against the FP64 oracle at the workloads' tau0:
    the 256 x 64 x 64 channel (Re_tau = 1000 parameters, tau0 = 0.500427), means over z
    and steps 1001-2000 of U(y) and <u'v'>(y) at x = delta, 2 delta, 4 delta, against the
    oracle's values stored in tests/golden/c4_profiles.txt (written by the oracle).  The
    HIP runs start from the library's FP32 equilibrium of the same seeded velocity field
    (the oracle's start is the FP64 equilibrium rounded to float32: they differ by ~1e-8).
    U error relative to max U, stress error relative to max |R12|."""
    import torch
    from paper_2304_04214_amd import synthetic as S
    if not os.path.exists(PROFILES_FILE):
        return None
    a = np.loadtxt(PROFILES_FILE)
    planes = sorted({int(x) for x in a[:, 0]})
    ref = np.stack([a[a[:, 0] == x][:, 2:5] for x in planes])  # [plane, y, (u, v, uv)]
    w = S.WORKLOADS["c4"]
    scale = np.abs(S.reynolds_stress(w["ny"], w["u_tau"])[1]).max()
    out = dict(workload="256x64x64, tau0 %.6f, statistics over steps 1001-2000 at x = %s" % (
        w["tau0"], ", ".join(map(str, planes))), reference="FP64 oracle (tests/golden/c4_profiles.txt)")
    for storage in ("f32", "f16ref", "f16dev"):
        ch, _ = make_channel("c4", storage, device, planes=planes, seed=4)
        ch.step(1000)
        ch.stats_reset()
        ch.step(1000)
        m = ch.stats_read()[0]
        ch.close()
        del ch
        torch.cuda.empty_cache()
        eU = np.abs(m[..., 0] - ref[..., 0]).max() / np.abs(ref[..., 0]).max()
        euv = np.abs((m[..., 6] - m[..., 0] * m[..., 1]) - (ref[..., 2] - ref[..., 0] * ref[..., 1])).max() / scale
        out[storage] = {"U_rel_err": float(eU), "uv_err_of_max_R12": float(euv)}
    return out


def fp16_profile_error(device, name="c3", spin=1000, window=1000):
    """Error of the FP16 storages in the mean statistics: U(y) and <u'v'>(y) at the four
    statistics planes over steps spin+1 .. spin+window of the Re_tau = 5200 shape, FP16
    against FP32 storage from the same initial state (the FP64 oracle cannot run this
    lattice for thousands of steps).  U error relative to max U, stress error relative to
    max |R12| of the synthetic inputs."""
    import torch
    from paper_2304_04214_amd import synthetic as S
    res = {}
    for storage in ("f32", "f16dev", "f16ref"):
        ch, _ = make_channel(name, storage, device)
        ch.step(spin)
        ch.stats_reset()
        ch.step(window)
        res[storage] = ch.stats_read()[0]
        ch.close()
        del ch
        torch.cuda.empty_cache()
    w = S.WORKLOADS[name]
    scale = np.abs(S.reynolds_stress(w["ny"], w["u_tau"])[1]).max()
    b = res["f32"]
    out = dict(workload="%dx%dx%d, statistics over steps %d-%d at x = delta, 2, 4, 8 delta" % (
        w["nx"], w["ny"], w["nz"], spin + 1, spin + window), reference="FP32 storage")
    for k in ("f16dev", "f16ref"):
        a = res[k]
        eU = np.abs(a[..., 0] - b[..., 0]).max() / np.abs(b[..., 0]).max()
        euv = np.abs((a[..., 6] - a[..., 0] * a[..., 1]) - (b[..., 6] - b[..., 0] * b[..., 1])).max() / scale
        out[k] = {"U_rel_err": float(eU), "uv_err_of_max_R12": float(euv)}
    return out


def copy_bandwidth(device, nbytes=2 << 30, reps=20):
    import torch
    from paper_2304_04214_amd.channel import copy_probe
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=device).fill_(1.0)
    b = torch.empty_like(a)
    copy_probe(a, b)
    torch.cuda.synchronize()
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        copy_probe(a, b)
    e.record()
    torch.cuda.synchronize()
    ms = s.elapsed_time(e) / reps
    del a, b
    torch.cuda.empty_cache()
    return 2 * nbytes / (ms * 1e-3) / 1e9


def measured_traffic(record, key):
    """HBM bytes per launch of a kernel from a committed rocprofv3 FETCH_SIZE /
    WRITE_SIZE record (profiles/<record>), or None when one of the kernel's
    source files changed since the counters were taken."""
    import hashlib
    try:
        t = json.load(open(os.path.join(ROOT, "profiles", record)))[key]
        h = hashlib.sha256()
        for src in t["sources"]:
            h.update(open(os.path.join(ROOT, src), "rb").read())
        if h.hexdigest() != t["sources_sha256"]:
            return None
        return t["traffic_bytes"]
    except (OSError, KeyError, ValueError):
        return None


def cpu_baseline(target_s=15.0, slab=64):
    """The FP64 oracle on the host cores, on an x-slab of the Re_tau = 5200 workload."""
    import oracle as O
    from paper_2304_04214_amd import synthetic as S
    w = S.WORKLOADS["c3"]
    nx, ny, nz = slab, w["ny"], w["nz"]
    cfg = O.make_cfg(nx, ny, nz, ywall=2, xbc=1, wall_model=1, tau0=w["tau0"], cs_smag=S.CS_SMAG, u_conv=S.U_C)
    U = O.reichardt_inflow(cfg, w["u_tau"])
    mt = S.mode_table(w["n_modes"], ny / 2, seed_offset=3)
    ab, boy = S.amp_bins(ny)
    stg = O.StgInputs(mt["q"], mt["sigma"], mt["kmag"], mt["d"], mt["phi"], mt["omega"], U,
                      S.reynolds_stress(ny, w["u_tau"]), ab, boy)
    du, _ = S.perturbations(nx, ny, nz, seed_offset=3)
    f, h = O.init(cfg, U[:, None, :, None] + 1e-3 * du)
    t0 = time.perf_counter()
    O.run(cfg, f, h, 0, 1, stg=stg)
    per = time.perf_counter() - t0
    steps = max(2, min(400, int(target_s / max(per, 1e-6))))
    t0 = time.perf_counter()
    st, f, h = O.run(cfg, f, h, 0, steps, stg=stg)
    dt = time.perf_counter() - t0
    N = nx * ny * nz
    cores = O.num_threads()
    # the same slab on one thread, about a third of the time budget
    O.set_num_threads(1)
    try:
        t0 = time.perf_counter()
        O.run(cfg, f, h, 0, 1, stg=stg)
        per1 = time.perf_counter() - t0
        steps1 = max(2, min(100, int(target_s / 3 / max(per1, 1e-6))))
        t0 = time.perf_counter()
        O.run(cfg, f, h, 0, steps1, stg=stg)
        dt1 = time.perf_counter() - t0
    finally:
        O.set_num_threads(cores)
    return dict(value=N * steps / dt / 1e6, unit="MLUPS", cores=cores, kind="oracle",
                single_thread_value=N * steps1 / dt1 / 1e6,
                sample="x-slab %dx%dx%d of the 1536x128x384 Re_tau=5200 workload (same boundaries, STG N=300), "
                       "%d steps, %.1f s on %d threads; %d steps, %.1f s on one thread" % (
                           nx, ny, nz, steps, dt, cores, steps1, dt1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200, help="steps per timed window (REPEATS windows per leg)")
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the FP16 mean-profile error legs")
    ap.add_argument("--only", default=None,
                    help="time one leg: workload:storage[:sponge|:shardN] (e.g. c3:f32, c5:f32:shard8), adjoint, fd, "
                         "adjoint-large, accuracy")
    ap.add_argument("--repeats", type=int, default=REPEATS)
    ap.add_argument("--copy-only", action="store_true", help="run the 2 GiB copy kernel only (counter calibration)")
    ap.add_argument("--adj-steps", type=int, default=400, help="steps of the adjoint workload (loss horizon)")
    ap.add_argument("--adj-large-steps", type=int, default=2000,
                    help="steps of the 512x64x128 adjoint workload (--only adjoint-large[-dev]; counter runs)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU only (the path shards over x-slabs by design, "
              "not implemented here); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    device = torch.device("cuda:0")
    rep = args.repeats
    if args.copy_only:
        print(json.dumps({"copy_kernel_gbs": copy_bandwidth(device, reps=args.steps)}), flush=True)
        return
    if args.only == "adjoint":
        print(json.dumps(time_adjoint(device, steps=args.adj_steps, repeats=rep)), flush=True)
        return
    if args.only in ("adjoint-large", "adjoint-large-dev"):
        storage = "f16dev" if args.only.endswith("-dev") else "f16ref"
        print(json.dumps(time_adjoint(device, "c5a", storage, steps=args.adj_large_steps, segment=45, repeats=rep)),
              flush=True)
        return
    if args.only == "accuracy":
        print(json.dumps(fp16_oracle_profile_error(device)), flush=True)
        return
    if args.only == "fd":
        print(json.dumps(fd_gradient_error(device)), flush=True)
        return
    if args.only:
        name, storage = args.only.split(":")[:2]
        shard = int(args.only.split(":shard")[1]) if ":shard" in args.only else 0
        r = time_channel(name, storage, args.steps, args.warmup, device, sponge=args.only.endswith(":sponge"),
                         repeats=rep, shard=shard)
        print(json.dumps(r), flush=True)
        return
    log("bench: c3 f32 (headline), f16ref, f16dev")
    r3 = time_channel("c3", "f32", args.steps, args.warmup, device, repeats=rep)
    r3r = time_channel("c3", "f16ref", args.steps, args.warmup, device, repeats=rep)
    r3h = time_channel("c3", "f16dev", args.steps, args.warmup, device, repeats=rep)
    log("bench: c2 f32 / f16ref / f16dev / f32 with the outlet sponge")
    # the 9.4 M-node lattice's steps take 0.14-0.25 ms: windows of at least C2_MIN_STEPS steps, so
    # that each window is tens of milliseconds of back-to-back launches
    c2_steps, c2_warm = max(args.steps, C2_MIN_STEPS), max(args.warmup, 50)
    r2 = time_channel("c2", "f32", c2_steps, c2_warm, device, repeats=rep)
    r2r = time_channel("c2", "f16ref", c2_steps, c2_warm, device, repeats=rep)
    r2h = time_channel("c2", "f16dev", c2_steps, c2_warm, device, repeats=rep)
    rsp = time_channel("c2", "f32", c2_steps, c2_warm, device, sponge=True, repeats=rep)
    log("bench: c5 f32 1536x256x384, %d steps (the workload's horizon, FP64 statistics on)" % C5_STEPS)
    r5 = time_channel("c5", "f32", C5_STEPS // rep, max(3, args.warmup // 4), device, repeats=rep)
    log("bench: the per-GPU x-slab of 1536x256x384 on 8 GPUs (192x256x384, x-periodic), f32 / f16ref")
    rsh = time_channel("c5", "f32", max(args.steps, C2_MIN_STEPS), max(args.warmup, 20), device, repeats=rep, shard=8)
    rshr = time_channel("c5", "f16ref", max(args.steps, C2_MIN_STEPS), max(args.warmup, 20), device, repeats=rep,
                        shard=8)
    log("bench: adjoint 256x64x64")
    radj = time_adjoint(device, steps=args.adj_steps, repeats=rep)
    log("bench: adjoint 512x64x128 FP16 (both FP16 storages)")
    radj5 = time_adjoint(device, "c5a", "f16ref", steps=2000, segment=45, repeats=rep)
    radj5d = time_adjoint(device, "c5a", "f16dev", steps=2000, segment=45, repeats=rep)
    acc_or = acc3 = gerr = gfd = None
    if not args.no_accuracy:
        log("bench: the 256x64x64 gradient against the oracle's finite differences (400 steps)")
        gfd = fd_gradient_error(device)
        log("bench: FP16-state gradients against the FP32-state gradient (512x64x128, 2000 steps)")
        gerr = fp16_gradient_error(device)
        log("bench: mean-profile error against the FP64 oracle (256x64x64, 2000 steps per storage)")
        acc_or = fp16_oracle_profile_error(device)
        log("bench: FP16 mean-profile error against FP32 (1536x128x384, 2000 steps per storage)")
        acc3 = fp16_profile_error(device)
    log("bench: copy bandwidth")
    copy_gbs = copy_bandwidth(device)
    cpu = None
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        cpu = cpu_baseline()
    achieved = r3["kernel_gbs"]
    out = {
        "metric": METRIC,
        "value": round(r3["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "repeats": rep,
        "ms_per_step": round(r3["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "Re_tau=5200 channel 1536x128x384 (x,y,z), FP32 populations, STG inlet N=300, "
                               "slip walls + Reichardt wall model, convective outlet, 4 FP64 statistics planes",
                   "nodes": r3["nodes"], "status": r3["status"],
                   "value_min": round(r3["mlups_min"], 1), "value_max": round(r3["mlups_max"], 1),
                   "timing": "median of %d windows of %d steps (min, max beside it)" % (rep, args.steps)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic("collide_traffic_re5200_1536x128x384.json", "c3:f32"),
                     "kernel": "collide_general_kernel<f32> (all blocks; a launch is one step's %d dispatches "
                               "over x-ranges of %d planes)" % (r3["dispatches_per_step"], r3["planes_per_dispatch"]),
                     "dispatches_per_launch": r3["dispatches_per_step"], "kernel_ms": round(r3["kernel_ms"], 5),
                     "kernel_ms_min": round(r3["kernel_ms_min"], 5), "kernel_ms_max": round(r3["kernel_ms_max"], 5),
                     "kernel_nodes": r3["kernel_nodes"], "bytes_per_node": BYTES_PER_NODE["f32"],
                     "step_frac": round(r3["step_frac"], 4), "copy_kernel_gbs": round(copy_gbs, 1),
                     "frac_of_copy": round(achieved / copy_gbs, 4)},
        "fp16": {"storage": "half deviations from the equilibrium at the mean inflow profile (line of record)",
                 "workload": "1536x128x384", **brief(r3r), "vs_fp32": round(r3r["mlups"] / r3["mlups"], 3),
                 "kernel": "collide_bulk_kernel<f16, reference> (blocks away from the inlet, outlet and "
                           "statistics planes; their general kernel runs first)",
                 "traffic": measured_traffic("collide_traffic_re5200_1536x128x384.json", "c3:f16ref"),
                 "error_vs_oracle": None if acc_or is None else acc_or.get("f16ref"),
                 "error_vs_fp32_1536x128x384": None if acc3 is None else acc3.get("f16ref")},
        "fp16dev": {"storage": "half deviations from the weights", "workload": "1536x128x384", **brief(r3h),
                    "vs_fp32": round(r3h["mlups"] / r3["mlups"], 3),
                    "error_vs_oracle": None if acc_or is None else acc_or.get("f16dev"),
                    "error_vs_fp32_1536x128x384": None if acc3 is None else acc3.get("f16dev")},
        "fp32_error_vs_oracle": None if acc_or is None else acc_or.get("f32"),
        "profile_error_setup": None if acc_or is None else {k: acc_or[k] for k in ("workload", "reference")},
        "re1000_768x64x192": {"steps_per_window": c2_steps,
                              "f32": {**brief(r2), "bytes_per_node": 152},
                              "f16ref": {**brief(r2r), "vs_fp32": round(r2r["mlups"] / r2["mlups"], 3),
                                         "kernel": "collide_fused_kernel<f16, reference> (all blocks, one launch)"},
                              "f16dev": {**brief(r2h), "vs_fp32": round(r2h["mlups"] / r2["mlups"], 3),
                                         "traffic": measured_traffic("collide_traffic_re1000_768x64x192.json",
                                                                     "c2:f16dev")},
                              "f32_with_outlet_sponge": {**brief(rsp), "vs_no_sponge": round(rsp["mlups"] / r2["mlups"], 3),
                                                         "sponge": "last 32 planes (1 delta), nu 1.4e-4 -> %g" % SPONGE_NU},
                              "f32_traffic": measured_traffic("collide_traffic_re1000_768x64x192.json", "c2:f32")},
        "re5200_1536x256x384_f32": {"steps": C5_STEPS, **brief(r5),
                                    "traffic": measured_traffic("collide_traffic_re5200_1536x256x384.json", "c5:f32")},
        "shard_192x256x384": {"what": "the x-slab one of 8 GPUs would own of 1536x256x384, x-periodic in place of "
                                      "the halo exchange (not part of it); no inlet, outlet or statistics planes",
                              "f32": brief(rsh), "f16ref": {**brief(rshr), "vs_fp32": round(rshr["mlups"] / rsh["mlups"], 3)},
                              "steps_per_window": max(args.steps, C2_MIN_STEPS)},
        "adjoint": {**radj, "gradient_error_vs_oracle_fd": gfd},
        "adjoint_512x64x128_fp16": {**radj5, "storage": "half deviations from the mean-inflow equilibrium",
                                    "gradient_error_vs_fp32_state": None if gerr is None else gerr.get("f16ref")},
        "adjoint_512x64x128_fp16dev": {**radj5d, "storage": "half deviations from the weights",
                                       "gradient_error_vs_fp32_state": None if gerr is None else gerr.get("f16dev")},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
