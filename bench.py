"""Throughput of the STG wall-modelled MRT-LBM channel step on one MI355X.

One step = one pass of the whole hot path over the lattice: STG inlet plane
(mode sum, Cholesky scaling) + fused pull-stream / slip walls / convective
outlet / regularised inlet / Reichardt wall model / MRT-Smagorinsky collision
+ FP64 plane statistics on four sampled x-planes.

Workload (default): the Re_tau = 1000 channel shape 768 x 64 x 192 (x, y, z),
FP32 populations, N = 200 STG modes, synthetic inputs.  Also timed: the same
lattice with FP16-deviation storage, the Re_tau = 5200 shape
1536 x 128 x 384 in both storages, and the discrete adjoint on the
256 x 64 x 64 channel (gradient of a mean-profile loss over 400 steps with
checkpoints every 20 steps).

Prints ONE JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "MLUPS & HBM GB/s (FP32 vs FP16-store) + adjoint-step MLUPS at stated error"
HBM_PEAK_GBS = 8000.0
BYTES_PER_NODE = {"f32": 152, "f16dev": 76, "f16ref": 76}  # 19 populations read + 19 written


def log(*a):
    print(*a, file=sys.stderr, flush=True)


C5_STEPS = 5000  # the 151 M-node workload's horizon
SPONGE_NU = 0.1  # viscosity at the outlet plane of the 1-delta sponge (the paper gives no value)


def make_channel(name, storage, device, sponge=False):
    """storage: "f32", "f16dev" (half deviations from the weights) or "f16ref" (half
    deviations from the equilibrium at the mean inflow profile)."""
    import torch
    from paper_2304_04214_amd import synthetic as S
    from paper_2304_04214_amd.channel import Channel
    w = S.WORKLOADS[name]
    nx, ny, nz = w["nx"], w["ny"], w["nz"]
    delta = ny / 2
    ch = Channel(nx, ny, nz, tau0=w["tau0"], storage="f16dev" if storage == "f16ref" else storage, ywall="slip",
                 xbc="inflow", wall_model=True, cs_smag=S.CS_SMAG, u_conv=S.U_C, device=device,
                 sponge_cells=int(delta) if sponge else 0, sponge_nu=SPONGE_NU if sponge else 0.0)
    U = ch.inflow_reichardt(w["u_tau"])
    if storage == "f16ref":
        ch.set_reference(U)
    k = int(name[1])
    mt = S.mode_table(w["n_modes"], delta, seed_offset=k)
    ab, boy = S.amp_bins(ny)
    ch.set_stg(mt, U, S.reynolds_stress(ny, w["u_tau"]), ab, boy)
    g = torch.Generator(device=device)
    g.manual_seed(S.SEED_BASE + k)
    u = U.float()[:, None, :, None].expand(3, nx, ny, nz).contiguous()
    u += 1e-3 * (2 * torch.rand((3, nx, ny, nz), generator=g, device=device) - 1)
    ch.init(u)
    del u
    planes = [p for p in (int(delta), int(2 * delta), int(4 * delta), int(8 * delta)) if p < nx]
    ch.stats_attach(planes)
    return ch, (nx, ny, nz)


def time_channel(name, storage, steps, warmup, device, sponge=False):
    import torch
    ch, (nx, ny, nz) = make_channel(name, storage, device, sponge=sponge)
    N = nx * ny * nz
    ch.step(warmup)
    ch.sync()
    ch.stats_reset()
    ch.kernel_timing(2)  # reset and enable the per-launch HIP events
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ch.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    k_ms, k_n, k_nodes = ch.kernel_timing(0)
    status = "ok"
    try:
        ch.sync()
    except Exception as e:  # a latched device error is reported, not hidden
        status = str(e)
    ms = (t1 - t0) * 1e3 / steps
    kern_ms = k_ms / max(k_n, 1)
    res = dict(workload=name, storage=storage, shape=[nx, ny, nz], nodes=N, ms_per_step=ms,
               mlups=N / (ms * 1e-3) / 1e6, kernel_ms=kern_ms, kernel_launches=k_n, kernel_nodes=k_nodes,
               kernel_gbs=BYTES_PER_NODE[storage] * k_nodes / (kern_ms * 1e-3) / 1e9, status=status)
    ch.close()
    del ch
    torch.cuda.empty_cache()
    return res


ADJ_BYTES_PER_NODE = 228  # s_n read + lam_{n+1} read + lam_n written, 19 floats each


def time_adjoint(device, name="c4", storage="f32", steps=400, segment=20, warmup=20):
    """Gradient of the mean-profile loss at x = 4 delta over `steps` steps w.r.t. the
    amplitude scalings (one bin per row) and C_s: forward with checkpoints, then the
    checkpointed adjoint sweep (recompute included).  Workloads: the 256 x 64 x 64
    channel (FP32, 400 steps, checkpoints every 20) and the 512 x 64 x 128 channel
    (FP16-deviation storage, 2000 steps, checkpoints every 45 ~ sqrt(2000))."""
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
    ch.kernel_timing(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ch.step(steps)
    torch.cuda.synchronize()
    fwd_ms = (time.perf_counter() - t0) * 1e3 / steps
    k_ms, k_n, _ = ch.kernel_timing(0)
    fwd_kernel_ms = k_ms / max(k_n, 1)
    run = StatsGradient(ch, [x_obs], steps, segment=segment)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    means = run.forward()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    m = torch.tensor(means, dtype=torch.float64, requires_grad=True)
    U_t = torch.as_tensor(ch._stg_tensors["u_rans"][0].cpu())
    R12_t = torch.as_tensor(S.reynolds_stress(ny, w["u_tau"])[1])
    loss = mean_profile_loss(m[0], U_t, R12_t)
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    g, adj_ms_total = run.backward(m.grad.numpy(), time_kernel=True)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    status = "ok"
    try:
        ch.sync()
    except Exception as e:
        status = str(e)
    adj_ms = adj_ms_total / steps
    bpn = ADJ_BYTES_PER_NODE if storage == "f32" else ADJ_BYTES_PER_NODE - 38  # s_n in half deviations
    res = dict(workload="%dx%dx%d channel (%s), loss at x=%d over %d steps, checkpoint every %d" % (
        nx, ny, nz, "FP32" if storage == "f32" else "FP16-deviation storage", x_obs, steps, segment),
        nodes=N, forward_ms_per_step=round(fwd_ms, 5),
        forward_kernel_ms=round(fwd_kernel_ms, 5), adjoint_step_ms=round(adj_ms, 5),
        adjoint_mlups=round(N / (adj_ms * 1e-3) / 1e6, 1),
        adjoint_vs_forward=round(adj_ms / fwd_ms, 3),
        roofline={"bound": "hbm", "achieved": round(bpn * N / (adj_ms * 1e-3) / 1e9, 1),
                  "peak": HBM_PEAK_GBS, "unit": "GB/s",
                  "frac": round(bpn * N / (adj_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                  "traffic": measured_traffic("adjoint_traffic_256x64x64.json", "c4:adjoint") if name == "c4" else None,
                  "kernel": "adjoint_kernel<%s> (one launch per adjoint step)" % storage,
                  "bytes_per_node": bpn},
        gradient_forward_ms=round((t1 - t0) * 1e3, 3), gradient_backward_ms=round((t3 - t2) * 1e3, 3),
        backward_vs_forward_end_to_end=round((t3 - t2) / (t1 - t0), 3),
        loss=float(loss), grad_cs=float(g[-1]), grad_amp_linf=float(np.abs(g[:-1]).max()), status=status)
    ch.close()
    del ch, run
    torch.cuda.empty_cache()
    return res


def fp16_profile_error(device, name="c3", spin=1000, window=1000):
    """Error of the FP16 storages in the mean statistics: U(y) and <u'v'>(y) at the four
    statistics planes over steps spin+1 .. spin+window of the Re_tau = 5200 shape, FP16
    against FP32 storage from the same initial state (the FP64 oracle cannot run this
    lattice for thousands of steps; the FP32 path matches it to 1e-5 per step).  U error
    relative to max U, stress error relative to max |R12| of the synthetic inputs."""
    import numpy as np
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


def cpu_baseline(target_s=15.0):
    """The FP64 oracle on the host cores, on an x-slab of the Re_tau=1000 workload."""
    import oracle as O
    from paper_2304_04214_amd import synthetic as S
    w = S.WORKLOADS["c2"]
    nx, ny, nz = 16, w["ny"], w["nz"]
    cfg = O.make_cfg(nx, ny, nz, ywall=2, xbc=1, wall_model=1, tau0=w["tau0"], cs_smag=S.CS_SMAG, u_conv=S.U_C)
    U = O.reichardt_inflow(cfg, w["u_tau"])
    mt = S.mode_table(w["n_modes"], ny / 2, seed_offset=2)
    ab, boy = S.amp_bins(ny)
    stg = O.StgInputs(mt["q"], mt["sigma"], mt["kmag"], mt["d"], mt["phi"], mt["omega"], U,
                      S.reynolds_stress(ny, w["u_tau"]), ab, boy)
    du, _ = S.perturbations(nx, ny, nz, seed_offset=2)
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
                sample="x-slab %dx%dx%d of the 768x64x192 Re_tau=1000 workload (same boundaries, STG N=200), "
                       "%d steps, %.1f s on %d threads; %d steps, %.1f s on one thread" % (
                           nx, ny, nz, steps, dt, cores, steps1, dt1))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-accuracy", action="store_true", help="skip the FP16 mean-profile error leg")
    ap.add_argument("--only", default=None, help="time one (workload:storage), e.g. c2:f32 (profiling)")
    ap.add_argument("--copy-only", action="store_true", help="run the 2 GiB copy kernel only (counter calibration)")
    ap.add_argument("--adj-steps", type=int, default=400, help="steps of the adjoint workload (loss horizon)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the library runs on one GPU only (the path shards over x-slabs by design, "
              "not implemented here); use --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    device = torch.device("cuda:0")
    if args.copy_only:
        print(json.dumps({"copy_kernel_gbs": copy_bandwidth(device, reps=args.steps)}), flush=True)
        return
    if args.only == "adjoint":
        print(json.dumps(time_adjoint(device, steps=args.adj_steps)), flush=True)
        return
    if args.only == "adjoint-large":
        print(json.dumps(time_adjoint(device, "c5a", "f16dev", steps=2000, segment=45)), flush=True)
        return
    if args.only:
        name, storage = args.only.split(":")[:2]
        r = time_channel(name, storage, args.steps, args.warmup, device, sponge=args.only.endswith(":sponge"))
        print(json.dumps(r), flush=True)
        return
    log("bench: c2 f32")
    main_r = time_channel("c2", "f32", args.steps, args.warmup, device)
    log("bench: c2 f16dev / f16ref")
    r16 = time_channel("c2", "f16dev", args.steps, args.warmup, device)
    r16r = time_channel("c2", "f16ref", args.steps, args.warmup, device)
    log("bench: c2 f32 with the outlet sponge")
    rsp = time_channel("c2", "f32", args.steps, args.warmup, device, sponge=True)
    log("bench: c3 f32 / f16dev")
    c3_steps = max(10, args.steps // 5)
    r3 = time_channel("c3", "f32", c3_steps, max(5, args.warmup // 5), device)
    r3h = time_channel("c3", "f16dev", c3_steps, max(5, args.warmup // 5), device)
    r3r = time_channel("c3", "f16ref", c3_steps, max(5, args.warmup // 5), device)
    log("bench: c5 f32 1536x256x384, 5000 steps (the workload's horizon, FP64 statistics on)")
    r5 = time_channel("c5", "f32", C5_STEPS, max(3, args.warmup // 10), device)
    log("bench: adjoint 256x64x64")
    radj = time_adjoint(device, steps=args.adj_steps)
    log("bench: adjoint 512x64x128 FP16")
    radj5 = time_adjoint(device, "c5a", "f16dev", steps=2000, segment=45)
    acc = None
    if not args.no_accuracy:
        log("bench: FP16 storage error in the mean profiles (1536x128x384, 2000 steps each)")
        acc = fp16_profile_error(device)
    log("bench: copy bandwidth")
    copy_gbs = copy_bandwidth(device)
    cpu = None
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        cpu = cpu_baseline()
    achieved = main_r["kernel_gbs"]
    out = {
        "metric": METRIC,
        "value": round(main_r["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_r["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "Re_tau=1000 channel 768x64x192 (x,y,z), FP32 SoA populations, STG inlet N=200, "
                               "slip walls + Reichardt wall model, convective outlet, 4 FP64 statistics planes",
                   "nodes": main_r["nodes"], "status": main_r["status"]},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic("collide_traffic_re1000_768x64x192.json", "c2:f32"),
                     "kernel": "collide_general_kernel<f32> (all blocks)", "kernel_ms": round(main_r["kernel_ms"], 5),
                     "kernel_nodes": main_r["kernel_nodes"],
                     "bytes_per_node": BYTES_PER_NODE["f32"], "copy_kernel_gbs": round(copy_gbs, 1),
                     "frac_of_copy": round(achieved / copy_gbs, 4)},
        "fp16dev": {"mlups": round(r16["mlups"], 1), "ms_per_step": round(r16["ms_per_step"], 5),
                    "kernel_gbs": round(r16["kernel_gbs"], 1), "vs_fp32": round(r16["mlups"] / main_r["mlups"], 3),
                    "kernel": "collide_fused_kernel<f16dev> (all blocks, one launch per step)",
                    "bytes_per_node": BYTES_PER_NODE["f16dev"], "frac": round(r16["kernel_gbs"] / HBM_PEAK_GBS, 4),
                    "traffic": measured_traffic("collide_traffic_re1000_768x64x192.json", "c2:f16dev"),
                    "status": r16["status"]},
        "fp16ref": {"storage": "half deviations from the equilibrium at the mean inflow profile",
                    "mlups": round(r16r["mlups"], 1), "ms_per_step": round(r16r["ms_per_step"], 5),
                    "kernel_gbs": round(r16r["kernel_gbs"], 1), "vs_fp32": round(r16r["mlups"] / main_r["mlups"], 3),
                    "status": r16r["status"]},
        "with_outlet_sponge": {"mlups": round(rsp["mlups"], 1), "vs_no_sponge": round(rsp["mlups"] / main_r["mlups"], 3),
                               "sponge": "last 32 planes (1 delta), nu 1.4e-4 -> %g" % SPONGE_NU,
                               "status": rsp["status"]},
        "re5200_1536x128x384": {"f32_mlups": round(r3["mlups"], 1), "f32_kernel_gbs": round(r3["kernel_gbs"], 1),
                                "f16dev_mlups": round(r3h["mlups"], 1),
                                "f16dev_kernel_gbs": round(r3h["kernel_gbs"], 1),
                                "f16dev_kernel": "collide_bulk_kernel<f16dev> (blocks away from the inlet, outlet "
                                                 "and statistics planes; their general kernel runs first)",
                                "f16dev_frac": round(r3h["kernel_gbs"] / HBM_PEAK_GBS, 4),
                                "f16dev_vs_f32": round(r3h["mlups"] / r3["mlups"], 3),
                                "f16ref_mlups": round(r3r["mlups"], 1),
                                "f16ref_kernel_gbs": round(r3r["kernel_gbs"], 1),
                                "f16ref_vs_f32": round(r3r["mlups"] / r3["mlups"], 3),
                                "status": [r3["status"], r3h["status"], r3r["status"]]},
        "re5200_1536x256x384_f32": {"steps": C5_STEPS, "mlups": round(r5["mlups"], 1),
                                    "kernel_gbs": round(r5["kernel_gbs"], 1),
                                    "frac": round(r5["kernel_gbs"] / HBM_PEAK_GBS, 4),
                                    "ms_per_step": round(r5["ms_per_step"], 5), "status": r5["status"]},
        "fp16_profile_error": acc,
        "adjoint": radj,
        "adjoint_512x64x128_fp16": radj5,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
