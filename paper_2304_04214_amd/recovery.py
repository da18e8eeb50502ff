"""Inflow-recovery runs of the STG channel (the setup of Sec. IV.A).

Domain 20 delta x 2 delta x 1.6 delta (x, y, z) with H = 2 delta lattice cells
across the channel, STG inlet, slip walls with the Reichardt wall model, a
1-delta outlet sponge, run for `periods` domain-through times T = nx / U_c with
statistics from 2 T.  Reported per run (synthetic inputs: the Reichardt mean
inflow and the synthetic Reynolds stresses of paper_2304_04214_amd.synthetic;
no DNS data are involved, so nothing here is a comparison with DNS):

* u_tau / u_theory at every x / delta: the wall law's friction velocity
  averaged over z, time and both walls, over the nominal u_tau of Re_tau;
* the first x / delta from which it stays within 5 % of 1;
* <u'v'>+ (y / delta) at chosen x / delta against the prescribed R12 / u_tau^2,
  as an L2 error relative to the prescribed profile;
* U+ against the Reichardt law at the same planes.

With --spectrum the STG takes per-row spectral weights from synthetic RANS
k, omega (the spectrum of the STG that Eq. (25) cites) instead of one table.

    python -m paper_2304_04214_amd.recovery --re 1000 --h 20 [--spectrum]
"""
import argparse
import json
import time

import numpy as np
import torch

from . import synthetic as S
from .channel import Channel

SPONGE_NU = 0.1  # viscosity at the outlet plane of the 1-delta sponge (the paper gives no value)
PLANES_DELTA = (0.5, 1, 2, 3, 4, 6, 8, 10, 12, 14, 16, 18)


def setup(re_tau, H, storage="f32", n_modes=200, seed=7, spectrum=False, device="cuda"):
    delta = H // 2
    nx, ny, nz = 20 * delta, 2 * delta, int(round(1.6 * delta))
    u_tau = S.U_TAU_OF_RE[float(re_tau)]
    nu0 = u_tau * delta / re_tau
    ch = Channel(nx, ny, nz, tau0=0.5 + 3 * nu0, storage="f16dev" if storage == "f16ref" else storage,
                 ywall="slip", xbc="inflow", wall_model=True, cs_smag=S.CS_SMAG, u_conv=S.U_C, sponge_cells=delta,
                 sponge_nu=SPONGE_NU, device=device)
    U = ch.inflow_reichardt(u_tau)
    if storage == "f16ref":  # FP16 deviations from the equilibrium at the mean inflow profile
        ch.set_reference(U)
    ab, boy = S.amp_bins(ny)
    R = S.reynolds_stress(ny, u_tau)
    if spectrum:
        k, om = S.rans_k_omega(ny, u_tau)
        ch.set_stg(S.mode_table(n_modes, delta, seed_offset=seed, k_range=S.spectrum_k_range(delta)), U, R, ab, boy,
                   k_rans=k, omega_rans=om)
    else:
        ch.set_stg(S.mode_table(n_modes, delta, seed_offset=seed), U, R, ab, boy)
    g = torch.Generator(device=device)
    g.manual_seed(S.SEED_BASE + seed)
    u = U.float()[:, None, :, None].expand(3, nx, ny, nz).contiguous()
    u += 1e-3 * (2 * torch.rand((3, nx, ny, nz), generator=g, device=device) - 1)
    ch.init(u)
    return ch, dict(delta=delta, nx=nx, ny=ny, nz=nz, u_tau=u_tau, nu0=nu0, U=U[0].cpu().numpy(), R12=R[1])


def run(re_tau, H, periods=10, stats_from=2, storage="f32", spectrum=False, device="cuda"):
    ch, p = setup(re_tau, H, storage=storage, spectrum=spectrum, device=device)
    delta, nx, ny = p["delta"], p["nx"], p["ny"]
    T = int(round(nx / S.U_C))
    planes = sorted({min(int(round(d * delta)), nx - 1) for d in PLANES_DELTA})
    t0 = time.perf_counter()
    ch.step(stats_from * T)
    ch.stats_attach(planes)
    ch.step((periods - stats_from) * T)
    means, n = ch.stats_read()
    wall, _ = ch.stats_read_wall()
    ch.sync()
    wall_s = time.perf_counter() - t0
    u_tau = p["u_tau"]
    ratio = 0.5 * (wall[0] + wall[1]) / u_tau
    x_d = (np.arange(nx) + 0.5) / delta
    ok = np.abs(ratio - 1) <= 0.05
    # first x/delta from which the ratio stays within 5 % (up to the sponge)
    last = nx - delta
    bad = np.nonzero(~ok[:last])[0]
    settle = float(x_d[bad[-1] + 1]) if len(bad) and bad[-1] + 1 < last else (0.0 if not len(bad) else None)
    yd = (np.arange(ny) + 0.5) / delta
    profiles = []
    for k, x in enumerate(planes):
        m = means[k]
        uv = (m[:, 6] - m[:, 0] * m[:, 1]) / u_tau ** 2
        target = p["R12"] / u_tau ** 2
        U_plus = m[:, 0] / u_tau
        Ur = p["U"] / u_tau
        profiles.append(dict(x_delta=round(x / delta, 3),
                             uv_plus_err_l2=float(np.sqrt(((uv - target) ** 2).sum() / (target ** 2).sum())),
                             U_plus_err_max=float(np.abs(U_plus - Ur).max() / np.abs(Ur).max()),
                             uv_plus=[round(float(v), 4) for v in uv]))
    return dict(re_tau=re_tau, H=H, shape=[nx, ny, p["nz"]], storage=storage, spectrum=spectrum, steps=periods * T,
                sampled_steps=n, wall_s=round(wall_s, 2), mlups=round(nx * ny * p["nz"] * periods * T / wall_s / 1e6, 1),
                u_tau_ratio_x_delta=[round(float(v), 3) for v in x_d[::max(1, delta // 2)]],
                u_tau_ratio=[round(float(v), 4) for v in ratio[::max(1, delta // 2)]],
                settle_x_delta_5pct=settle, y_delta=[round(float(v), 3) for v in yd],
                uv_target_plus=[round(float(v), 4) for v in p["R12"] / u_tau ** 2], planes=profiles)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--re", type=float, nargs="+", default=[1000.0, 2000.0, 5200.0])
    ap.add_argument("--h", type=int, nargs="+", default=[20])
    ap.add_argument("--periods", type=int, default=10)
    ap.add_argument("--storage", default="f32", choices=["f32", "f16dev", "f16ref"],
                    help="populations in FP32, FP16 deviations from the weights, or FP16 deviations from the "
                         "equilibrium at the mean inflow profile")
    ap.add_argument("--spectrum", action="store_true", help="per-row STG spectrum from synthetic RANS k, omega")
    a = ap.parse_args()
    for re_tau in a.re:
        for H in a.h:
            print(json.dumps(run(re_tau, H, periods=a.periods, storage=a.storage, spectrum=a.spectrum)), flush=True)


if __name__ == "__main__":
    main()
