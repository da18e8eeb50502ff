"""Builds one seeded channel case on both sides: the FP64 oracle and the HIP
library.  Each side computes its own mean inflow (Reichardt law), Cholesky
factors, mode amplitudes and equilibrium initial state from the same raw
synthetic inputs (paper_2304_04214_amd.synthetic)."""
import numpy as np
import torch

import oracle as O
from paper_2304_04214_amd import synthetic as S
from paper_2304_04214_amd.channel import Channel

YW = {"periodic": 0, "bounceback": 1, "slip": 2}
XB = {"periodic": 0, "inflow": 1}


def rel_linf(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def reference_offsets(u_ref):
    """FP16 storage reference offsets r_i(y) = f_eq_i(1, u_ref(y)) - w_i, float32 [19, ny]
    (the library's definition, evaluated in float64 without fused operations)."""
    t = O.tables()
    c, w = t["c"].astype(np.float64), t["w"]
    u = np.asarray(u_ref, dtype=np.float64)
    cu = c[:, 0:1] * u[0] + c[:, 1:2] * u[1] + c[:, 2:3] * u[2]
    uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2]
    return (w[:, None] * (3.0 * cu + 4.5 * cu * cu - 1.5 * uu)).astype(np.float32)


class Case:
    def __init__(self, nx, ny, nz, *, ywall="slip", xbc="inflow", wall_model=True, tau0=0.52, cs_smag=0.1,
                 u_tau=0.008369396673286735, n_modes=24, seed=0, storage="f32", g=(0.0, 0.0, 0.0), eps=0.05,
                 du_amp=1e-3, u_conv=0.1, newton_iters=4, amp_scale=1.0, rates=None, sponge_cells=0,
                 sponge_nu=0.0, outlet="convective", wall_law="reichardt", spectrum=False,
                 wall_avg="local", reference=False):
        self.nx, self.ny, self.nz = nx, ny, nz
        self.xbc = xbc
        self.ocfg = O.make_cfg(nx, ny, nz, ywall=YW[ywall], xbc=XB[xbc], wall_model=int(wall_model), tau0=tau0,
                               cs_smag=cs_smag, u_conv=u_conv, g=g, rates=rates, sponge_cells=sponge_cells,
                               sponge_nu=sponge_nu, outlet={"convective": 0, "zero-gradient": 1}[outlet],
                               wall_law={"reichardt": 0, "musker": 1}[wall_law],
                               wall_avg={"local": 0, "line": 1}[wall_avg])
        # spectrum: per-row spectral weights from synthetic RANS k, omega (the table's q is then unused)
        self.mt = S.mode_table(n_modes, ny / 2, seed_offset=seed,
                               k_range=S.spectrum_k_range(ny / 2) if spectrum else None)
        self.k_om = S.rans_k_omega(ny, u_tau) if spectrum else (None, None)
        self.R = S.reynolds_stress(ny, u_tau) * amp_scale ** 2
        self.ab, self.boy = S.amp_bins(ny)
        du, dp = S.perturbations(nx, ny, nz, seed_offset=seed)
        # ---- oracle side ----
        U_or = O.reichardt_inflow(self.ocfg, u_tau)
        u_or = U_or[:, None, :, None] + du_amp * du
        self.f_or, self.hist_or = O.init(self.ocfg, u_or, pert=dp, eps=eps)
        mt = self.mt
        self.stg_or = O.StgInputs(mt["q"], mt["sigma"], mt["kmag"], mt["d"], mt["phi"], mt["omega"], U_or,
                                  self.R, self.ab, self.boy, k_rans=self.k_om[0], omega_rans=self.k_om[1])
        # ---- HIP side ----
        self.ch = Channel(nx, ny, nz, tau0=tau0, storage=storage, ywall=ywall, xbc=xbc, wall_model=wall_model,
                          cs_smag=cs_smag, u_conv=u_conv, g=g, newton_iters=newton_iters, rates=rates,
                          sponge_cells=sponge_cells, sponge_nu=sponge_nu, outlet=outlet, wall_law=wall_law,
                          wall_avg=wall_avg)
        U_g = self.ch.inflow_reichardt(u_tau)
        self.U_g = U_g
        u_g = U_g.float()[:, None, :, None] + du_amp * torch.as_tensor(du, dtype=torch.float32, device="cuda")
        # FP16 storage as deviations from the equilibrium at the mean inflow profile
        self.dref = None
        if reference:
            self.ch.set_reference(U_g)
            self.dref = reference_offsets(U_g.cpu().numpy())
        if xbc == "inflow":
            self.ch.set_stg(self.mt, U_g, self.R, self.ab, self.boy, want_fluct=True, k_rans=self.k_om[0],
                            omega_rans=self.k_om[1])
        self.ch.init(u_g, pert=dp, eps=eps)
        self.U_or = U_or

    def run_oracle(self, nsteps, planes=None):
        acc = None if planes is None else np.zeros((len(planes), self.ny, 9))
        st, f, hist = O.run(self.ocfg, self.f_or, self.hist_or if self.xbc == "inflow" else None, 0, nsteps,
                            stg=self.stg_or if self.xbc == "inflow" else None, planes=planes, acc=acc)
        return st, f, hist, acc

    def gpu_state(self):
        f = self.ch.populations().cpu().numpy().astype(np.float64)
        _, hist = self.ch.state()
        return f, hist.cpu().numpy().astype(np.float64)
