"""Gradients of plane-statistics losses by the library's discrete adjoint step.

The forward run keeps the state every `segment` steps (default about
sqrt(T)); the backward sweep recomputes each segment from its checkpoint into
a ring of state buffers (lbm_step_record, which also keeps each step's inlet
plane) and runs lbm_adjoint_step backwards through it.  Every step of both sweeps runs in the
library's kernels; this module only orders the calls and holds the buffers.

    run = StatsGradient(ch, planes=[128], nsteps=400)
    means = plane_statistics(run, amp_bin, cs)   # torch.autograd.Function
    loss = mean_profile_loss(means[0], U_target, R12_target)
    loss.backward()                              # amp_bin.grad, cs.grad
"""
import math

import numpy as np
import torch


class StatsGradient:
    """Forward statistics run and adjoint gradient sweep on one Channel.

    The channel's current state at construction is the initial state s_0 of
    every run.  Statistics are the means over z and steps 1..nsteps at the x
    planes given (lbm_stats); the gradient is taken with respect to the STG
    amplitude scalings s_b and C_s.
    """

    def __init__(self, ch, planes, nsteps, segment=None):
        self.ch = ch
        self.planes = [int(p) for p in planes]
        self.T = int(nsteps)
        self.seg = int(segment) if segment else max(1, int(round(math.sqrt(self.T))))
        f, h = ch.state()
        self.t0 = ch.time
        self.f0 = f.clone()
        self.h0 = h.clone()
        self.ckpt = []
        self._ring = None

    def forward(self):
        """Run nsteps from s_0 with statistics; returns the means [n_planes, ny, 9] (float64 numpy)."""
        ch = self.ch
        ch.set_state(self.f0, self.h0, self.t0)
        ch.stats_attach(self.planes)
        self.ckpt = []
        k = 0
        while k < self.T:
            f, h = ch.state()
            self.ckpt.append((f.clone(), h.clone(), ch.time))
            n = min(self.seg, self.T - k)
            ch.step(n)
            k += n
        means, n = ch.stats_read()
        assert n == self.T, (n, self.T)
        return means

    def _buffers(self):
        if self._ring is None:
            ch = self.ch
            f, h = ch.state()
            n = max(self.seg - 1, 1)
            plane = (3, ch.ny, ch.nz)
            self._ring = dict(f=[torch.empty_like(f) for _ in range(n)], h=[torch.empty_like(h) for _ in range(n)],
                              u=[torch.empty(plane, dtype=torch.float32, device=ch.device) for _ in range(n)],
                              fl=[torch.empty(plane, dtype=torch.float32, device=ch.device) for _ in range(n)])
            self._lam = [ch.new_field(), ch.new_field()]
            self._eta = [torch.zeros_like(h), torch.zeros_like(h)]
        return self._ring

    def backward(self, dmeans, time_kernel=False):
        """Gradient from dL/dmeans [n_planes, ny, 9]: returns float64 numpy [n_bins + 1]
        (dL/ds_b..., dL/dC_s).  With time_kernel, also the summed time of the adjoint steps in ms
        (HIP events around each segment's adjoint steps)."""
        ch = self.ch
        ring = self._buffers()
        ch.stats_detach()  # the sampled planes keep their kernel: the recompute matches the forward run bit for bit
        open_ = ch.cfg.xbc == 1
        # each step adds one z-sum per (plane, y) to the accumulators; means divide by nz T
        coef = torch.as_tensor(np.asarray(dmeans, dtype=np.float64) / (ch.nz * self.T), dtype=torch.float32,
                               device=ch.device).contiguous()
        n_bins = 0 if ch._stg is None else int(ch._stg.n_bins)
        grad = torch.zeros(n_bins + 1, dtype=torch.float64, device=ch.device)
        lam, eta = self._lam, self._eta
        for t in lam + eta:
            t.zero_()
        ev = []
        t_last = self.t0 + 1  # the sweep's last adjoint step reduces the parameter gradient
        for f_k, h_k, t_k in reversed(self.ckpt):
            L = min(self.seg, self.t0 + self.T - t_k)
            # recompute s_{t_k + j}, j = 1 .. L-1, and the inlet planes of those steps
            if L > 1:
                ch.step_record(f_k, h_k, t_k, ring["f"][:L - 1], ring["h"][:L - 1],
                               ring["u"][:L - 1] if open_ else None, ring["fl"][:L - 1] if open_ else None)
            states = [f_k] + ring["f"][:L - 1]
            hists = [h_k] + ring["h"][:L - 1]
            if time_kernel:
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record()
            for j in reversed(range(L)):
                kept = open_ and j < L - 1  # the plane of step j was kept by the recompute
                ch.adjoint_step(states[j], hists[j], t_k + j + 1, lam[0], lam[1], eta[0], eta[1], coef=coef,
                                grad=grad if t_k + j + 1 == t_last else None,
                                u_in=ring["u"][j] if kept else None, fluct=ring["fl"][j] if kept else None)
                lam.reverse()
                eta.reverse()
            if time_kernel:
                e1.record()
                ev.append((e0, e1))
        ch.point_state(ch.f[0], ch.f[1], ch.hist[0], ch.hist[1], self.t0)
        ch.set_state(self.f0, self.h0, self.t0)
        ch.sync()
        g = grad.cpu().numpy()
        if time_kernel:
            return g, sum(a.elapsed_time(b) for a, b in ev)
        return g


class _PlaneStatistics(torch.autograd.Function):
    @staticmethod
    def forward(ctx, amp_bin, cs, run):
        run.ch.set_amp_bin(amp_bin.detach().cpu().numpy())
        run.ch.set_cs_smag(float(cs))
        ctx.run = run
        return torch.as_tensor(run.forward(), dtype=torch.float64)

    @staticmethod
    def backward(ctx, gmeans):
        g = ctx.run.backward(gmeans.detach().cpu().numpy())
        return torch.as_tensor(g[:-1]), torch.as_tensor(g[-1]), None


def plane_statistics(run, amp_bin, cs):
    """Means [n_planes, ny, 9] of (u, v, w, uu, vv, ww, uv, uw, vw) as a differentiable
    function of the amplitude scalings amp_bin [n_bins] and C_s (float64 CPU tensors)."""
    return _PlaneStatistics.apply(amp_bin, cs, run)


def mean_profile_loss(means, U_target, R12_target):
    """sum_y (U - U_t)^2 / sum U_t^2 + sum_y (<u'v'> - R12)^2 / sum R12^2 for one plane's
    means [ny, 9], <u'v'> = <uv> - <u><v>."""
    U_target = torch.as_tensor(U_target, dtype=torch.float64)
    R12_target = torch.as_tensor(R12_target, dtype=torch.float64)
    U, V, UV = means[:, 0], means[:, 1], means[:, 6]
    uv = UV - U * V
    return ((U - U_target) ** 2).sum() / (U_target ** 2).sum() + ((uv - R12_target) ** 2).sum() / (R12_target ** 2).sum()
