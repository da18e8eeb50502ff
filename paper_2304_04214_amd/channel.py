"""Python binding of the HIP channel library: device buffers from PyTorch,
every step of the method runs in the library's kernels.

    ch = Channel(768, 64, 192, tau0=..., ywall="slip", xbc="inflow", wall_model=True)
    ch.set_stg(mode_table, u_rans, R, amp_bin, bin_of_y)
    ch.init(u)                      # f = f_eq(1, u)
    ch.step(1000)
    means, n = ch.stats_read()
"""
import ctypes as C

import numpy as np
import torch

from . import _abi as A

PAPER_RATES = (1.0, 1.19, 1.6, 1.0, 1.2, 1.0, 1.2, 1.0, 1.2, 1.0,
               1.6, 1.0, 1.6, 1.0, 1.0, 1.0, 1.98, 1.98, 1.98)
_YWALL = {"periodic": A.Y_PERIODIC, "bounceback": A.Y_BOUNCEBACK, "slip": A.Y_SLIP}
_XBC = {"periodic": A.X_PERIODIC, "inflow": A.X_INFLOW}
_STORE = {"f32": A.STORE_F32, "f16dev": A.STORE_F16DEV}
_OUTLET = {"convective": A.OUTLET_CONVECTIVE, "zero-gradient": A.OUTLET_ZERO_GRADIENT}
_WALL_LAW = {"reichardt": A.WALL_REICHARDT, "musker": A.WALL_MUSKER}


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _dev(x, dtype, device):
    if isinstance(x, torch.Tensor):
        return x.to(device=device, dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device=device).contiguous()


class Channel:
    """One D3Q19 channel lattice on one GPU (state double-buffered in HBM)."""

    def __init__(self, nx, ny, nz, *, tau0, storage="f32", ywall="slip", xbc="periodic", wall_model=False,
                 cs_smag=0.1, rates=None, kappa=0.41, b_reich=7.8, y_wall=0.5, u_conv=0.1, g=(0.0, 0.0, 0.0),
                 newton_iters=4, sponge_cells=0, sponge_nu=0.0, outlet="convective", wall_law="reichardt",
                 wall_avg="local", device=None):
        self.device = torch.device(device if device is not None else "cuda")
        self.nx, self.ny, self.nz = nx, ny, nz
        self.N = nx * ny * nz
        self.storage = storage
        cfg = A.Config()
        cfg.nx, cfg.ny, cfg.nz = nx, ny, nz
        cfg.storage = _STORE[storage]
        cfg.ywall = _YWALL[ywall]
        cfg.xbc = _XBC[xbc]
        cfg.wall_model = 1 if wall_model else 0
        cfg.newton_iters = newton_iters
        cfg.tau0, cfg.cs_smag = tau0, cs_smag
        for i, v in enumerate(rates if rates is not None else PAPER_RATES):
            cfg.s[i] = v
        cfg.kappa, cfg.b_reich, cfg.y_wall, cfg.u_conv = kappa, b_reich, y_wall, u_conv
        for a in range(3):
            cfg.g[a] = g[a]
        cfg.sponge_cells, cfg.sponge_nu = int(sponge_cells), float(sponge_nu)
        cfg.outlet = _OUTLET[outlet]
        cfg.wall_law = _WALL_LAW[wall_law]
        cfg.wall_avg = {"local": A.WALL_AVG_LOCAL, "line": A.WALL_AVG_LINE}[wall_avg]
        self.cfg = cfg
        dt = torch.float32 if storage == "f32" else torch.float16
        elems = C.c_int64()
        A.check(A.lib().lbm_state_elems(C.byref(cfg), C.byref(elems)), "lbm_state_elems")
        self.zc = (nz + 63) // 64
        shape = (nx, self.zc, ny, 19, 64)  # 64-node bricks, see include/lbm.h
        assert elems.value == nx * self.zc * ny * 19 * 64
        self.f = [torch.empty(shape, dtype=dt, device=self.device) for _ in range(2)]
        self.hist = [torch.zeros((5, ny, nz), dtype=torch.float32, device=self.device) for _ in range(2)]
        self._stg = None
        h = C.c_void_p()
        stream = torch.cuda.current_stream(self.device).cuda_stream
        st = A.lib().lbm_create(C.byref(cfg), _ptr(self.f[0]), _ptr(self.f[1]), _ptr(self.hist[0]),
                                _ptr(self.hist[1]), C.c_void_p(stream), C.byref(h))
        A.check(st, "lbm_create")
        self._h = h

    # ---- lifetime ----
    def close(self):
        if getattr(self, "_h", None):
            A.lib().lbm_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- inputs ----
    def inflow_reichardt(self, u_tau):
        """Reichardt mean inflow U(y) computed by the library: device float64 [3, ny]."""
        out = torch.zeros((3, self.ny), dtype=torch.float64, device=self.device)
        A.check(A.lib().lbm_inflow_reichardt(self._h, float(u_tau), _ptr(out)), "lbm_inflow_reichardt")
        return out

    def set_stg(self, modes, u_rans, R, amp_bin, bin_of_y, want_fluct=False, k_rans=None, omega_rans=None):
        """Bind the inlet STG inputs (mode table dict q, sigma, kmag, d, phi, omega).  With RANS
        k_rans[ny] and omega_rans[ny] every row takes its own spectral weights (q is not read)."""
        dev = self.device
        keep = dict((k, _dev(modes[k], torch.float64, dev)) for k in ("q", "sigma", "kmag", "d", "phi", "omega"))
        keep["k_rans"] = None if k_rans is None else _dev(k_rans, torch.float64, dev)
        keep["omega_rans"] = None if omega_rans is None else _dev(omega_rans, torch.float64, dev)
        keep["u_rans"] = _dev(u_rans, torch.float64, dev)
        keep["R"] = _dev(R, torch.float64, dev)
        keep["amp_bin"] = _dev(amp_bin, torch.float64, dev)
        keep["bin_of_y"] = _dev(bin_of_y, torch.int32, dev)
        keep["u_in"] = torch.zeros((3, self.ny, self.nz), dtype=torch.float32, device=dev)
        keep["fluct"] = torch.zeros((3, self.ny, self.nz), dtype=torch.float32, device=dev) if want_fluct else None
        s = A.Stg()
        s.n_modes = int(keep["q"].numel())
        s.n_bins = int(keep["amp_bin"].numel())
        for k in ("q", "sigma", "kmag", "d", "phi", "omega", "u_rans", "R", "amp_bin", "bin_of_y", "k_rans",
                  "omega_rans", "u_in", "fluct"):
            setattr(s, k, None if keep[k] is None else keep[k].data_ptr())
        self._stg_tensors = keep
        self._stg = s
        self._stg_dirty = True
        return keep

    def _stg_arg(self):
        if self._stg is None:
            return None
        if self._stg_dirty:
            self._stg_dirty = False
            return C.byref(self._stg)
        return None

    def set_amp_bin(self, amp_bin):
        """Replace the amplitude scalings s_b (rebinds the STG tables on the next call)."""
        self._stg_tensors["amp_bin"].copy_(_dev(amp_bin, torch.float64, self.device))
        self._stg_dirty = True

    @property
    def u_in(self):
        return self._stg_tensors["u_in"]

    @property
    def fluct(self):
        return self._stg_tensors["fluct"]

    def init(self, u, rho=None, pert=None, eps=0.0):
        """f = f_eq(rho, u) + eps w pert in the current buffer; time index set to 0.  A float64 u
        (torch or numpy) takes the FP64 path (lbm_init_equilibrium_f64), rho and pert with it."""
        dev = self.device
        f64 = (u.dtype == torch.float64) if torch.is_tensor(u) else (np.asarray(u).dtype == np.float64)
        dt = torch.float64 if f64 else torch.float32
        u = _dev(u, dt, dev).reshape(3, self.N)
        rho = None if rho is None else _dev(rho, dt, dev).reshape(self.N)
        pert = None if pert is None else _dev(pert, dt, dev).reshape(19, self.N)
        A.check(A.lib().lbm_set_state(self._h, _ptr(self.f[0]), _ptr(self.f[1]), _ptr(self.hist[0]),
                                      _ptr(self.hist[1]), 0), "lbm_set_state")
        if f64:
            A.check(A.lib().lbm_init_equilibrium_f64(self._h, _ptr(rho), _ptr(u), _ptr(pert), float(eps)),
                    "lbm_init_equilibrium_f64")
        else:
            A.check(A.lib().lbm_init_equilibrium(self._h, _ptr(rho), _ptr(u), _ptr(pert), float(eps)),
                    "lbm_init_equilibrium")
        self._keep_init = (u, rho, pert)  # alive until the enqueued kernel has read them

    # ---- time stepping ----
    def stg_fill(self, t):
        A.check(A.lib().stg_inlet_fill(self._h, self._stg_arg(), float(t)), "stg_inlet_fill")
        return self.u_in

    def stg_fill_noalloc(self, t):
        """The inlet plane at time t from the current STG inputs, with their tables in the
        library's static device scratch (stg_inlet_fill_noalloc: no device allocation; the
        handle's bound inputs are not changed)."""
        A.check(A.lib().stg_inlet_fill_noalloc(self._h, C.byref(self._stg), float(t)), "stg_inlet_fill_noalloc")
        return self.u_in

    def step(self, n=1):
        A.check(A.lib().lbm_step(self._h, self._stg_arg(), int(n)), "lbm_step")

    def stream_only(self):
        A.check(A.lib().lbm_stream_only(self._h), "lbm_stream_only")

    def sync(self):
        A.check(A.lib().lbm_sync(self._h), "lbm_sync")

    # ---- state ----
    def _cur(self):
        fp = C.c_void_p()
        hp = C.c_void_p()
        t = C.c_int64()
        A.check(A.lib().lbm_get_state(self._h, C.byref(fp), C.byref(hp), C.byref(t)), "lbm_get_state")
        k = 0 if fp.value == self.f[0].data_ptr() else 1
        return k, t.value

    @property
    def time(self):
        return self._cur()[1]

    def state(self):
        """(populations buffer, outlet-history buffer) that hold the current state."""
        k, _ = self._cur()
        return self.f[k], self.hist[k]

    def populations(self):
        """Current state as float32 [19, nx, ny, nz] (library export)."""
        out = torch.empty((19, self.nx, self.ny, self.nz), dtype=torch.float32, device=self.device)
        A.check(A.lib().lbm_export_f32(self._h, _ptr(out)), "lbm_export_f32")
        return out

    def load_populations(self, f):
        """Overwrite the current state from float populations [19, nx, ny, nz] (library import)."""
        f = _dev(f, torch.float32, self.device).reshape(19, self.N)
        A.check(A.lib().lbm_import_f32(self._h, _ptr(f)), "lbm_import_f32")
        self._keep_import = f

    def set_reference(self, u_ref):
        """FP16 storage: store deviations from the second-order equilibrium at the per-row
        reference velocity u_ref ([3, ny] or the streamwise [ny]; None: the weights).  The
        current state is re-encoded."""
        if u_ref is not None:
            u = _dev(u_ref, torch.float64, self.device)
            if u.dim() == 1:
                u = torch.stack([u, torch.zeros_like(u), torch.zeros_like(u)])
            u = u.reshape(3, self.ny).contiguous()
        else:
            u = None
        A.check(A.lib().lbm_set_reference(self._h, _ptr(u)), "lbm_set_reference")
        self._reference = u

    def point_state(self, f_a, f_b, hist_a, hist_b, time):
        """Point the handle at caller buffers (no copy): the state is in f_a / hist_a at `time`,
        the next step writes f_b / hist_b."""
        A.check(A.lib().lbm_set_state(self._h, _ptr(f_a), _ptr(f_b), _ptr(hist_a), _ptr(hist_b), int(time)),
                "lbm_set_state")

    def set_state(self, f_cur, hist_cur, time):
        """Restore a state (checkpoint): copies into the buffers and sets the time index."""
        self.f[0].copy_(f_cur)
        self.hist[0].copy_(hist_cur)
        A.check(A.lib().lbm_set_state(self._h, _ptr(self.f[0]), _ptr(self.f[1]), _ptr(self.hist[0]),
                                      _ptr(self.hist[1]), int(time)), "lbm_set_state")

    # ---- statistics ----
    def stats_attach(self, planes):
        arr = (C.c_int32 * len(planes))(*[int(p) for p in planes])
        A.check(A.lib().lbm_stats(self._h, A.STATS_ATTACH, arr, len(planes), None, None), "lbm_stats attach")
        self._planes = list(planes)

    def stats_detach(self):
        A.check(A.lib().lbm_stats(self._h, A.STATS_DETACH, None, 0, None, None), "lbm_stats detach")

    def stats_reset(self):
        A.check(A.lib().lbm_stats(self._h, A.STATS_RESET, None, 0, None, None), "lbm_stats reset")

    def stats_read(self):
        """Means over z and sampled steps: array [n_planes, ny, 9] (u v w uu vv ww uv uw vw), n_samples."""
        out = np.zeros((len(self._planes), self.ny, 9))
        n = C.c_int64()
        A.check(A.lib().lbm_stats(self._h, A.STATS_READ, None, 0, out.ctypes.data_as(C.c_void_p), C.byref(n)),
                "lbm_stats read")
        return out, n.value

    def stats_read_wall(self):
        """Means over z and sampled steps of the wall law's u_tau: array [2, nx] (bottom, top), n_samples."""
        out = np.zeros((2, self.nx))
        n = C.c_int64()
        A.check(A.lib().lbm_stats(self._h, A.STATS_READ_WALL, None, 0, out.ctypes.data_as(C.c_void_p),
                                  C.byref(n)), "lbm_stats read wall")
        return out, n.value

    # ---- adjoint ----
    def set_cs_smag(self, cs):
        A.check(A.lib().lbm_set_cs_smag(self._h, float(cs)), "lbm_set_cs_smag")
        self.cfg.cs_smag = float(cs)

    def new_field(self):
        """A zeroed float brick field (an adjoint lam), shape (nx, zc, ny, 19, 64)."""
        return torch.zeros((self.nx, self.zc, self.ny, 19, 64), dtype=torch.float32, device=self.device)

    def field_export(self, bricks):
        out = torch.empty((19, self.nx, self.ny, self.nz), dtype=torch.float32, device=self.device)
        A.check(A.lib().lbm_field_export(self._h, _ptr(bricks), _ptr(out)), "lbm_field_export")
        return out

    def field_import(self, soa, bricks=None):
        soa = _dev(soa, torch.float32, self.device).reshape(19, self.N)
        bricks = self.new_field() if bricks is None else bricks
        A.check(A.lib().lbm_field_import(self._h, _ptr(soa), _ptr(bricks)), "lbm_field_import")
        self._keep_import = soa
        return bricks

    def adjoint_step(self, s_n, hist_n, t_next, lam_next, lam_prev, eta_next=None, eta_prev=None, coef=None,
                     g_uin=None, grad=None, u_in=None, fluct=None):
        """lam_prev = dL/ds_n (and eta_prev = dL/dhist_n) from lam_next = dL/ds_{n+1}.  The parameter
        sensitivities accumulate in the library; grad (device float64 [n_bins + 1]), when given, receives
        (dL/ds_b..., dL/dC_s) accumulated so far.  coef: [n_planes, ny, 9] statistics weights; u_in and
        fluct: the step's inlet plane if kept by step_record (else recomputed)."""
        coef = None if coef is None else _dev(coef, torch.float32, self.device)
        st = A.lib().lbm_adjoint_step(self._h, self._stg_arg(), _ptr(s_n), _ptr(hist_n), float(t_next),
                                      _ptr(lam_next), _ptr(eta_next), _ptr(lam_prev), _ptr(eta_prev), _ptr(coef),
                                      _ptr(g_uin), _ptr(grad), _ptr(u_in), _ptr(fluct))
        A.check(st, "lbm_adjoint_step")
        self._keep_coef = coef

    def step_record(self, s_start, hist_start, t_start, f_out, hist_out, uin_out=None, fluct_out=None):
        """len(f_out) steps from (s_start, hist_start) at time t_start into the given buffers, keeping
        each step's inlet plane in uin_out / fluct_out (lists of device tensors) when given."""
        n = len(f_out)
        arr = lambda ts: None if ts is None else (C.c_void_p * n)(*[t.data_ptr() for t in ts])
        st = A.lib().lbm_step_record(self._h, self._stg_arg(), _ptr(s_start), _ptr(hist_start), float(t_start), n,
                                     arr(f_out), arr(hist_out), arr(uin_out), arr(fluct_out))
        A.check(st, "lbm_step_record")

    # ---- timing ----
    def kernel_timing(self, enable):
        """(summed ms, launches, nodes per launch) of the timed interior collide kernel."""
        ms = C.c_double()
        n = C.c_int64()
        nodes = C.c_int64()
        A.check(A.lib().lbm_kernel_timing(self._h, int(enable), C.byref(ms), C.byref(n), C.byref(nodes)),
                "lbm_kernel_timing")
        return ms.value, n.value, nodes.value

    def collide_dispatches(self):
        """(dispatches per step, x-planes per dispatch) of the general collide kernel."""
        d = C.c_int32()
        p = C.c_int32()
        A.check(A.lib().lbm_collide_dispatches(self._h, C.byref(d), C.byref(p)), "lbm_collide_dispatches")
        return d.value, p.value


def copy_probe(src, dst):
    """Plain device copy kernel of the library (bandwidth calibration)."""
    nbytes = src.numel() * src.element_size()
    stream = torch.cuda.current_stream(src.device).cuda_stream
    A.check(A.lib().lbm_copy_probe(_ptr(src), _ptr(dst), nbytes, C.c_void_p(stream)), "lbm_copy_probe")


def lattice_tables():
    """The library's own lattice tables (host data): c[19,3], w[19], opp[19], refl_y[19]."""
    c = np.zeros((19, 3), np.int32)
    w = np.zeros(19)
    opp = np.zeros(19, np.int32)
    refl = np.zeros(19, np.int32)
    P = C.c_void_p
    A.lib().lbm_lattice_tables(c.ctypes.data_as(P), w.ctypes.data_as(P), opp.ctypes.data_as(P),
                               refl.ctypes.data_as(P))
    return dict(c=c, w=w, opp=opp, refl=refl)
