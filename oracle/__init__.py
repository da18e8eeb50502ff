"""FP64 CPU oracle of the STG wall-modelled MRT-LBM channel step (arXiv 2304.04214).

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()`` and
the CPU-baseline leg of ``bench.py`` may import this package.  It shares no code
with the HIP library ``paper_2304_04214_amd``; it is compiled from
``oracle.cpp`` with g++ (``build()``), and reached through ctypes.

Parity status per function (see the pins in ``tests/test_oracle_*.py``):
every function below is pinned by a closed form, an identity or a printed
value of the paper, except the whole-system step at turbulent sizes, whose
agreement with anything but the HIP path is unpinned by the paper (it gives no
worked example); its parts are pinned one by one.  The adjoint step is pinned
by the definition of an adjoint: its inner products with random directions
equal central finite differences of the forward step (tests/test_oracle_adjoint.py).
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, ERR_ARG, ERR_MACH, ERR_NONFINITE, ERR_NEWTON = 0, 1, 4, 5, 7

# Appendix A.1 free rates (reading: omega_0,3,5,7 = 1, omega_1 = 1.19);
# 9, 11, 13, 14, 15 are overwritten by 1/tau_eff inside the collision.
PAPER_RATES = [1.0, 1.19, 1.6, 1.0, 1.2, 1.0, 1.2, 1.0, 1.2, 1.0,
               1.6, 1.0, 1.6, 1.0, 1.0, 1.0, 1.98, 1.98, 1.98]


def build(force=True):
    """Compile oracle.cpp into liboracle.so (g++, OpenMP, -O2)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


class Cfg(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("ywall", C.c_int32), ("xbc", C.c_int32), ("wall_model", C.c_int32),
                ("newton_max", C.c_int32), ("sponge_cells", C.c_int32),
                ("newton_tol", C.c_double), ("tau0", C.c_double), ("cs_smag", C.c_double),
                ("s", C.c_double * 19), ("kappa", C.c_double), ("b_reich", C.c_double),
                ("y_wall", C.c_double), ("u_conv", C.c_double), ("g", C.c_double * 3), ("sponge_nu", C.c_double),
                ("outlet", C.c_int32), ("wall_law", C.c_int32), ("wall_avg", C.c_int32), ("pad_", C.c_int32)]


class Stg(C.Structure):
    _fields_ = [("n_modes", C.c_int32), ("n_bins", C.c_int32),
                ("q", C.c_void_p), ("sigma", C.c_void_p), ("kmag", C.c_void_p), ("d", C.c_void_p),
                ("phi", C.c_void_p), ("omega", C.c_void_p), ("u_rans", C.c_void_p), ("R", C.c_void_p),
                ("amp_bin", C.c_void_p), ("bin_of_y", C.c_void_p), ("k_rans", C.c_void_p),
                ("omega_rans", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        _lib = C.CDLL(_LIB)
        P = C.c_void_p
        D = C.c_double
        I = C.c_int
        sig = {
            "oracle_set_mutation": (None, [I]),
            "oracle_tables": (None, [P] * 6),
            "oracle_feq": (None, [D, P, P]),
            "oracle_meq": (None, [D, P, P]),
            "oracle_guo": (None, [P, P, P]),
            "oracle_collide_node": (None, [P, P, P, P, P, P]),
            "oracle_tau_eff": (D, [D, D, D, D]),
            "oracle_uplus": (D, [D, D, D]),
            "oracle_duplus": (D, [D, D, D]),
            "oracle_uplus_musker": (D, [D]),
            "oracle_duplus_musker": (D, [D]),
            "oracle_utau": (I, [P, D, P]),
            "oracle_wall_force": (I, [P, D, P, P, I, P, P]),
            "oracle_inlet_node": (None, [P, P, P, P]),
            "oracle_cholesky": (None, [P, P]),
            "oracle_stg_plane": (I, [P, P, D, P, P]),
            "oracle_stg_weights": (I, [P, P, I, P]),
            "oracle_wall_lines": (I, [P, P, D, P, P, P, P]),
            "oracle_reichardt_inflow": (None, [P, D, P]),
            "oracle_init": (I, [P, P, P, P, D, P, P]),
            "oracle_stream_only": (I, [P, P, P]),
            "oracle_step": (I, [P, P, D, P, P, P, P, P, I, P, P]),
            "oracle_step_uin": (I, [P, P, P, P, P, P, P, I, P]),
            "oracle_adjoint_step": (I, [P, P, D, P, P, P, P, P, P, I, P, P, P, P, P, P]),
            "oracle_step_nodes": (I, [P, P, D, P, P, C.c_int64, P, P, P]),
            "oracle_macro": (None, [P, P, P, P]),
            "oracle_run": (I, [P, P, D, I, P, P, P, I, P, P]),
            "oracle_num_threads": (I, []),
            "oracle_set_num_threads": (None, [I]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(_lib, name)
            fn.restype = res
            fn.argtypes = args
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def make_cfg(nx, ny, nz, *, ywall=0, xbc=0, wall_model=0, tau0=0.52, cs_smag=0.1, rates=None,
             kappa=0.41, b_reich=7.8, y_wall=0.5, u_conv=0.1, g=(0.0, 0.0, 0.0),
             newton_max=50, newton_tol=1e-14, sponge_cells=0, sponge_nu=0.0, outlet=0, wall_law=0,
             wall_avg=0):
    c = Cfg()
    c.nx, c.ny, c.nz = nx, ny, nz
    c.ywall, c.xbc, c.wall_model = ywall, xbc, wall_model
    c.newton_max, c.newton_tol = newton_max, newton_tol
    c.tau0, c.cs_smag = tau0, cs_smag
    for i, v in enumerate(rates if rates is not None else PAPER_RATES):
        c.s[i] = v
    c.kappa, c.b_reich, c.y_wall, c.u_conv = kappa, b_reich, y_wall, u_conv
    for a in range(3):
        c.g[a] = g[a]
    c.sponge_cells, c.sponge_nu = sponge_cells, sponge_nu
    c.outlet = outlet
    c.wall_law = wall_law
    c.wall_avg = wall_avg
    return c


class StgInputs:
    """Host FP64 STG inputs with their ctypes view (keeps arrays alive)."""

    def __init__(self, q, sigma, kmag, d, phi, omega, u_rans, R, amp_bin, bin_of_y, k_rans=None, omega_rans=None):
        self.q, self.sigma, self.kmag, self.d = _d(q), _d(sigma), _d(kmag), _d(d)
        self.phi, self.omega, self.u_rans, self.R = _d(phi), _d(omega), _d(u_rans), _d(R)
        self.amp_bin = _d(amp_bin)
        self.bin_of_y = np.ascontiguousarray(bin_of_y, dtype=np.int32)
        s = Stg()
        s.n_modes, s.n_bins = len(self.q), len(self.amp_bin)
        s.q, s.sigma, s.kmag, s.d = _p(self.q), _p(self.sigma), _p(self.kmag), _p(self.d)
        s.phi, s.omega, s.u_rans, s.R = _p(self.phi), _p(self.omega), _p(self.u_rans), _p(self.R)
        s.amp_bin, s.bin_of_y = _p(self.amp_bin), _p(self.bin_of_y)
        # per-row spectrum inputs (RANS k and omega); None: the table q serves every row
        self.k_rans = None if k_rans is None else _d(k_rans)
        self.omega_rans = None if omega_rans is None else _d(omega_rans)
        s.k_rans, s.omega_rans = _p(self.k_rans), _p(self.omega_rans)
        self.c = s


def _ref(x):
    return None if x is None else C.byref(x)


# ---------------- building blocks ----------------

def tables():
    c = np.zeros((19, 3), np.int32)
    w = np.zeros(19)
    M = np.zeros((19, 19))
    Mi = np.zeros((19, 19))
    opp = np.zeros(19, np.int32)
    refl = np.zeros(19, np.int32)
    lib().oracle_tables(_p(c), _p(w), _p(M), _p(Mi), _p(opp), _p(refl))
    return dict(c=c, w=w, M=M, Minv=Mi, opp=opp, refl=refl)


def set_mutation(k):
    lib().oracle_set_mutation(int(k))


def feq(rho, u):
    out = np.zeros(19)
    lib().oracle_feq(float(rho), _p(_d(u)), _p(out))
    return out


def meq(rho, u):
    out = np.zeros(19)
    lib().oracle_meq(float(rho), _p(_d(u)), _p(out))
    return out


def guo(u, F):
    out = np.zeros(19)
    lib().oracle_guo(_p(_d(u)), _p(_d(F)), _p(out))
    return out


def collide_node(cfg, f, F):
    out = np.zeros(19)
    tau = np.zeros(1)
    u = np.zeros(3)
    lib().oracle_collide_node(C.byref(cfg), _p(_d(f)), _p(_d(F)), _p(out), _p(tau), _p(u))
    return out, float(tau[0]), u


def tau_eff(Qhalf, rho, tau0, cs):
    return lib().oracle_tau_eff(Qhalf, rho, tau0, cs)


def uplus(yp, kappa=0.41, B=7.8):
    return lib().oracle_uplus(float(yp), kappa, B)


def uplus_musker(yp):
    return lib().oracle_uplus_musker(float(yp))


def duplus_musker(yp):
    return lib().oracle_duplus_musker(float(yp))


def duplus(yp, kappa=0.41, B=7.8):
    return lib().oracle_duplus(float(yp), kappa, B)


def utau(cfg, uhat_abs):
    out = np.zeros(1)
    st = lib().oracle_utau(C.byref(cfg), float(uhat_abs), _p(out))
    return st, float(out[0])


def wall_force(cfg, rho_w, uw, u2, top):
    F = np.zeros(3)
    ut = np.zeros(1)
    st = lib().oracle_wall_force(C.byref(cfg), float(rho_w), _p(_d(uw)), _p(_d(u2)), int(top), _p(F), _p(ut))
    return st, F, float(ut[0])


def inlet_node(f, uin):
    out = np.zeros(19)
    r = np.zeros(1)
    lib().oracle_inlet_node(_p(_d(f)), _p(_d(uin)), _p(out), _p(r))
    return out, float(r[0])


def cholesky(R6):
    a = np.zeros(6)
    lib().oracle_cholesky(_p(_d(R6)), _p(a))
    return a


def stg_plane(cfg, stg, t, want_fluct=False):
    uin = np.zeros((3, cfg.ny, cfg.nz))
    fl = np.zeros((3, cfg.ny, cfg.nz)) if want_fluct else None
    st = lib().oracle_stg_plane(C.byref(cfg), C.byref(stg.c), float(t), _p(uin), _p(fl))
    return (st, uin, fl) if want_fluct else (st, uin)


def stg_weights(cfg, stg, y):
    """Spectral weights q^n of inlet row y (the bound table, or the per-row spectrum)."""
    q = np.zeros(stg.c.n_modes)
    st = lib().oracle_stg_weights(C.byref(cfg), C.byref(stg.c), int(y), _p(q))
    return st, q


def wall_lines(cfg, f, hist, t_next, stg=None):
    """Line-averaged wall model (reading R23): (status, signed line u_tau [2][nx], u_hat [2][nx][nz])."""
    line = np.zeros((2, cfg.nx))
    uhat = np.zeros((2, cfg.nx, cfg.nz))
    st = lib().oracle_wall_lines(C.byref(cfg), _ref(None if stg is None else stg.c), float(t_next), _p(_d(f)),
                                 _p(None if hist is None else _d(hist)), _p(line), _p(uhat))
    return st, line, uhat


def reichardt_inflow(cfg, u_tau):
    out = np.zeros((3, cfg.ny))
    lib().oracle_reichardt_inflow(C.byref(cfg), float(u_tau), _p(out))
    return out


# ---------------- lattice operations ----------------

def shape(cfg):
    return (19, cfg.nx, cfg.ny, cfg.nz)


def init(cfg, u, rho=None, pert=None, eps=0.0):
    """f = f_eq(rho, u) + eps w pert; returns (f[19,nx,ny,nz], hist[5,ny,nz])."""
    f = np.zeros(shape(cfg))
    hist = np.zeros((5, cfg.ny, cfg.nz))
    u = _d(u)
    rho = None if rho is None else _d(rho)
    pert = None if pert is None else _d(pert)
    st = lib().oracle_init(C.byref(cfg), _p(rho), _p(u), _p(pert), float(eps), _p(f), _p(hist))
    assert st == OK, st
    return f, hist


def stream_only(cfg, f):
    out = np.zeros(shape(cfg))
    st = lib().oracle_stream_only(C.byref(cfg), _p(_d(f)), _p(out))
    assert st == OK, st
    return out


def step(cfg, f, hist, t_next, stg=None, planes=None, acc=None, wall_acc=None):
    """One step; returns (status, f_new, hist_new).  acc[p,ny,9] accumulates sums in place;
    wall_acc[2, nx] (bottom, top) accumulates the sums over z of the wall law's u_tau."""
    out = np.empty(shape(cfg))
    hist_out = hist.copy() if hist is not None else None
    pl = None if planes is None else np.ascontiguousarray(planes, dtype=np.int32)
    st = lib().oracle_step(C.byref(cfg), _ref(stg.c if stg is not None else None), float(t_next),
                           _p(_d(f)), _p(out), _p(None if hist is None else _d(hist)), _p(hist_out),
                           _p(pl), 0 if pl is None else len(pl), _p(acc), _p(wall_acc))
    return st, out, hist_out


def step_uin(cfg, f, hist, uin, planes=None, acc=None):
    """One step with the inlet velocity plane uin[3,ny,nz] given; returns (status, f_new, hist_new)."""
    out = np.empty(shape(cfg))
    hist_out = hist.copy() if hist is not None else None
    pl = None if planes is None else np.ascontiguousarray(planes, dtype=np.int32)
    st = lib().oracle_step_uin(C.byref(cfg), _p(None if uin is None else _d(uin)), _p(_d(f)), _p(out),
                               _p(None if hist is None else _d(hist)), _p(hist_out),
                               _p(pl), 0 if pl is None else len(pl), _p(acc))
    return st, out, hist_out


def adjoint_step(cfg, f, hist, t_next, lam_next, eta_next=None, stg=None, uin=None, planes=None, coef=None,
                 want_amp=False):
    """Adjoint of step(f, hist, t_next): returns dict(status, lam, eta, g_uin, g_cs, g_amp).

    lam_next = dL/ds_{n+1}, eta_next = dL/dhist_{n+1}, coef[p, y, 9] = dL/d(each
    statistics sum of this step) or None.  uin, when given, replaces the STG plane.
    """
    ny, nz = cfg.ny, cfg.nz
    lam = np.zeros(shape(cfg))
    open_ = cfg.xbc == 1
    eta = np.zeros((5, ny, nz)) if open_ else None
    if open_ and eta_next is None:
        eta_next = np.zeros((5, ny, nz))
    g_uin = np.zeros((3, ny, nz)) if open_ else None
    g_cs = np.zeros(1)
    g_amp = np.zeros(len(stg.amp_bin)) if (want_amp and stg is not None) else None
    pl = None if planes is None else np.ascontiguousarray(planes, dtype=np.int32)
    st = lib().oracle_adjoint_step(
        C.byref(cfg), _ref(stg.c if stg is not None else None), float(t_next), _p(None if uin is None else _d(uin)),
        _p(_d(f)), _p(None if hist is None else _d(hist)), _p(_d(lam_next)),
        _p(None if eta_next is None else _d(eta_next)), _p(pl), 0 if pl is None else len(pl),
        _p(None if coef is None else _d(coef)), _p(lam), _p(eta), _p(g_uin), _p(g_cs), _p(g_amp))
    return dict(status=st, lam=lam, eta=eta, g_uin=g_uin, g_cs=float(g_cs[0]), g_amp=g_amp)


def gradient_run(cfg, stg, f0, hist0, t0, nsteps, planes, coef, sample_from=1, want_states=False):
    """Loss gradient over nsteps steps from (f0, hist0) at time t0 by the adjoint.

    The loss depends on the statistics sums acc accumulated over the steps
    n = sample_from..nsteps (step n produces the state at time t0 + n);
    coef[p, y, 9] = dL/dacc.  Returns dict(g_amp, g_cs, lam0, acc): the gradient
    with respect to the amplitude scalings s_b and C_s, dL/df0, and acc.
    All forward states are kept in memory (small lattices only).
    """
    open_ = cfg.xbc == 1
    states = [(_d(f0).copy(), None if hist0 is None else _d(hist0).copy())]
    acc = np.zeros((len(planes), cfg.ny, 9))
    for n in range(1, nsteps + 1):
        f, h = states[-1]
        st, f1, h1 = step(cfg, f, h, t0 + n, stg=stg if open_ else None, planes=planes,
                          acc=acc if n >= sample_from else None)
        assert st == OK, st
        states.append((f1, h1))
    lam = np.zeros(shape(cfg))
    eta = np.zeros((5, cfg.ny, cfg.nz)) if open_ else None
    g_amp = np.zeros(len(stg.amp_bin)) if (open_ and stg is not None) else None
    g_cs = 0.0
    for n in range(nsteps, 0, -1):
        f, h = states[n - 1]
        r = adjoint_step(cfg, f, h, t0 + n, lam, eta, stg=stg if open_ else None, planes=planes,
                         coef=coef if n >= sample_from else None, want_amp=g_amp is not None)
        assert r["status"] == OK, r["status"]
        lam, eta = r["lam"], r["eta"]
        g_cs += r["g_cs"]
        if g_amp is not None:
            g_amp += r["g_amp"]
    out = dict(g_amp=g_amp, g_cs=g_cs, lam0=lam, acc=acc)
    if want_states:
        out["states"] = states
    return out


def run(cfg, f, hist, t0, nsteps, stg=None, planes=None, acc=None, wall_acc=None):
    """nsteps steps from time t0; returns (status, f, hist) as new arrays (acc, wall_acc as for step)."""
    f = _d(f).copy()
    hist = None if hist is None else _d(hist).copy()
    pl = None if planes is None else np.ascontiguousarray(planes, dtype=np.int32)
    st = lib().oracle_run(C.byref(cfg), _ref(stg.c if stg is not None else None), float(t0), int(nsteps),
                          _p(f), _p(hist), _p(pl), 0 if pl is None else len(pl), _p(acc), _p(wall_acc))
    return st, f, hist


def step_nodes(cfg, f, hist, t_next, nodes, stg=None):
    nodes = np.ascontiguousarray(nodes, dtype=np.int64)
    out = np.zeros((19, len(nodes)))
    u = np.zeros((3, len(nodes)))
    st = lib().oracle_step_nodes(C.byref(cfg), _ref(stg.c if stg is not None else None), float(t_next),
                                 _p(_d(f)), _p(None if hist is None else _d(hist)), len(nodes), _p(nodes),
                                 _p(out), _p(u))
    return st, out, u


def macro(cfg, f):
    N = cfg.nx * cfg.ny * cfg.nz
    rho = np.zeros(N)
    u = np.zeros(3 * N)
    lib().oracle_macro(C.byref(cfg), _p(_d(f)), _p(rho), _p(u))
    return rho.reshape(cfg.nx, cfg.ny, cfg.nz), u.reshape(3, cfg.nx, cfg.ny, cfg.nz)


def num_threads():
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().oracle_num_threads())


def set_num_threads(n):
    """Set the OpenMP threads of the oracle's parallel loops (n >= 1)."""
    lib().oracle_set_num_threads(int(n))
