"""Reference values of the 256 x 64 x 64 channel workload (the adjoint workload's
lattice, Re_tau = 1000 parameters), computed by the FP64 oracle alone.

    python tests/golden/c4_reference.py profiles   ->  tests/golden/c4_profiles.txt
    python tests/golden/c4_reference.py fd         ->  tests/golden/c4_fd_gradient.txt

Only ``oracle`` and the seeded input generators (``paper_2304_04214_amd.synthetic``,
which hold none of the method's arithmetic) are used.  The GPU tests import
``case`` and ``loss`` from here to start the HIP path from the same state.

* ``profiles``: 2000 steps; the means over z and steps 1001-2000 of u, v and uv
  at x = delta, 2 delta, 4 delta (Sec. IV.A: statistics after a spin-up), for the
  mean-profile error of the storage formats against the FP64 oracle.
* ``fd``: the mean-profile loss at x_obs = 4 delta over steps 1-400
  (L = sum_y (U - U_t)^2 / sum U_t^2 + sum_y (<u'v'> - R12)^2 / sum R12^2, with
  U_t the Reichardt mean inflow and R12 the prescribed shear stress of the STG
  inputs) and its central differences with h = 1e-4 with respect to the STG
  amplitude scalings s_b of rows 2, 10, 20, 31, 43, 53, 61 (Sec. III.A,
  Eq. (22)-(23)) and C_s (Sec. II.B, Eq. (13)-(15)).
About 20 and 70 minutes on 8 host threads.
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
from paper_2304_04214_amd import synthetic as S  # noqa: E402

NAME = "c4"
SEED = 4  # the workload index: seed offset of the mode table and the perturbations
X_OBS = 128  # 4 delta
STEPS = 400
FD_BINS = [2, 10, 20, 31, 43, 53, 61]
FD_H = 1e-4
PROFILE_PLANES = [32, 64, 128]  # delta, 2 delta, 4 delta
PROFILE_SPIN, PROFILE_WINDOW = 1000, 1000
PROFILES_FILE = os.path.join(HERE, "c4_profiles.txt")
FD_FILE = os.path.join(HERE, "c4_fd_gradient.txt")


def case(cs_smag=S.CS_SMAG, amp_bin=None):
    """(cfg, stg, f0, h0, U, R12): oracle configuration and STG inputs of the workload,
    the initial state f_eq(1, U(y) + 1e-3 noise) and its outlet history rounded to
    float32 (the values both sides start from), the mean inflow U [3, ny] and R12 [ny]."""
    w = S.WORKLOADS[NAME]
    nx, ny, nz = w["nx"], w["ny"], w["nz"]
    cfg = O.make_cfg(nx, ny, nz, ywall=2, xbc=1, wall_model=1, tau0=w["tau0"], cs_smag=cs_smag, u_conv=S.U_C)
    U = O.reichardt_inflow(cfg, w["u_tau"])
    mt = S.mode_table(w["n_modes"], ny / 2, seed_offset=SEED)
    R = S.reynolds_stress(ny, w["u_tau"])
    ab, boy = S.amp_bins(ny)
    if amp_bin is not None:
        ab = np.asarray(amp_bin, dtype=np.float64)
    stg = O.StgInputs(mt["q"], mt["sigma"], mt["kmag"], mt["d"], mt["phi"], mt["omega"], U, R, ab, boy)
    du, _ = S.perturbations(nx, ny, nz, seed_offset=SEED)
    f, h = O.init(cfg, U[:, None, :, None] + 1e-3 * du)
    f0 = f.astype(np.float32).astype(np.float64)
    h0 = h.astype(np.float32).astype(np.float64)
    return cfg, stg, f0, h0, U, R[1]


def loss(means, U_t, R12_t):
    """Mean-profile loss of one plane's means [ny, 9] (u v w uu vv ww uv uw vw)."""
    U, V, UV = means[:, 0], means[:, 1], means[:, 6]
    return float(((U - U_t) ** 2).sum() / (U_t ** 2).sum() + ((UV - U * V - R12_t) ** 2).sum() / (R12_t ** 2).sum())


def run_loss(amp_bin, cs):
    cfg, stg, f0, h0, U, R12 = case(cs_smag=cs, amp_bin=amp_bin)
    acc = np.zeros((1, cfg.ny, 9))
    st, _, _ = O.run(cfg, f0, h0, 0.0, STEPS, stg=stg, planes=[X_OBS], acc=acc)
    assert st == O.OK, st
    return loss(acc[0] / (cfg.nz * STEPS), U[0], R12)


def write_fd():
    ny = S.WORKLOADS[NAME]["ny"]
    amp0 = np.ones(ny)
    t0 = time.time()
    L0 = run_loss(amp0, S.CS_SMAG)
    print("L0 %.17g (%.0f s)" % (L0, time.time() - t0), flush=True)
    rows = []
    for name in ["s%d" % b for b in FD_BINS] + ["cs"]:
        vals = []
        for sgn in (1.0, -1.0):
            amp, cs = amp0.copy(), S.CS_SMAG
            if name == "cs":
                cs += sgn * FD_H
            else:
                amp[int(name[1:])] += sgn * FD_H
            vals.append(run_loss(amp, cs))
            print("%s %+g: L %.17g (%.0f s)" % (name, sgn, vals[-1], time.time() - t0), flush=True)
        rows.append((name, vals[0], vals[1], (vals[0] - vals[1]) / (2 * FD_H)))
    with open(FD_FILE, "w") as fh:
        fh.write("# Central differences of the mean-profile loss of the 256x64x64 channel (FP64 oracle),\n")
        fh.write("# written by tests/golden/c4_reference.py fd with %d threads.\n" % O.num_threads())
        fh.write("# Loss at x = %d over steps 1-%d from f_eq(1, U + 1e-3 noise) rounded to float32; h = %g;\n"
                 % (X_OBS, STEPS, FD_H))
        fh.write("# parameters: s_b of the rows below (Eq. (22)-(23), all 1) and C_s (Eq. (13)-(15), %g).\n"
                 % S.CS_SMAG)
        fh.write("# L0 %.17g\n" % L0)
        fh.write("# columns: parameter  L(+h)  L(-h)  dL/dp (central difference)\n")
        for name, lp, lm, g in rows:
            fh.write("%s %.17g %.17g %.17g\n" % (name, lp, lm, g))
    print("wrote", FD_FILE, flush=True)


def write_profiles():
    cfg, stg, f0, h0, _, _ = case()
    t0 = time.time()
    st, f, h = O.run(cfg, f0, h0, 0.0, PROFILE_SPIN, stg=stg)
    assert st == O.OK, st
    print("spin-up %d steps (%.0f s)" % (PROFILE_SPIN, time.time() - t0), flush=True)
    acc = np.zeros((len(PROFILE_PLANES), cfg.ny, 9))
    st, f, h = O.run(cfg, f, h, float(PROFILE_SPIN), PROFILE_WINDOW, stg=stg, planes=PROFILE_PLANES, acc=acc)
    assert st == O.OK, st
    print("window %d steps (%.0f s)" % (PROFILE_WINDOW, time.time() - t0), flush=True)
    m = acc / (cfg.nz * PROFILE_WINDOW)
    with open(PROFILES_FILE, "w") as fh:
        fh.write("# Means over z and steps %d-%d of u, v and uv at x = %s of the 256x64x64 channel\n"
                 % (PROFILE_SPIN + 1, PROFILE_SPIN + PROFILE_WINDOW, ", ".join(map(str, PROFILE_PLANES))))
        fh.write("# (FP64 oracle, from f_eq(1, U + 1e-3 noise) rounded to float32), written by\n")
        fh.write("# tests/golden/c4_reference.py profiles with %d threads.\n" % O.num_threads())
        fh.write("# columns: x  y  <u>  <v>  <uv>\n")
        for p, x in enumerate(PROFILE_PLANES):
            for y in range(cfg.ny):
                fh.write("%d %d %.17g %.17g %.17g\n" % (x, y, m[p, y, 0], m[p, y, 1], m[p, y, 6]))
    print("wrote", PROFILES_FILE, flush=True)


def read_profiles():
    """{x: array [ny, 3] of (<u>, <v>, <uv>)} from the stored file."""
    a = np.loadtxt(PROFILES_FILE)
    return {int(x): a[a[:, 0] == x][:, 2:5] for x in PROFILE_PLANES}


def read_fd():
    """(names, fd values, L0) from the stored file."""
    names, g, L0 = [], [], None
    for line in open(FD_FILE):
        if line.startswith("# L0"):
            L0 = float(line.split()[2])
        if line.startswith("#") or not line.strip():
            continue
        t = line.split()
        names.append(t[0])
        g.append(float(t[3]))
    return names, np.array(g), L0


if __name__ == "__main__":
    what = sys.argv[1:] or ["profiles", "fd"]
    O.build(force=False)
    for w in what:
        {"profiles": write_profiles, "fd": write_fd}[w]()
