"""The C-ABI library loads on a host without a GPU, exports every symbol that
include/lbm.h declares, and rejects bad configurations before touching the
device.  No compute call is made here."""
import ctypes as C
import os
import re

import numpy as np

import oracle as O
from paper_2304_04214_amd import _abi as A
from paper_2304_04214_amd.channel import lattice_tables

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "lbm.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:lbm_status|void|const char\*)\s+(\w+)\s*\(", txt, flags=re.M)))


def test_every_declared_symbol_is_exported():
    names = _declared()
    assert "lbm_create" in names and "lbm_step" in names and "stg_inlet_fill" in names
    L = A.lib()
    for n in names:
        assert hasattr(L, n), n
    assert sorted(A.EXPORTED) == names


def test_library_tables_match_oracle_tables():
    a, b = lattice_tables(), O.tables()
    assert np.array_equal(a["c"], b["c"])
    assert np.array_equal(a["opp"], b["opp"])
    assert np.array_equal(a["refl"], b["refl"])
    assert np.array_equal(a["w"], b["w"])


def test_status_strings():
    for s in range(7):
        assert A.status_str(s)
    assert "Mach" in A.status_str(A.LBM_ERR_MACH) or "0.3" in A.status_str(A.LBM_ERR_MACH)


def _cfg(**kw):
    c = A.Config()
    c.nx, c.ny, c.nz = kw.get("nx", 8), kw.get("ny", 8), kw.get("nz", 8)
    c.storage = kw.get("storage", 0)
    c.ywall = kw.get("ywall", 2)
    c.xbc = kw.get("xbc", 0)
    c.wall_model = kw.get("wall_model", 0)
    c.newton_iters = 8
    c.sponge_cells, c.sponge_nu = kw.get("sponge_cells", 0), kw.get("sponge_nu", 0.0)
    c.tau0 = kw.get("tau0", 0.6)
    c.cs_smag = 0.1
    c.kappa, c.b_reich, c.y_wall = 0.41, 7.8, 0.5
    return c


def test_bad_configurations_are_rejected_without_a_device():
    L = A.lib()
    h = C.c_void_p()
    buf = C.c_void_p(256)  # never dereferenced: validation fails first
    for kw, code in [(dict(ny=3), A.LBM_ERR_SHAPE), (dict(nx=0), A.LBM_ERR_SHAPE),
                     (dict(xbc=1, nx=2), A.LBM_ERR_SHAPE), (dict(tau0=0.5), A.LBM_ERR_ARG),
                     (dict(storage=7), A.LBM_ERR_ARG), (dict(ywall=0, wall_model=1), A.LBM_ERR_ARG),
                     (dict(nx=2048, ny=2048, nz=1024), A.LBM_ERR_SHAPE),
                     (dict(sponge_cells=3), A.LBM_ERR_ARG),  # sponge needs the open channel
                     (dict(xbc=1, sponge_cells=8, sponge_nu=0.1), A.LBM_ERR_ARG),  # more planes than nx - 1
                     (dict(xbc=1, sponge_cells=3, sponge_nu=0.0), A.LBM_ERR_ARG)]:
        st = L.lbm_create(C.byref(_cfg(**kw)), buf, C.c_void_p(512), None, None, None, C.byref(h))
        assert st == code, (kw, st)
    assert L.lbm_create(None, buf, buf, None, None, None, C.byref(h)) == A.LBM_ERR_ARG
    assert L.lbm_step(None, None, 1) == A.LBM_ERR_ARG
    assert L.lbm_copy_probe(buf, buf, 15, None) == A.LBM_ERR_ARG
    assert L.lbm_init_equilibrium_f64(None, None, buf, None, 0.0) == A.LBM_ERR_ARG
    assert L.lbm_init_equilibrium(None, None, buf, None, 0.0) == A.LBM_ERR_ARG
    d, p = C.c_int32(-1), C.c_int32(-1)
    assert L.lbm_collide_dispatches(None, C.byref(d), C.byref(p)) == A.LBM_ERR_ARG
    assert (d.value, p.value) == (-1, -1)  # outputs untouched on error
