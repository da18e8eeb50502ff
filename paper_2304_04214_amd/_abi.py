"""ctypes view of the C ABI declared in include/lbm.h (argument marshalling only)."""
import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

LBM_OK, LBM_ERR_ARG, LBM_ERR_SHAPE, LBM_ERR_HIP, LBM_ERR_MACH, LBM_ERR_NONFINITE, LBM_ERR_STATE = range(7)
STORE_F32, STORE_F16DEV = 0, 1
Y_PERIODIC, Y_BOUNCEBACK, Y_SLIP = 0, 1, 2
X_PERIODIC, X_INFLOW = 0, 1
OUTLET_CONVECTIVE, OUTLET_ZERO_GRADIENT = 0, 1
WALL_REICHARDT, WALL_MUSKER = 0, 1
WALL_AVG_LOCAL, WALL_AVG_LINE = 0, 1
STATS_ATTACH, STATS_DETACH, STATS_RESET, STATS_READ, STATS_READ_WALL = 1, 2, 3, 4, 5
MAX_MODES = 1024

EXPORTED = [
    "lbm_create", "lbm_destroy", "lbm_set_state", "lbm_get_state", "lbm_init_equilibrium",
    "lbm_init_equilibrium_f64",
    "lbm_inflow_reichardt", "stg_inlet_fill", "stg_inlet_fill_noalloc", "lbm_step", "lbm_stream_only", "lbm_export_f32", "lbm_import_f32",
    "lbm_set_reference", "lbm_state_elems",
    "lbm_stats", "lbm_sync", "lbm_status_str", "lbm_kernel_timing", "lbm_collide_dispatches", "lbm_copy_probe", "lbm_lattice_tables",
    "lbm_set_cs_smag", "lbm_adjoint_step", "lbm_step_record", "lbm_field_export", "lbm_field_import",
]


class Config(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("storage", C.c_int32),
                ("ywall", C.c_int32), ("xbc", C.c_int32), ("wall_model", C.c_int32), ("newton_iters", C.c_int32),
                ("sponge_cells", C.c_int32), ("outlet", C.c_int32), ("wall_law", C.c_int32), ("wall_avg", C.c_int32),
                ("tau0", C.c_double), ("cs_smag", C.c_double), ("s", C.c_double * 19),
                ("kappa", C.c_double), ("b_reich", C.c_double), ("y_wall", C.c_double),
                ("u_conv", C.c_double), ("g", C.c_double * 3), ("sponge_nu", C.c_double)]


class Stg(C.Structure):
    _fields_ = [("n_modes", C.c_int32), ("n_bins", C.c_int32),
                ("q", C.c_void_p), ("sigma", C.c_void_p), ("kmag", C.c_void_p), ("d", C.c_void_p),
                ("phi", C.c_void_p), ("omega", C.c_void_p), ("u_rans", C.c_void_p), ("R", C.c_void_p),
                ("amp_bin", C.c_void_p), ("bin_of_y", C.c_void_p), ("k_rans", C.c_void_p),
                ("omega_rans", C.c_void_p), ("u_in", C.c_void_p), ("fluct", C.c_void_p)]


class LbmError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        super().__init__("%s: %s (status %d)" % (where, status_str(status), status))


_lib = None


def lib():
    """The loaded HIP library; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblbm.so is not built (%s); run __graft_entry__.build() or "
                               "python -m paper_2304_04214_amd.build" % LIB_PATH)
        L = C.CDLL(LIB_PATH)
        P, I32, I64, D = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        sig = {
            "lbm_create": [P, P, P, P, P, P, P],
            "lbm_destroy": [P],
            "lbm_set_state": [P, P, P, P, P, I64],
            "lbm_get_state": [P, P, P, P],
            "lbm_init_equilibrium": [P, P, P, P, C.c_float],
            "lbm_init_equilibrium_f64": [P, P, P, P, D],
            "lbm_inflow_reichardt": [P, D, P],
            "stg_inlet_fill": [P, P, D],
            "stg_inlet_fill_noalloc": [P, P, D],
            "lbm_step": [P, P, I32],
            "lbm_stream_only": [P],
            "lbm_export_f32": [P, P],
            "lbm_import_f32": [P, P],
            "lbm_set_reference": [P, P],
            "lbm_state_elems": [P, P],
            "lbm_stats": [P, I32, P, I32, P, P],
            "lbm_sync": [P],
            "lbm_kernel_timing": [P, I32, P, P, P],
            "lbm_collide_dispatches": [P, P, P],
            "lbm_copy_probe": [P, P, I64, P],
            "lbm_set_cs_smag": [P, D],
            "lbm_adjoint_step": [P, P, P, P, D, P, P, P, P, P, P, P, P, P],
            "lbm_step_record": [P, P, P, P, D, I32, P, P, P, P],
            "lbm_field_export": [P, P, P],
            "lbm_field_import": [P, P, P],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.lbm_status_str.argtypes = [C.c_int]
        L.lbm_status_str.restype = C.c_char_p
        L.lbm_lattice_tables.argtypes = [P, P, P, P]
        L.lbm_lattice_tables.restype = None
        _lib = L
    return _lib


def status_str(s):
    try:
        return lib().lbm_status_str(int(s)).decode()
    except Exception:  # library not loadable: still format the code
        return "status"


def check(status, where=""):
    if status != LBM_OK:
        raise LbmError(status, where)
