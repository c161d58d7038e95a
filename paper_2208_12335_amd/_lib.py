"""ctypes declarations of the C ABI in include/aims_grid.h (argument marshalling only).

Importing this module loads ``libaimsgrid.so`` from the package directory and fails loudly if
it has not been built; there is no fallback implementation.
"""
import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_int32, c_int64, c_void_p

# AIMS_LIB selects another build of the same library (the host-sanitized one, for CPU checks)
LIB_PATH = os.environ.get("AIMS_LIB") or os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                                      "libaimsgrid.so")

AIMS_OK, AIMS_ERR_ARG, AIMS_ERR_OOM, AIMS_ERR_HIP, AIMS_ERR_STALE, AIMS_ERR_UNSUPPORTED = 0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "AIMS_OK", -1: "AIMS_ERR_ARG", -2: "AIMS_ERR_OOM", -3: "AIMS_ERR_HIP",
                -4: "AIMS_ERR_STALE", -5: "AIMS_ERR_UNSUPPORTED"}
PRECISION = {"fp64": 0, "fp32": 1, "bf16x3": 2, "int8x7": 3}
DM_METHOD = {"eigen": 0, "purify": 1}
XC_FUNCTIONAL = {"lda": 0, "pbe": 1}


class AimsSystem(ctypes.Structure):
    _fields_ = [
        ("n_atoms", c_int32),
        ("atom_xyz", POINTER(c_double)),
        ("atom_species", POINTER(c_int32)),
        ("n_species", c_int32),
        ("species_nshell", POINTER(c_int32)),
        ("shell_l", POINTER(c_int32)),
        ("n_log", c_int32),
        ("r0", c_double),
        ("rc", c_double),
        ("shell_R", POINTER(c_double)),
        ("shell_K", POINTER(c_double)),
        ("n_points", c_int64),
        ("pt_xyz", POINTER(c_double)),
        ("pt_w", POINTER(c_double)),
        ("max_batch", c_int32),
        ("screen_margin", c_double),
    ]


class AimsTuning(ctypes.Structure):
    _fields_ = [("h_merge", c_int32), ("density_pblocks", c_int32), ("persistent", c_int32),
                ("h_flops_per_atomic", c_int32), ("h_tile32_mask", c_int32),
                ("density_bucket_pblocks", c_int32 * 8)]


class AimsHartreeGrid(ctypes.Structure):
    _fields_ = [("pt_owner", POINTER(c_int32)), ("pt_node", POINTER(c_int32)),
                ("n_radial", c_int32), ("r_map", c_double), ("l_max", c_int32)]


class AimsMovingGrid(ctypes.Structure):
    _fields_ = [("pt_owner", POINTER(c_int32)), ("pt_wgrid", POINTER(c_double)),
                ("atom_Z", POINTER(c_double)), ("nuc_sigma", c_double), ("partition_a", c_double)]


# every symbol the header declares, with its signature
SIGNATURES = {
    "aims_grid_setup": (c_int, [POINTER(AimsSystem), c_int, c_void_p, POINTER(c_void_p)]),
    "aims_grid_setup_many": (c_int, [POINTER(AimsSystem), c_int32, c_int, c_void_p, POINTER(c_void_p)]),
    "aims_update_density": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "aims_update_density_noalloc": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p]),
    "aims_integrate_h": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p]),
    "aims_integrate_h_backward": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p,
                                          c_void_p, c_void_p, c_void_p]),
    "aims_grid_set_moving": (c_int, [c_void_p, c_int32, POINTER(AimsMovingGrid)]),
    "aims_total_forces": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p]),
    "aims_integrate_h_gga": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p]),
    "aims_density_gradient": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "aims_grid_set_hartree": (c_int, [c_void_p, c_int32, POINTER(AimsHartreeGrid)]),
    "aims_hartree": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p]),
    "aims_xc": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    "aims_xc_gga": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "aims_density_matrix": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, POINTER(c_double), c_double,
                                    c_void_p, c_void_p, POINTER(c_double)]),
    "aims_last_purify_products": (c_int32, [c_void_p]),
    "aims_step_graph_create": (c_int, [c_void_p, c_int, c_void_p, c_void_p, c_void_p, c_void_p,
                                       c_void_p, POINTER(c_void_p)]),
    "aims_step_graph_launch": (c_int, [c_void_p]),
    "aims_step_graph_destroy": (None, [c_void_p]),
    "aims_get_tuning": (c_int, [c_void_p, c_int, POINTER(AimsTuning)]),
    "aims_set_tuning": (c_int, [c_void_p, c_int, POINTER(AimsTuning)]),
    "aims_work_stats": (c_int, [c_void_p, POINTER(c_int64), POINTER(c_double), POINTER(c_double)]),
    "aims_positions_status": (c_int, [c_void_p]),
    "aims_bucket_stats": (c_int, [c_void_p, c_int, c_int32, POINTER(c_int64), POINTER(c_double)]),
    "aims_n_basis": (c_int64, [c_void_p]),
    "aims_n_points": (c_int64, [c_void_p]),
    "aims_n_atoms": (c_int32, [c_void_p]),
    "aims_profile_enable": (c_int, [c_void_p, c_int]),
    "aims_profile_read": (c_int, [c_void_p, c_char_p, POINTER(c_int64), POINTER(c_double),
                                  POINTER(c_double)]),
    "aims_last_error": (c_char_p, [c_void_p]),
    "aims_grid_destroy": (None, [c_void_p]),
}

_lib = None


def load():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2208_12335_amd.build.build() "
                              "(there is no non-HIP implementation)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class AimsError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status
