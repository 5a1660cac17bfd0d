"""ctypes view of libmps.so (include/mps.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmps.so")

MPS_OK = 0
ERRORS = {-1: "MPS_E_ARG", -2: "MPS_E_NONFINITE", -3: "MPS_E_ZEROWEIGHT",
          -4: "MPS_E_NOMEM", -5: "MPS_E_HIP", -6: "MPS_E_TIMEOUT",
          -7: "MPS_E_BUSY", -8: "MPS_E_TOOBIG"}
MPS_F32, MPS_F64 = 1, 2
BULKFLOW_SUBTRACT, NO_SHOTNOISE, NO_DECONVOLVE, KERNEL_BL3_EXACT = 1, 2, 4, 8
KERNEL_ORDER_SHIFT = 4
CATALOG_HOST = 1 << 7
KERNEL_BL3_QUADRATIC = 7 << KERNEL_ORDER_SHIFT
KERNELS = {"bl3": 0, "bl3_exact": KERNEL_BL3_EXACT, "bl3q": KERNEL_BL3_QUADRATIC}
# centred B-splines of order p (MPS_KERNEL_BSPLINE(p))
for _name, _p in (("ngp", 1), ("cic", 2), ("tsc", 3), ("pcs", 4), ("pqs", 5), ("bspline6", 6)):
    KERNELS[_name] = _p << KERNEL_ORDER_SHIFT
for _p in range(1, 7):
    KERNELS[f"bspline{_p}"] = _p << KERNEL_ORDER_SHIFT
MAX_BINS = 128
STATIC_MAX_GRID = 64              # MPS_STATIC_MAX_GRID
STATIC_MAX_PARTICLES = 1 << 20    # MPS_STATIC_MAX_PARTICLES
SCATTER_MIN_GRID = 128            # MPS_SCATTER_MIN_GRID
SCATTER_GATHER_MAX_MEAN = 384     # MPS_SCATTER_GATHER_MAX_MEAN
SCATTER_HALO_MAX_MEAN = 2048      # MPS_SCATTER_HALO_MAX_MEAN
SCATTER_GATHER64_MAX_MEAN = 384   # MPS_SCATTER_GATHER64_MAX_MEAN
NUM_STAGES = 9
STAGES = ("moments+count", "scan", "permute", "clear", "scatter",
          "fft_z", "fft_y", "fft_x+bin", "finalize")


class Catalog(C.Structure):
    _fields_ = [("n_particles", C.c_int64), ("pos", C.c_void_p), ("vel", C.c_void_p),
                ("weight", C.c_void_p), ("box", C.c_double), ("haf", C.c_double),
                ("n_bins", C.c_int), ("k_edges", C.POINTER(C.c_double)),
                ("flags", C.c_uint32)]


class Result(C.Structure):
    _fields_ = [("k_mean", C.POINTER(C.c_double)), ("p_pp", C.POINTER(C.c_double)),
                ("p_tt", C.POINTER(C.c_double)), ("p_dt", C.POINTER(C.c_double)),
                ("p_dd", C.POINTER(C.c_double)), ("sn_pp", C.POINTER(C.c_double)),
                ("sn_tt", C.POINTER(C.c_double)), ("sn_dd", C.POINTER(C.c_double)),
                ("n_modes", C.POINTER(C.c_int64)), ("v_bulk", C.c_double * 3),
                ("sigma_v2", C.c_double), ("n_eff", C.c_double)]


MU_KEYS = ("k_mean", "mu_mean", "p_pp", "p_tt", "p_dd", "p_dt_re", "p_dt_im", "p_dpb_re",
           "p_dpb_im", "sn_pp", "sn_tt", "sn_dd", "sn_dt_im", "sn_dpb")
MAX_MU_BINS = 64
MAX_MU_CELLS = 512
MAX_DIV = 8


class ResultMu(C.Structure):
    _fields_ = ([(k, C.POINTER(C.c_double)) for k in MU_KEYS]
                + [("n_modes", C.POINTER(C.c_int64)), ("axis", C.c_double * 3),
                   ("v_bulk", C.c_double * 3), ("sigma_v2", C.c_double), ("n_eff", C.c_double)])


SPT_KEYS = ("p13", "p22", "p13_dt", "p22_dt", "p13_tt", "p22_tt", "i1", "i2", "i3", "pcov1", "pcov2",
            "p_lin", "p_dd", "p_theta_p", "p_dtheta_p", "p_mom")
SPT_MAX_K = 65536
SPT_MAX_TABLE = 2048


class SptResult(C.Structure):
    _fields_ = [(k, C.POINTER(C.c_double)) for k in SPT_KEYS]


class MpsError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        name = ERRORS.get(status, str(status))
        super().__init__(f"{what}: {name} ({_strerror(status)})" if what else name)


_lib = None


def lib():
    """Load libmps.so; raise if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2005_06170_amd.build`")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int, C.c_int64, C.c_double
    sig = {
        "mps_plan_create": (i32, [C.POINTER(vp), i32, i32]),
        "mps_plan_destroy": (i32, [vp]),
        "mps_plan_reserve": (i32, [vp, i64]),
        "mps_footprint": (C.c_size_t, [i32, i32, i64]),
        "mps_estimate": (i32, [vp, C.POINTER(Catalog), C.POINTER(Result), vp]),
        "mps_estimate_batch": (i32, [C.POINTER(vp), C.POINTER(Catalog), C.POINTER(Result), i32, vp]),
        "mps_estimate_mu": (i32, [vp, C.POINTER(Catalog), i32, C.POINTER(dbl), C.POINTER(ResultMu), vp]),
        "mps_estimate_subcubes": (i32, [vp, C.POINTER(Catalog), i32, C.POINTER(Result), C.POINTER(i32),
                                        C.POINTER(Result), C.POINTER(Result), vp]),
        "mps_spt_one_loop": (i32, [C.POINTER(dbl), i32, C.POINTER(dbl), C.POINTER(dbl), i32, dbl, dbl,
                                   C.POINTER(SptResult), vp]),
        "mps_assign": (i32, [vp, C.POINTER(Catalog), vp, vp]),
        "mps_fft": (i32, [vp, vp, vp]),
        "mps_plan_set_timing": (i32, [vp, i32]),
        "mps_plan_stage_times": (i32, [vp, C.POINTER(dbl), i32]),
        "mps_strerror": (C.c_char_p, [i32]),
        "mps_estimate_static": (i32, [C.POINTER(Catalog), i32, i32, C.POINTER(Result), vp]),
    }
    optional = {
        "mps_server_create": (i32, [C.POINTER(vp), C.c_size_t, i32, i64]),
        "mps_submit": (i32, [vp, C.POINTER(Catalog), i32, i32, C.POINTER(Result), vp, C.POINTER(C.c_uint64)]),
        "mps_wait": (i32, [vp, C.c_uint64, dbl]),
        "mps_server_destroy": (i32, [vp]),
    }
    for name, (res, args) in {**sig, **optional}.items():
        if not hasattr(L, name):
            if name in sig:
                raise ImportError(f"{LIB_PATH} does not export {name}")
            continue
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _strerror(status: int) -> str:
    try:
        return lib().mps_strerror(status).decode()
    except Exception:  # pragma: no cover - only while reporting another error
        return "?"


def check(status: int, what: str = "") -> None:
    if status != MPS_OK:
        raise MpsError(status, what)


def exported_symbols():
    """Names declared in include/mps.h that the loaded library exports."""
    L = lib()
    names = ["mps_plan_create", "mps_plan_destroy", "mps_plan_reserve", "mps_footprint",
             "mps_estimate", "mps_estimate_batch", "mps_estimate_mu", "mps_estimate_subcubes",
             "mps_spt_one_loop", "mps_assign", "mps_fft",
             "mps_plan_set_timing", "mps_plan_stage_times", "mps_server_create",
             "mps_submit", "mps_wait", "mps_server_destroy", "mps_strerror", "mps_estimate_static"]
    return {n: hasattr(L, n) for n in names}
