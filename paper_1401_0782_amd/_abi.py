"""ctypes declarations of the libnegf C ABI (include/negf.h)."""

from __future__ import annotations

import ctypes as C
import pathlib

LIB_PATH = pathlib.Path(__file__).resolve().parent / "libnegf.so"

NEGF_OK = 0
NEGF_E_INVALID_ARG = 1
NEGF_E_OUT_OF_MEMORY = 2
NEGF_E_DEVICE = 3
NEGF_E_NOT_CONVERGED = 4
NEGF_E_BREAKDOWN = 5
STATUS_NAMES = {0: "OK", 1: "INVALID_ARG", 2: "OUT_OF_MEMORY", 3: "DEVICE",
                4: "NOT_CONVERGED", 5: "BREAKDOWN"}

NEGF_ITEM_CONVERGED, NEGF_ITEM_MAX_ITER, NEGF_ITEM_BREAKDOWN, NEGF_ITEM_INACCURATE = 0, 1, 2, 3
NEGF_FP64, NEGF_MIXED = 0, 1
NEGF_CORE_AUTO, NEGF_CORE_PER_ENERGY, NEGF_CORE_MULTISHIFT = 0, 1, 2
NEGF_DIR_RL, NEGF_DIR_LR = 0, 1
NEGF_SOLVER_COCG, NEGF_SOLVER_QMR = 0, 1
NEGF_RECOVER_OFF, NEGF_RECOVER_RESTART = 0, 1

# every function the header declares
EXPORTS = (
    "negf_build_operator",
    "negf_apply_operator",
    "negf_apply_operator_noalloc",
    "negf_solve_columns",
    "negf_transmission",
    "negf_transmission_batch",
    "negf_transmission_batch_shards",
    "negf_tune",
    "negf_tune_cached",
    "negf_set_launch_shape",
    "negf_current",
    "negf_spectral_transmission",
    "negf_eigenpairs",
    "negf_transmission_grad",
    "negf_destroy",
    "negf_last_error",
    "negf_version",
)


class negf_grid(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("h", C.c_double)]


class negf_kb(C.Structure):
    _fields_ = [("n_proj", C.c_int32), ("offsets", C.POINTER(C.c_int64)),
                ("idx", C.POINTER(C.c_int32)), ("val", C.POINTER(C.c_double)),
                ("e_kb", C.POINTER(C.c_double))]


class negf_opts(C.Structure):
    _fields_ = [("precision", C.c_int32), ("core", C.c_int32), ("solver", C.c_int32),
                ("direction", C.c_int32),
                ("tol", C.c_double), ("max_iter", C.c_int32), ("block_width", C.c_int32),
                ("shift_group", C.c_int32), ("max_refine", C.c_int32), ("col_begin", C.c_int32),
                ("col_count", C.c_int32), ("stream", C.c_void_p),
                ("recover", C.c_int32)]


class negf_diag(C.Structure):
    _fields_ = [("iters", C.POINTER(C.c_int32)), ("resid", C.POINTER(C.c_double)),
                ("t_col", C.POINTER(C.c_double)), ("item_status", C.POINTER(C.c_int32)),
                ("total_iters", C.c_int64), ("n_not_converged", C.c_int32),
                ("seconds", C.c_double), ("time_matvec", C.c_int32),
                ("matvec_seconds", C.c_double), ("matvec_launches", C.c_int64),
                ("matvec_bytes", C.c_double), ("optical_err", C.POINTER(C.c_double)),
                ("refine_steps", C.POINTER(C.c_int32))]


NEGF_TUNE_MAX = 64


class negf_tune_result(C.Structure):
    _fields_ = [("block_width", C.c_int32), ("wg_target", C.c_int32),
                ("plane_kernel", C.c_int32), ("n_tried", C.c_int32),
                ("tried_block_width", C.c_int32 * NEGF_TUNE_MAX),
                ("tried_wg_target", C.c_int32 * NEGF_TUNE_MAX),
                ("tried_plane_kernel", C.c_int32 * NEGF_TUNE_MAX),
                ("us_per_column_iteration", C.c_double * NEGF_TUNE_MAX)]


_lib = None


def load(path: str | None = None):
    """Load libnegf.so; raises if it has not been built (no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    p = pathlib.Path(path) if path else LIB_PATH
    if not p.exists():
        raise RuntimeError(
            f"libnegf is not built ({p} missing); run __graft_entry__.build() "
            "or python paper_1401_0782_amd/build.py")
    # torch's ROCm wheel carries its own HIP and HSA runtimes.  In a process
    # that also uses torch they must be loaded before this library: loaded
    # after it, one of the two sides finds no GPU.
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = C.CDLL(str(p))
    vp = C.c_void_p
    lib.negf_build_operator.argtypes = [C.POINTER(negf_grid), C.c_int32, vp, C.POINTER(negf_kb),
                                        vp, vp, C.POINTER(vp)]
    lib.negf_apply_operator.argtypes = [vp, C.c_int32, C.c_int32, vp, vp, vp]
    lib.negf_apply_operator_noalloc.argtypes = [vp, C.c_int32, vp, vp, vp, vp]
    lib.negf_solve_columns.argtypes = [vp, C.POINTER(negf_opts), C.c_int32, vp, C.c_int32, vp, vp,
                                       C.c_int32, vp, vp, vp]
    lib.negf_transmission.argtypes = [vp, C.POINTER(negf_opts), C.c_int32, vp, vp,
                                      C.POINTER(negf_diag)]
    lib.negf_transmission_grad.argtypes = [vp, C.POINTER(negf_opts), C.c_int32, vp, vp, vp, vp]
    lib.negf_transmission_batch.argtypes = [C.c_int32, C.POINTER(vp), C.POINTER(negf_opts),
                                            vp, C.POINTER(vp), C.POINTER(vp), vp, C.c_int32]
    lib.negf_transmission_batch_shards.argtypes = [C.c_int32, C.POINTER(vp), C.POINTER(negf_opts),
                                                   vp, C.POINTER(vp), vp, vp, C.POINTER(vp), vp,
                                                   C.c_int32]
    lib.negf_tune.argtypes = [vp, C.POINTER(negf_opts), C.c_int32, vp, C.c_int32,
                              C.POINTER(negf_tune_result)]
    lib.negf_tune_cached.argtypes = [vp, C.POINTER(negf_opts), C.c_int32, vp, C.c_int32,
                                     C.c_char_p, C.POINTER(negf_tune_result)]
    lib.negf_set_launch_shape.argtypes = [vp, C.c_int32, C.c_int32, C.c_int32]
    lib.negf_spectral_transmission.argtypes = [vp, C.c_int32, vp, vp, C.c_double, C.c_int32, vp,
                                               vp]
    lib.negf_current.argtypes = [C.c_int32, vp, vp, C.c_int32, vp, C.c_double, C.c_double, vp, vp]
    lib.negf_eigenpairs.argtypes = [vp, C.c_double, C.c_double, C.c_double, C.c_int32, C.c_double,
                                    C.c_int32, vp, vp, vp, vp]
    lib.negf_destroy.argtypes = [vp]
    lib.negf_destroy.restype = None
    lib.negf_last_error.restype = C.c_char_p
    lib.negf_version.restype = C.c_char_p
    for name in ("negf_build_operator", "negf_apply_operator", "negf_apply_operator_noalloc",
                 "negf_solve_columns",
                 "negf_transmission", "negf_transmission_grad", "negf_transmission_batch",
                 "negf_transmission_batch_shards", "negf_tune", "negf_tune_cached",
                 "negf_set_launch_shape", "negf_current",
                 "negf_spectral_transmission", "negf_eigenpairs"):
        getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib
