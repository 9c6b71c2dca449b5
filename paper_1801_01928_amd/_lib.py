"""ctypes loader for libttgfx.so and the C structures of include/ttgfx.h.

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  Loading fails loudly when the library has not been built.
"""
import ctypes as C
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libttgfx.so")
# The host-AddressSanitizer build of the same sources (build.py --asan), for
# the validation and bookkeeping tests of the C ABI on the CPU.
ASAN_LIB_PATH = os.path.join(_HERE, "libttgfx_asan.so")

TT_OK = 0
TT_ERR_ARG = -1
TT_ERR_SHAPE = -2
TT_ERR_UNSUPPORTED = -3
TT_ERR_WORKSPACE = -4
TT_ERR_HIP = -5
TT_ERR_INDEX = -6
TT_LR = 0
TT_RL = 1
TT_LOSS = {"squared": 0, "huber": 1, "logistic": 2}
TT_MAX_D = 32
TT_MAX_RANK = 64

ERROR_NAMES = {
    TT_ERR_ARG: "TT_ERR_ARG", TT_ERR_SHAPE: "TT_ERR_SHAPE",
    TT_ERR_UNSUPPORTED: "TT_ERR_UNSUPPORTED", TT_ERR_WORKSPACE: "TT_ERR_WORKSPACE",
    TT_ERR_HIP: "TT_ERR_HIP", TT_ERR_INDEX: "TT_ERR_INDEX",
}


class TTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERROR_NAMES.get(code, "?"), code, msg))
        self.code = code


class tt_tensor(C.Structure):
    _fields_ = [("d", C.c_int32), ("n", C.POINTER(C.c_int32)), ("r", C.POINTER(C.c_int32)),
                ("off", C.POINTER(C.c_int64)), ("data", C.c_void_p)]


class tt_batch(C.Structure):
    _fields_ = [("b", C.c_int32), ("tt", C.POINTER(tt_tensor))]


class tt_tensor_f64(C.Structure):
    _fields_ = [("d", C.c_int32), ("n", C.POINTER(C.c_int32)), ("r", C.POINTER(C.c_int32)),
                ("off", C.POINTER(C.c_int64)), ("data", C.c_void_p)]


class tt_batch_f64(C.Structure):
    _fields_ = [("b", C.c_int32), ("tt", C.POINTER(tt_tensor_f64))]


class tt_matrix(C.Structure):
    _fields_ = [("d", C.c_int32), ("m", C.POINTER(C.c_int32)), ("n", C.POINTER(C.c_int32)),
                ("r", C.POINTER(C.c_int32)), ("off", C.POINTER(C.c_int64)), ("data", C.c_void_p)]


P_TT = C.POINTER(tt_tensor)
P_BATCH = C.POINTER(tt_batch)
P_TTM = C.POINTER(tt_matrix)
P_BATCH64 = C.POINTER(tt_batch_f64)
VP = C.c_void_p
I64 = C.c_int64
I32 = C.c_int32
SZ = C.c_size_t
PI32 = C.POINTER(C.c_int32)
PI64 = C.POINTER(C.c_int64)

# name -> (restype, argtypes); the full exported surface of include/ttgfx.h
SIGNATURES = {
    "tt_gather_workspace": (I64, [P_TT, I64]),
    "tt_gather": (C.c_int, [P_TT, VP, I64, VP, VP, SZ, VP]),
    "tt_gather_backward_workspace": (I64, [P_TT, I64]),
    "tt_gather_backward": (C.c_int, [P_TT, VP, I64, VP, P_TT, VP, SZ, VP]),
    "tt_gather_mse_workspace": (I64, [P_TT, I64]),
    "tt_gather_mse_backward": (C.c_int, [P_TT, VP, I64, VP, VP, VP, VP, P_TT, VP, SZ, VP]),
    "tt_gather_mse_noalloc_limit": (I64, []),
    "tt_gather_mse_backward_noalloc": (C.c_int, [P_TT, VP, I64, VP, VP, VP, VP, P_TT, VP]),
    "tt_check_indices": (C.c_int, [P_TT, VP, I64, VP, VP]),
    "tt_set_suffix_depth": (C.c_int, [I32]),
    "tt_set_deterministic": (C.c_int, [I32]),
    "tt_deterministic": (I32, []),
    "tt_suffix_depth": (I32, [P_TT, I64]),
    "tt_halves_split": (C.c_int32, [P_TT]),
    "tt_halves_bytes": (I64, [P_TT, C.c_int32]),
    "tt_halves_build": (C.c_int, [P_TT, C.c_int32, VP, SZ, VP]),
    "tt_halves_gather": (C.c_int, [P_TT, C.c_int32, VP, SZ, VP, I64, VP, VP]),
    "tt_line_search_workspace": (I64, [P_TT, I64]),
    "tt_line_search": (C.c_int, [P_TT, VP, I64, VP, VP, VP, VP, SZ, VP]),
    "tt_orthogonalize_ranks": (C.c_int, [P_TT, C.c_int, PI32]),
    "tt_orthogonalize_workspace": (I64, [P_TT, C.c_int]),
    "tt_orthogonalize_both_workspace": (I64, [P_TT]),
    "tt_orthogonalize_both": (C.c_int, [P_TT, P_TT, P_TT, VP, SZ, VP]),
    "tt_orthogonalize": (C.c_int, [P_TT, C.c_int, P_TT, VP, SZ, VP]),
    "tt_project_sparse_workspace": (I64, [P_TT, I64]),
    "tt_project_sparse": (C.c_int, [P_TT, P_TT, VP, I64, VP, C.c_float, C.c_int, P_TT, VP, SZ, VP]),
    "tt_project_sum_workspace": (I64, [P_TT, P_BATCH]),
    "tt_project_sum": (C.c_int, [P_TT, P_TT, P_BATCH, VP, C.c_float, C.c_int, P_TT, VP, SZ, VP]),
    "tt_tangent_inner": (C.c_int, [P_TT, P_TT, P_TT, VP, VP]),
    "tt_tangent_gram_workspace": (I64, [P_TT, P_BATCH]),
    "tt_tangent_gram": (C.c_int, [P_TT, P_BATCH, VP, VP, SZ, VP]),
    "tt_tangent_axpby": (C.c_int, [P_TT, C.c_float, P_TT, C.c_float, P_TT, P_TT, VP]),
    "tt_tangent_combine": (C.c_int, [P_TT, P_TT, C.c_float, C.c_int, P_TT, VP]),
    "tt_tangent_combine_dev": (C.c_int, [P_TT, P_TT, VP, C.c_float, C.c_int, P_TT, VP]),
    "tt_cg_direction": (C.c_int, [P_TT, P_TT, P_TT, P_TT, VP, P_TT, VP, VP]),
    "tt_observed_loss_workspace": (I64, [I64]),
    "tt_observed_loss": (C.c_int, [VP, VP, I64, C.c_int, C.c_float, VP, VP, VP, SZ, VP]),
    "tt_riemannian_grad_workspace": (I64, [P_TT]),
    "tt_riemannian_grad": (C.c_int, [P_TT, P_TT, P_TT, C.c_float, C.c_int, P_TT, VP, SZ, VP]),
    "tt_project_tt_workspace": (I64, [P_TT, P_TT]),
    "tt_project_tt": (C.c_int, [P_TT, P_TT, P_TT, C.c_float, C.c_int, P_TT, VP, SZ, VP]),
    "tt_round_ranks": (C.c_int, [P_TT, I32, PI32]),
    "tt_round_workspace": (I64, [P_TT, I32]),
    "tt_round": (C.c_int, [P_TT, I32, P_TT, VP, VP, SZ, VP]),
    "tt_round_status": (C.c_int, [P_TT, I32, P_TT, VP, VP, VP, SZ, VP]),
    "tt_gram_workspace": (I64, [P_BATCH, P_BATCH]),
    "tt_gram": (C.c_int, [P_BATCH, P_BATCH, VP, VP, SZ, VP]),
    "tt_plan_create": (C.c_int, [P_BATCH, VP, VP, PI64, P_BATCH, VP, C.POINTER(VP)]),
    "tt_plan_run": (C.c_int, [VP, VP]),
    "tt_plan_capture": (C.c_int, [VP, VP]),
    "tt_plan_run_plain": (C.c_int, [VP, VP]),
    "tt_plan_autotune": (C.c_int, [VP, VP, PI32]),
    "tt_plan_config": (C.c_int, [VP, PI32]),
    "tt_plan_set_config": (C.c_int, [VP, PI32]),
    "tt_plan_destroy": (None, [VP]),
    "tt_matmul_workspace": (I64, [P_TTM, I64, C.c_int]),
    "tt_matmul_set_path": (C.c_int, [I32]),
    "tt_matmul_path": (I32, [P_TTM, I64, C.c_int]),
    "tt_matmul": (C.c_int, [P_TTM, VP, I64, VP, C.c_int, VP, SZ, VP]),
    "tt_matvec": (C.c_int, [P_TTM, P_BATCH, P_BATCH, VP]),
    "tt_matmat": (C.c_int, [P_TTM, P_TTM, P_TTM, VP]),
    "tt_norms": (C.c_int, [P_BATCH, VP, VP]),
    "tt_matvec_f64": (C.c_int, [P_TTM, P_BATCH64, P_BATCH64, VP]),
    "tt_matmat_f64": (C.c_int, [P_TTM, P_TTM, P_TTM, VP]),
    "tt_norms_f64": (C.c_int, [P_BATCH64, VP, VP]),
    "tt_gram_f64_workspace": (I64, [P_BATCH64, P_BATCH64]),
    "tt_gram_f64": (C.c_int, [P_BATCH64, P_BATCH64, VP, VP, SZ, VP]),
    "tt_matmul_backward": (C.c_int, [P_TTM, VP, I64, VP, VP, VP, C.c_int, VP, SZ, VP]),
    "tt_peak_work": (C.c_double, [C.c_int, I32, I32]),
    "tt_peak_launch": (C.c_int, [C.c_int, I32, I32, VP, VP]),
    "tt_timer_start": (C.c_int, []),
    "tt_timer_stop": (C.c_int, [C.POINTER(C.c_float), PI32]),
    "tt_last_error": (C.c_char_p, []),
    "tt_version": (C.c_int, []),
}

_lib = None


def load(path=None):
    """Load libttgfx.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    path = path or os.environ.get("TTGFX_LIB") or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError("libttgfx.so not found at %s: build it first "
                           "(python paper_1801_01928_amd/build.py)" % path)
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def last_error():
    return load().tt_last_error().decode(errors="replace")


def check(rc):
    if rc < 0:
        raise TTError(rc, last_error())
    return rc
