"""ctypes binding of ``librsvd_mi355x.so`` (argument marshalling only).

The shared library is built in-tree by ``paper_1608_02148_amd.build``.  There
is no fallback: if the library is missing or fails to load, ``load()`` raises.
"""
import ctypes
import os

from .build import LIB_PATH

c_int32, c_int64, c_uint32, c_uint64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
c_void_p, c_size_t, c_double = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_double

RSVD_F64, RSVD_F32, RSVD_BF16 = 0, 1, 2
SDIST = {"normal": 0, "unif": 1, "rademacher": 2}
PRECISION = {"plain": 0, "bf16_mixed": 1}
SCHEME = {"qr": 0, "lu": 1}
ARITH = {"storage": 0, "bf16": 1, "split": 2}

STATUS = {
    0: "ok", -1: "invalid argument", -2: "unsupported dtype, mode or size",
    -3: "HIP runtime error", -4: "non-finite values reached a Gram matrix",
    -5: "numerical breakdown after the shifted Cholesky",
}
FLAG_CHOL_SHIFT, FLAG_DEGENERATE, FLAG_NONFINITE, FLAG_JACOBI_SLOW, FLAG_ZERO_SCALE = 1, 2, 4, 8, 16
MAX_L = 128              # batches and kernel-level entry points
MAX_L_SINGLE = 256       # rsvd_run / rpca_run


class Params(ctypes.Structure):
    _fields_ = [("p", c_int32), ("q", c_int32), ("seed", c_uint64), ("stream_id", c_uint32),
                ("sdist", c_int32), ("precision", c_int32), ("probes", c_int32), ("scheme", c_int32),
                ("reserved", c_int32)]


class Info(ctypes.Structure):
    _fields_ = [("l", c_int32), ("q", c_int32), ("p", c_int32), ("flags", c_uint32),
                ("est_err", c_double)]


class KernelStat(ctypes.Structure):
    _fields_ = [("count", c_int32), ("reserved", c_int32), ("total_ms", c_double),
                ("flops", c_double), ("bytes", c_double)]


class RpcaOptions(ctypes.Structure):
    _fields_ = [("center", c_int32), ("scale", c_int32), ("reserved", c_int32 * 2)]


class RpcaOutputs(ctypes.Structure):
    _fields_ = [("rotation", c_void_p), ("ldr", c_int64), ("eigvals", c_void_p), ("sdev", c_void_p),
                ("x", c_void_p), ("ldx", c_int64), ("x_white", c_void_p), ("ldxw", c_int64),
                ("loadings", c_void_p), ("ldl", c_int64), ("center", c_void_p), ("scale", c_void_p),
                ("total_var", c_void_p)]


class RrpcaOptions(ctypes.Structure):
    _fields_ = [("lam", c_double), ("tol", c_double), ("rho", c_double), ("mu0_scale", c_double),
                ("maxiter", c_int32), ("k_max", c_int32)]


class RrpcaResult(ctypes.Structure):
    _fields_ = [("iterations", c_int32), ("rank", c_int32), ("k", c_int32), ("reserved", c_int32),
                ("residual", c_double), ("lam", c_double)]


class MlpHeader(ctypes.Structure):
    _fields_ = [("version", c_uint32), ("params", c_uint32), ("step", c_uint32), ("reserved", c_uint32),
                ("seed", c_uint64), ("n_train", c_uint64), ("digest", ctypes.c_uint8 * 8),
                ("tau", ctypes.c_float), ("reserved2", c_uint32)]


class BatchDesc(ctypes.Structure):
    _fields_ = [("A", c_void_p), ("lda", c_int64), ("m", c_int64), ("n", c_int64), ("k", c_int32),
                ("stream_id", c_uint32), ("U", c_void_p), ("ldu", c_int64), ("S", c_void_p),
                ("V", c_void_p), ("ldv", c_int64), ("info", c_void_p), ("features", c_void_p),
                ("q", c_int32), ("p", c_int32)]


BATCH_GRAPH, BATCH_STAMPS, BATCH_FEATURES, BATCH_OWN_QP, BATCH_CHUNKED = 1, 2, 4, 8, 16
MLP_INPUTS, MLP_HIDDEN, MLP_CLASSES, MLP_PARAMS = 131, 64, 15, 13583
LEARNED_QMAX, LEARNED_PMAX, LEARNED_FALLBACK_Q = 4, 20, 3

PROFILE_KINDS = 2
PROFILE_NAMES = ("A_X", "AT_Q")


class RsvdError(RuntimeError):
    def __init__(self, status, where=""):
        self.status = status
        super().__init__(f"{where}: {STATUS.get(status, 'unknown status')} ({status})")


_PROTOS = {
    "rsvd_default_params": (None, [c_void_p]),
    "rsvd_create": (c_int32, [c_void_p, c_void_p]),
    "rsvd_destroy": (c_int32, [c_void_p]),
    "rsvd_set_stream": (c_int32, [c_void_p, c_void_p]),
    "rsvd_last_hip_error": (c_int32, [c_void_p]),
    "rsvd_set_tile_variants": (c_int32, [c_void_p, c_void_p]),
    "rsvd_get_tile_variants": (c_int32, [c_void_p, c_void_p]),
    "rsvd_status_string": (ctypes.c_char_p, [c_int32]),
    "rsvd_workspace_size": (c_int32, [c_void_p, c_int32, c_int64, c_int64, c_int32, c_void_p, c_void_p]),
    "rsvd_run": (c_int32, [c_void_p, c_int32, c_int64, c_int64, c_void_p, c_int64, c_int32, c_void_p,
                           c_void_p, c_int64, c_void_p, c_void_p, c_int64, c_void_p, c_size_t, c_void_p]),
    "rpca_run": (c_int32, [c_void_p, c_int32, c_int64, c_int64, c_void_p, c_int64, c_int32, c_int32,
                           c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p, c_int64, c_void_p,
                           c_void_p, c_size_t, c_void_p]),
    "rpca_run_ex": (c_int32, [c_void_p, c_int32, c_int64, c_int64, c_void_p, c_int64, c_int32, c_void_p,
                              c_void_p, c_void_p, c_void_p, c_size_t, c_void_p]),
    "rpca_predict_workspace_size": (c_int32, [c_void_p, c_int32, c_int64, c_int64, c_int32, c_void_p]),
    "rpca_predict": (c_int32, [c_void_p, c_int32, c_int64, c_int64, c_void_p, c_int64, c_int32, c_void_p,
                               c_int64, c_void_p, c_void_p, c_void_p, c_int64, c_void_p, c_size_t]),
    "rrpca_default_options": (None, [c_void_p]),
    "rrpca_workspace_size": (c_int32, [c_void_p, c_int32, c_int64, c_int64, c_void_p, c_void_p, c_void_p]),
    "rrpca_run": (c_int32, [c_void_p, c_int32, c_int64, c_int64, c_void_p, c_int64, c_void_p, c_void_p,
                            c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_size_t, c_void_p]),
    "rid_workspace_size": (c_int32, [c_void_p, c_int32, c_int64, c_int64, c_int32, c_void_p, c_int32, c_void_p]),
    "rid_run": (c_int32, [c_void_p, c_int32, c_int64, c_int64, c_void_p, c_int64, c_int32, c_void_p, c_void_p,
                          c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_size_t]),
    "rcur_run": (c_int32, [c_void_p, c_int32, c_int64, c_int64, c_void_p, c_int64, c_int32, c_void_p, c_void_p,
                           c_void_p, c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_size_t]),
    "rsvd_sync_info": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "rsvd_run_noalloc": (c_int32, [c_void_p, c_int32, c_int64, c_int64, c_void_p, c_int64, c_int32, c_void_p,
                                   c_void_p, c_int64, c_void_p, c_void_p, c_int64, c_void_p]),
    "rsvd_batch_create": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_int32, c_void_p,
                                    c_void_p]),
    "rsvd_batch_bind": (c_int32, [c_void_p, c_void_p, c_size_t]),
    "rsvd_batch_run": (c_int32, [c_void_p]),
    "rsvd_batch_stamps": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "rsvd_batch_destroy": (c_int32, [c_void_p]),
    "rsvd_batch_create_learned": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p,
                                            ctypes.c_float, c_int32, c_void_p, c_void_p]),
    "rsvd_batch_choices": (c_int32, [c_void_p, c_void_p]),
    "rsvd_select_workspace_size": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p]),
    "rsvd_select": (c_int32, [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p, ctypes.c_float, c_void_p,
                              c_void_p, c_void_p, c_void_p, c_size_t]),
    "rsvd_mlp_workspace_size": (c_int32, [c_int32, c_void_p]),
    "rsvd_mlp_init": (c_int32, [c_void_p, c_void_p, c_uint64]),
    "rsvd_mlp_forward": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_void_p, c_void_p]),
    "rsvd_mlp_train_step": (c_int32, [c_void_p, c_void_p, c_void_p, c_void_p, c_int32, ctypes.c_float, c_int32,
                                      c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_size_t]),
    "rsvd_mlp_load": (c_int32, [c_void_p, ctypes.c_char_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "rsvd_profile_enable": (c_int32, [c_void_p, c_int32]),
    "rsvd_profile_collect": (c_int32, [c_void_p, c_void_p]),
    "rsvd_philox_words": (c_int32, [c_void_p, c_int64, c_int32, c_uint64, c_uint32, c_void_p]),
    "rsvd_test_matrix": (c_int32, [c_void_p, c_int32, c_int64, c_int32, c_uint64, c_uint32, c_int32,
                                   c_void_p, c_int64]),
    "rsvd_gemm_nn": (c_int32, [c_void_p, c_int32, c_int32, c_int64, c_int64, c_int32, c_void_p, c_int64,
                               c_void_p, c_int64, c_void_p, c_int64, c_int32, c_void_p, c_size_t]),
    "rsvd_gemm_tn": (c_int32, [c_void_p, c_int32, c_int32, c_int64, c_int64, c_int32, c_void_p, c_int64,
                               c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_size_t]),
    "rsvd_orthonormalize": (c_int32, [c_void_p, c_int32, c_int64, c_int32, c_void_p, c_int64, c_void_p,
                                      c_void_p, c_void_p, c_size_t]),
    "rsvd_block_workspace_size": (c_int32, [c_void_p, c_int32, c_int64, c_int64, c_int32, c_void_p]),
    "rsvd_lu_normalize": (c_int32, [c_void_p, c_int32, c_int64, c_int32, c_void_p, c_int64, c_void_p, c_void_p,
                                    c_void_p, c_void_p, c_size_t]),
    "rsvd_small_svd": (c_int32, [c_void_p, c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                 c_void_p, c_size_t]),
}

EXPORTED = tuple(_PROTOS)

_LIB = None


def load(path=None):
    """Load the library once and attach argument types.  Raises if missing."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = path or LIB_PATH
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is not built; run `python -m paper_1608_02148_amd.build`")
    lib = ctypes.CDLL(path)
    for name, (res, args) in _PROTOS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def check(status, where):
    if status != 0:
        raise RsvdError(status, where)
