"""ctypes binding of include/cpcrit.h (libcpcrit.so, built in-tree).

Functions keep the C names and take C-level arguments (descriptor structs,
integer device addresses, stream handles).  Loading fails loudly when the
library has not been built: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcpcrit.so")

CP_OK, CP_EINVAL, CP_EDOMAIN, CP_ENOMEM, CP_EDEVICE, CP_EUNSUPPORTED = range(6)
CP_UNIFORM, CP_EPANECHNIKOV, CP_HISTOGRAM, CP_MVGAUSS, CP_GAUSSIAN = range(5)
CP_F32, CP_F64 = 0, 1
CP_MC_CONDITIONAL, CP_MC_HIT = 0, 1
CP_BATCH_FWD, CP_BATCH_BWD, CP_BATCH_GRAPH, CP_BATCH_PER_FIELD, CP_BATCH_TUNE = 1, 2, 4, 8, 16

EXPORTS = ["cpu_fit_params", "cp_fit_forward", "cp_fit_error_bound", "cp_prob_forward", "cp_prob_backward",
           "cp_prob_backward_noalloc", "cp_prob_classify",
           "cp_prob_semianalytical",
           "cp_prob_batched", "cp_batched_pin", "cp_batched_describe",
           "cp_n_params", "cp_status_string", "cp_last_error", "cp_release", "cp_philox4x32_10", "cp_gauss_legendre"]


class cp_field_desc_t(ctypes.Structure):
    _fields_ = [("height", ctypes.c_int32), ("width", ctypes.c_int32), ("row_stride", ctypes.c_int64),
                ("model", ctypes.c_int32), ("dtype", ctypes.c_int32), ("nbins", ctypes.c_int32),
                ("nsamples", ctypes.c_int32), ("seed", ctypes.c_uint64), ("field_id", ctypes.c_uint32),
                ("estimator", ctypes.c_int32)]


class cp_fit_opts_t(ctypes.Structure):
    _fields_ = [("ddof", ctypes.c_int32), ("bw_factor", ctypes.c_double), ("cov_jitter", ctypes.c_double),
                ("degenerate_eps", ctypes.c_double)]


class CPError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"cpcrit status {status}: {msg}")
        self.status = status


_lib = None


def load() -> ctypes.CDLL:
    """Load libcpcrit.so from the package directory (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                           "(or python paper_2407_18015_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    P, i32, i64, u32, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
    D = ctypes.POINTER(cp_field_desc_t)
    O = ctypes.POINTER(cp_fit_opts_t)
    PP = ctypes.POINTER(ctypes.c_void_p)
    sigs = {
        "cpu_fit_params": (i32, [D, P, i32, O, P, P]),
        "cp_fit_forward": (i32, [D, P, i32, O, P, P, P, P]),
        "cp_fit_error_bound": (i32, [D, P, ctypes.c_double, P, P]),
        "cp_prob_forward": (i32, [D, P, P, P, P]),
        "cp_prob_backward": (i32, [D, P, P, P, P, P]),
        "cp_prob_backward_noalloc": (i32, [D, P, P, P, P, P]),
        "cp_prob_classify": (i32, [D, P, P, P, P, P, P, P]),
        "cp_prob_semianalytical": (i32, [D, P, P, P, P, P]),
        "cp_prob_batched": (i32, [i32, D, PP, PP, PP, PP, PP, PP, u32, P]),
        "cp_batched_pin": (i32, [i32, D, u32, ctypes.POINTER(i32), ctypes.POINTER(i32)]),
        "cp_batched_describe": (ctypes.c_char_p, [i32, D, u32]),
        "cp_n_params": (i32, [i32, i32]),
        "cp_status_string": (ctypes.c_char_p, [i32]),
        "cp_last_error": (ctypes.c_char_p, []),
        "cp_release": (i32, []),
        "cp_philox4x32_10": (i32, [i64, P, u64, P, P]),
        "cp_gauss_legendre": (i32, [i32, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_double)]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != CP_OK:
        lib = load()
        raise CPError(status, f"{lib.cp_status_string(status).decode()}: {lib.cp_last_error().decode()}")


def cpu_fit_params(desc, members, n_members, opts, params, stream) -> int:
    return load().cpu_fit_params(ctypes.byref(desc), members, n_members, ctypes.byref(opts) if opts else None,
                                 params, stream)


def cp_fit_forward(desc, members, n_members, opts, params, p_min, p_max, stream) -> int:
    return load().cp_fit_forward(ctypes.byref(desc), members, n_members, ctypes.byref(opts) if opts else None,
                                 params, p_min, p_max, stream)


def cp_fit_error_bound(desc, decompressed, eb, params, stream) -> int:
    return load().cp_fit_error_bound(ctypes.byref(desc), decompressed, eb, params, stream)


def cp_prob_classify(desc, params, p_min, p_max, p_saddle, p_regular, terms, stream) -> int:
    return load().cp_prob_classify(ctypes.byref(desc), params, p_min, p_max, p_saddle, p_regular, terms, stream)


def cp_prob_semianalytical(desc, params, p_min, p_max, terms, stream) -> int:
    return load().cp_prob_semianalytical(ctypes.byref(desc), params, p_min, p_max, terms, stream)


def cp_prob_forward(desc, params, p_min, p_max, stream) -> int:
    return load().cp_prob_forward(ctypes.byref(desc), params, p_min, p_max, stream)


def cp_prob_backward(desc, params, g_min, g_max, grad_params, stream) -> int:
    return load().cp_prob_backward(ctypes.byref(desc), params, g_min, g_max, grad_params, stream)


def cp_prob_backward_noalloc(desc, params, g_min, g_max, grad_params, stream) -> int:
    return load().cp_prob_backward_noalloc(ctypes.byref(desc), params, g_min, g_max, grad_params, stream)


def _ptr_array(vals):
    if vals is None:
        return None
    return (ctypes.c_void_p * len(vals))(*[v if v else None for v in vals])


def cp_prob_batched(n, descs, params, p_min, p_max, g_min, g_max, grad_params, flags, stream) -> int:
    arr = (cp_field_desc_t * n)(*descs)
    cast = lambda a: ctypes.cast(a, ctypes.POINTER(ctypes.c_void_p)) if a is not None else None
    return load().cp_prob_batched(n, arr, cast(_ptr_array(params)), cast(_ptr_array(p_min)),
                                  cast(_ptr_array(p_max)), cast(_ptr_array(g_min)), cast(_ptr_array(g_max)),
                                  cast(_ptr_array(grad_params)), flags, stream)


def cp_batched_pin(n, descs, flags, shape, chunk) -> int:
    """shape, chunk: 5 entries each, indexed by pass (forward, histogram
    forward, adjoint, histogram adjoint sweep, histogram gather)."""
    arr = (cp_field_desc_t * n)(*descs)
    sh = (ctypes.c_int32 * 5)(*shape)
    ch = (ctypes.c_int32 * 5)(*chunk)
    return load().cp_batched_pin(n, arr, flags, sh, ch)


def cp_batched_describe(n, descs, flags):
    """Text of the plan a cp_prob_batched call with these descriptors and
    flags uses, or None before that plan exists."""
    arr = (cp_field_desc_t * n)(*descs)
    r = load().cp_batched_describe(n, arr, flags)
    return None if r is None else r.decode()


def cp_n_params(model: int, nbins: int) -> int:
    return load().cp_n_params(model, nbins)


def cp_release() -> int:
    return load().cp_release()


def cp_philox4x32_10(n, counters, seed, out, stream) -> int:
    return load().cp_philox4x32_10(n, counters, seed, out, stream)


def cp_gauss_legendre(n: int):
    x = (ctypes.c_double * max(n, 1))()
    w = (ctypes.c_double * max(n, 1))()
    check(load().cp_gauss_legendre(n, x, w))
    return list(x)[:n], list(w)[:n]
