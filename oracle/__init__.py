"""Plain FP64 CPU reference (oracle) for critical-point probabilities.

TEST INFRASTRUCTURE ONLY: imported by the test-suite, by the smoke check of
``__graft_entry__`` and by the CPU-baseline leg of ``bench.py``.  The product
package never imports it, and it imports nothing from the product package.

The arithmetic lives in ``cp_oracle.c`` (C, FP64, OpenMP); this module builds
it with gcc and wraps it with ctypes over numpy arrays.  See the header of
``cp_oracle.c`` for what each function computes and which part of the paper
(Athawale et al., arXiv 2407.18015) it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cp_oracle.c")
_LIB = os.path.join(_HERE, "libcp_oracle.so")

UNIFORM, EPANECHNIKOV, HISTOGRAM, MVG, GAUSSIAN = 0, 1, 2, 3, 4
NSLOT = 5  # stencil slots: 0 = v, 1 = e (x+1), 2 = n (y-1), 3 = w (x-1), 4 = s (y+1)
SLOT_OFFSETS = ((0, 0), (0, 1), (-1, 0), (0, -1), (1, 0))  # (dy, dx)


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP contraction off, OpenMP)."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp"
    cmd = ["gcc", "-O2", "-std=gnu11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-Wall", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    i32, i64, u32, u64, f64 = ctypes.c_int, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_double
    sigs = {
        "or_n_param": (i32, [i32, i32]),
        "or_forward": (i32, [i32, i32, i32, i32, P, P, P]),
        "or_forward_at": (i32, [i32, i32, i32, i32, P, i64, P, P, P]),
        "or_jacobian_at": (i32, [i32, i32, i32, i32, P, i64, P, P, P]),
        "or_saddle_at": (i32, [i32, i32, i32, i32, P, i64, P, P, P]),
        "or_gauss_at": (i32, [i32, i32, P, i64, P, P]),
        "or_gauss_jacobian_at": (i32, [i32, i32, P, i64, P, P, P, i32]),
        "or_gauss_grad_at": (i32, [i32, i32, P, P, P, i64, P, P, i32]),
        "or_semi_at": (i32, [i32, i32, i32, P, i32, ctypes.c_uint64, ctypes.c_uint32, i64, P, P]),
        "or_semi_samples": (i32, [i32, i32, i32, P, i32, i32, i32, ctypes.c_uint64, ctypes.c_uint32, P]),
        "or_grad_at": (i32, [i32, i32, i32, i32, P, P, P, i64, P, P, i32]),
        "or_grad": (i32, [i32, i32, i32, i32, P, P, P, P, i32]),
        "or_fit": (i32, [i32, i32, P, i32, i32, i32, i32, i32, f64, f64, P]),
        "or_philox4x32_10": (None, [P, P, P]),
        "or_mvg_fit": (i32, [P, i32, i32, i32, i32, f64, P]),
        "or_mvg_forward_at": (i32, [P, i32, i32, i32, u64, u32, i64, P, P, P]),
        "or_mvg_grad_at": (i32, [P, i32, i32, i32, u64, u32, P, P, i64, P, P, P]),
    }
    for name, (res, args) in sigs.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def n_param(model: int, nbins: int = 0) -> int:
    return int(_load().or_n_param(model, nbins))


def _check(rc: int, what: str):
    if rc != 0:
        raise ValueError(f"oracle {what} rejected its arguments (code {rc})")


def _grid(params: np.ndarray, model: int):
    params = _f64(params)
    npar, H, W = params.shape
    nb = npar - 2 if model == HISTOGRAM else 0
    if npar != n_param(model, nb):
        raise ValueError("parameter plane count does not match the model")
    return params, H, W, nb


def forward(model: int, params) -> tuple[np.ndarray, np.ndarray]:
    """P_min, P_max for every vertex; params [n_param][H][W]."""
    params, H, W, nb = _grid(params, model)
    pmin = np.empty((H, W)); pmax = np.empty((H, W))
    _check(_load().or_forward(model, H, W, nb, _ptr(params), _ptr(pmin), _ptr(pmax)), "forward")
    return pmin, pmax


def forward_at(model: int, params, idx) -> tuple[np.ndarray, np.ndarray]:
    """P_min, P_max at flat vertex indices idx (y * W + x)."""
    params, H, W, nb = _grid(params, model)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    pmin = np.empty(idx.size); pmax = np.empty(idx.size)
    _check(_load().or_forward_at(model, H, W, nb, _ptr(params), idx.size, _ptr(idx), _ptr(pmin),
                                 _ptr(pmax)), "forward_at")
    return pmin, pmax


def saddle_at(model: int, params, idx) -> tuple[np.ndarray, np.ndarray]:
    """Saddle terms (t1, t2) at flat vertex indices; P_saddle = t1 + t2
    (interior vertices; boundary vertices give 0)."""
    params, H, W, nb = _grid(params, model)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    t1 = np.empty(idx.size); t2 = np.empty(idx.size)
    _check(_load().or_saddle_at(model, H, W, nb, _ptr(params), idx.size, _ptr(idx), _ptr(t1), _ptr(t2)),
           "saddle_at")
    return t1, t2


def saddle(model: int, params) -> np.ndarray:
    """P_saddle = t1 + t2 for every vertex: [H][W]."""
    params = _f64(params)
    _, H, W = params.shape
    t1, t2 = saddle_at(model, params, np.arange(H * W))
    return (t1 + t2).reshape(H, W)


def jacobian_at(model: int, params, idx) -> tuple[np.ndarray, np.ndarray]:
    """dP/dtheta of the stencils centred at idx: arrays [n][NSLOT][n_param]."""
    params, H, W, nb = _grid(params, model)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    npar = params.shape[0]
    jmin = np.zeros((idx.size, NSLOT, npar)); jmax = np.zeros((idx.size, NSLOT, npar))
    _check(_load().or_jacobian_at(model, H, W, nb, _ptr(params), idx.size, _ptr(idx), _ptr(jmin),
                                  _ptr(jmax)), "jacobian_at")
    return jmin, jmax


def grad(model: int, params, gmin, gmax, absolute: bool = False) -> np.ndarray:
    """Adjoint over the whole grid: [n_param][H][W].  absolute=True returns
    the sum of the magnitudes of the contributing terms instead."""
    params, H, W, nb = _grid(params, model)
    gmin = _f64(gmin); gmax = _f64(gmax)
    out = np.empty_like(params)
    _check(_load().or_grad(model, H, W, nb, _ptr(params), _ptr(gmin), _ptr(gmax), _ptr(out), int(absolute)),
           "grad")
    return out


def grad_at(model: int, params, gmin, gmax, idx, absolute: bool = False) -> np.ndarray:
    """Adjoint at flat vertex indices: [n][n_param] (absolute: see grad)."""
    params, H, W, nb = _grid(params, model)
    gmin = _f64(gmin); gmax = _f64(gmax)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty((idx.size, params.shape[0]))
    _check(_load().or_grad_at(model, H, W, nb, _ptr(params), _ptr(gmin), _ptr(gmax), idx.size,
                              _ptr(idx), _ptr(out), int(absolute)), "grad_at")
    return out


def fit(model: int, members, nbins: int = 0, single: bool = False, ddof: int = 1,
        bw: float = 1.06, eps: float | None = None) -> np.ndarray:
    """Per-vertex parameters from ensemble members [M][H][W].

    single=True: the field is FP32 (members are FP32 values) and the decisions
    floating point takes (degenerate widening, histogram bins) follow FP32.
    """
    members = _f64(members)
    M, H, W = members.shape
    if eps is None:
        eps = 2.0 ** -20 if single else 2.0 ** -30
    out = np.empty((n_param(model, nbins), H, W))
    _check(_load().or_fit(model, int(single), _ptr(members), M, H, W, nbins, ddof, bw, eps, _ptr(out)),
           "fit")
    return out


def gauss_at(params, idx) -> np.ndarray:
    """Independent Gaussian model, params [2][H][W] = (mu, sigma): returns
    [n][4] = (P_min, P_max, t1, t2) at flat vertex indices (saddle terms 0
    off the interior)."""
    params = _f64(params)
    _, H, W = params.shape
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty((idx.size, 4))
    _check(_load().or_gauss_at(H, W, _ptr(params), idx.size, _ptr(idx), _ptr(out)), "gauss_at")
    return out


def gauss(params) -> np.ndarray:
    """[4][H][W] = (P_min, P_max, t1, t2) of every vertex (independent Gaussian)."""
    params = _f64(params)
    _, H, W = params.shape
    return gauss_at(params, np.arange(H * W)).T.reshape(4, H, W).copy()


def gauss_jacobian_at(params, idx, absolute: bool = False):
    """Independent Gaussian: derivatives of P_min and P_max of the stencils
    centred at idx with respect to (mu, sigma) of their slots (v, e, n, w,
    s): two arrays [n][5][2] (absent slots 0).  absolute: the integrals of
    the magnitudes of the same integrands (the scale of rounding in any
    quadrature of them)."""
    params = _f64(params)
    _, H, W = params.shape
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    jm = np.empty((idx.size, 5, 2))
    jx = np.empty((idx.size, 5, 2))
    _check(_load().or_gauss_jacobian_at(H, W, _ptr(params), idx.size, _ptr(idx), _ptr(jm), _ptr(jx),
                                               int(absolute)),
           "gauss_jacobian_at")
    return jm, jx


def gauss_grad_at(params, gmin, gmax, idx, absolute: bool = False) -> np.ndarray:
    """Independent Gaussian adjoint at flat indices: [n][2] (d/d mu, d/d sigma)
    of sum g_min P_min + g_max P_max (absolute: the sum over the contributing
    terms of |g| times the integral of the magnitude of the integrand)."""
    params = _f64(params)
    _, H, W = params.shape
    gmin = _f64(gmin); gmax = _f64(gmax)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty((idx.size, 2))
    _check(_load().or_gauss_grad_at(H, W, _ptr(params), _ptr(gmin), _ptr(gmax), idx.size, _ptr(idx), _ptr(out),
                                    int(absolute)), "gauss_grad_at")
    return out


def semi_at(params, idx, nsamples: int, seed: int, field_id: int = 0) -> np.ndarray:
    """Semianalytical histogram estimator (Sec. 4.4.2), params [2+h][H][W]:
    [n][4] = (P_min, P_max, t1, t2) estimates from `nsamples` Philox samples
    of each vertex histogram (saddle terms 0 off the interior)."""
    params, H, W, nb = _grid(params, HISTOGRAM)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty((idx.size, 4))
    _check(_load().or_semi_at(H, W, nb, _ptr(params), nsamples, seed, field_id, idx.size, _ptr(idx), _ptr(out)),
           "semi_at")
    return out


def semi_samples(params, y: int, x: int, nsamples: int, seed: int, field_id: int = 0) -> np.ndarray:
    """The sample positions the semianalytical estimator draws at (y, x)."""
    params, H, W, nb = _grid(params, HISTOGRAM)
    out = np.empty(nsamples)
    _check(_load().or_semi_samples(H, W, nb, _ptr(params), y, x, nsamples, seed, field_id, _ptr(out)),
           "semi_samples")
    return out


def fit_error_bound(decompressed, eb: float, single: bool = False) -> np.ndarray:
    """Uniform model of an error-bounded lossy reconstruction (Sec. 5.3,
    climate data): every value lies in [d' - eb/2, d' + eb/2] around the
    decompressed value d'.  single=True: both ends are FP32 values, each the
    FP32 rounding of the exact difference / sum (FP32 inputs and eb/2
    rounded to FP32)."""
    if single:
        d = np.asarray(decompressed, dtype=np.float32)
        h = np.float32(eb * 0.5)
        out = np.stack([d - h, d + h]).astype(np.float64)
    else:
        d = _f64(decompressed)
        out = np.stack([d - eb * 0.5, d + eb * 0.5])
    return out


def philox4x32_10(counter, key) -> np.ndarray:
    c = np.ascontiguousarray(counter, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.empty(4, dtype=np.uint32)
    _load().or_philox4x32_10(_ptr(c), _ptr(k), _ptr(out))
    return out


def mvg_fit(members, ddof: int = 1, jitter: float = 1e-6) -> np.ndarray:
    """Mean plane + packed Cholesky factor: [16][H][W]."""
    members = _f64(members)
    M, H, W = members.shape
    out = np.empty((16, H, W))
    rc = _load().or_mvg_fit(_ptr(members), M, H, W, ddof, jitter, _ptr(out))
    _check(rc, "mvg_fit")
    return out


def mvg_forward_at(params, idx, nsamples: int, seed: int, field_id: int = 0):
    """Returns (est [n][4] = hit_min, hit_max, rb_min, rb_max; amb [n][2])."""
    params = _f64(params)
    _, H, W = params.shape
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty((idx.size, 4)); amb = np.empty((idx.size, 2), dtype=np.int32)
    _check(_load().or_mvg_forward_at(_ptr(params), H, W, nsamples, seed, field_id, idx.size, _ptr(idx),
                                     _ptr(out), _ptr(amb)), "mvg_forward_at")
    return out, amb


def mvg_grad_at(params, gmin, gmax, idx, nsamples: int, seed: int, field_id: int = 0, slack: bool = False):
    """Gradient of the conditional estimator at idx: [n][16] (mu gathered, L
    local).  With slack=True also returns the near-tie slack [n][16]: per
    component, the summed magnitude of the sample terms whose extreme
    neighbour is within rounding of another present neighbour (0 where no
    such sample occurs), i.e. how far a computation that breaks those ties
    the other way may differ."""
    params = _f64(params)
    _, H, W = params.shape
    gmin = _f64(gmin); gmax = _f64(gmax)
    idx = np.ascontiguousarray(idx, dtype=np.int64)
    out = np.empty((idx.size, 16))
    sl = np.empty((idx.size, 16)) if slack else None
    _check(_load().or_mvg_grad_at(_ptr(params), H, W, nsamples, seed, field_id, _ptr(gmin), _ptr(gmax),
                                  idx.size, _ptr(idx), _ptr(out), _ptr(sl) if slack else None), "mvg_grad_at")
    return (out, sl) if slack else out
