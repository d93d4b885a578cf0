"""Torch-level entry points over the C ABI.

torch supplies device memory (tensors) and the current HIP stream; every
computation runs in libcpcrit.so.  Shapes: parameters [n_param, H, W],
probabilities and upstream gradients [H, W], members [M, H, W].  Tensors may
have a row stride larger than W (all planes of one call must share it).
"""
from __future__ import annotations

from dataclasses import dataclass

import torch

from . import _lib as L

MODELS = {"uniform": L.CP_UNIFORM, "epanechnikov": L.CP_EPANECHNIKOV, "histogram": L.CP_HISTOGRAM,
          "mvg": L.CP_MVGAUSS, "gaussian": L.CP_GAUSSIAN}


def model_id(model) -> int:
    return MODELS[model] if isinstance(model, str) else int(model)


def n_params(model, nbins: int = 0) -> int:
    n = L.cp_n_params(model_id(model), nbins)
    if n < 0:
        raise ValueError("unknown model or bad nbins")
    return n


@dataclass
class Field:
    """Description of one field (mirrors cp_field_desc_t)."""
    height: int
    width: int
    model: int
    dtype: torch.dtype = torch.float32
    nbins: int = 0
    nsamples: int = 0
    seed: int = 0
    field_id: int = 0
    estimator: int = L.CP_MC_CONDITIONAL
    row_stride: int = 0

    def desc(self) -> L.cp_field_desc_t:
        dt = {torch.float32: L.CP_F32, torch.float64: L.CP_F64}[self.dtype]
        return L.cp_field_desc_t(self.height, self.width, self.row_stride, model_id(self.model), dt, self.nbins,
                                 self.nsamples, self.seed, self.field_id, self.estimator)

    @property
    def n_param(self) -> int:
        return n_params(self.model, self.nbins)

    @property
    def param_dtype(self) -> torch.dtype:
        return torch.float64 if model_id(self.model) == L.CP_MVGAUSS else self.dtype

    @property
    def out_dtype(self) -> torch.dtype:
        return torch.float32 if model_id(self.model) == L.CP_MVGAUSS else self.dtype


def _stream(t: torch.Tensor) -> int:
    """The current stream of t's device; the library works on the current
    HIP device, so t must live there."""
    if t.device.type != "cuda":
        raise ValueError(f"expected a GPU tensor, got one on {t.device}")
    if t.device.index != torch.cuda.current_device():
        raise ValueError(f"tensors on {t.device} but the current device is cuda:{torch.cuda.current_device()}: "
                         "call under torch.cuda.device(...)")
    return torch.cuda.current_stream(t.device).cuda_stream


def _ptr(t: torch.Tensor | None):
    return None if t is None else t.data_ptr()


def _planes(t: torch.Tensor, H: int, W: int, dtype: torch.dtype, name: str, row_stride: int = 0) -> None:
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if t.dim() == 2:
        t = t.unsqueeze(0)
    if t.dim() != 3 or t.shape[1] != H or t.shape[2] != W:
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected [*, {H}, {W}]")
    rs = row_stride or W
    if t.stride(2) != 1 or t.stride(1) != rs or (t.shape[0] > 1 and t.stride(0) != H * rs):
        raise ValueError(f"{name} must be dense planes with row stride {rs}")


def field_of(params: torch.Tensor, model, nbins: int = 0, **kw) -> Field:
    m = model_id(model)
    H, W = params.shape[-2], params.shape[-1]
    dtype = kw.pop("dtype", torch.float32 if m == L.CP_MVGAUSS else params.dtype)
    if m == L.CP_HISTOGRAM and nbins == 0:
        nbins = params.shape[0] - 2
    return Field(H, W, m, dtype, nbins, **kw)


def fit(members: torch.Tensor, model, nbins: int = 0, ddof: int = 1, bw_factor: float = 1.06,
        cov_jitter: float = 1e-6, degenerate_eps: float = 0.0, out: torch.Tensor | None = None) -> torch.Tensor:
    """cpu_fit_params: per-vertex model parameters from members [M, H, W]."""
    M, H, W = members.shape
    f = Field(H, W, model_id(model), members.dtype, nbins)
    _planes(members, H, W, members.dtype, "members")
    if out is None:
        out = torch.empty((f.n_param, H, W), dtype=f.param_dtype, device=members.device)
    _planes(out, H, W, f.param_dtype, "params")
    opts = L.cp_fit_opts_t(ddof, bw_factor, cov_jitter, degenerate_eps)
    L.check(L.cpu_fit_params(f.desc(), _ptr(members), M, opts, _ptr(out), _stream(members)))
    return out


def fit_forward(members: torch.Tensor, model, nbins: int = 0, ddof: int = 1, bw_factor: float = 1.06,
                cov_jitter: float = 1e-6, degenerate_eps: float = 0.0, out: torch.Tensor | None = None,
                pmin: torch.Tensor | None = None, pmax: torch.Tensor | None = None, **kw):
    """cp_fit_forward: fit (as `fit`) and forward (as `forward`) in one call;
    returns (params, P_min, P_max).  kw: Field options of the forward
    (nsamples, seed, field_id, estimator for the multivariate Gaussian)."""
    M, H, W = members.shape
    f = Field(H, W, model_id(model), members.dtype, nbins, **kw)
    _planes(members, H, W, members.dtype, "members")
    if out is None:
        out = torch.empty((f.n_param, H, W), dtype=f.param_dtype, device=members.device)
    _planes(out, H, W, f.param_dtype, "params")
    if pmin is None:
        pmin = torch.empty((H, W), dtype=f.out_dtype, device=members.device)
    if pmax is None:
        pmax = torch.empty((H, W), dtype=f.out_dtype, device=members.device)
    _planes(pmin, H, W, f.out_dtype, "p_min")
    _planes(pmax, H, W, f.out_dtype, "p_max")
    opts = L.cp_fit_opts_t(ddof, bw_factor, cov_jitter, degenerate_eps)
    L.check(L.cp_fit_forward(f.desc(), _ptr(members), M, opts, _ptr(out), _ptr(pmin), _ptr(pmax),
                             _stream(members)))
    return out, pmin, pmax


def fit_error_bound(decompressed: torch.Tensor, eb: float, out: torch.Tensor | None = None) -> torch.Tensor:
    """cp_fit_error_bound: uniform parameters [2, H, W] = d' -/+ eb/2 of an
    error-bounded reconstruction d' [H, W]."""
    H, W = decompressed.shape
    f = Field(H, W, L.CP_UNIFORM, decompressed.dtype)
    _planes(decompressed, H, W, decompressed.dtype, "decompressed")
    if out is None:
        out = torch.empty((2, H, W), dtype=decompressed.dtype, device=decompressed.device)
    _planes(out, H, W, decompressed.dtype, "params")
    L.check(L.cp_fit_error_bound(f.desc(), _ptr(decompressed), float(eb), _ptr(out), _stream(decompressed)))
    return out


def forward(params: torch.Tensor, f: Field, pmin: torch.Tensor | None = None, pmax: torch.Tensor | None = None):
    """cp_prob_forward: (P_min, P_max) of every vertex."""
    _planes(params, f.height, f.width, f.param_dtype, "params", f.row_stride)
    if params.shape[0] != f.n_param:
        raise ValueError(f"params needs {f.n_param} planes")
    if pmin is None:
        pmin = torch.empty((f.height, f.width), dtype=f.out_dtype, device=params.device)
    if pmax is None:
        pmax = torch.empty((f.height, f.width), dtype=f.out_dtype, device=params.device)
    _planes(pmin, f.height, f.width, f.out_dtype, "p_min", f.row_stride)
    _planes(pmax, f.height, f.width, f.out_dtype, "p_max", f.row_stride)
    L.check(L.cp_prob_forward(f.desc(), _ptr(params), _ptr(pmin), _ptr(pmax), _stream(params)))
    return pmin, pmax


def backward(params: torch.Tensor, gmin: torch.Tensor, gmax: torch.Tensor, f: Field,
             grad: torch.Tensor | None = None, noalloc: bool = False) -> torch.Tensor:
    """cp_prob_backward: gradient of sum g_min P_min + g_max P_max w.r.t. params.
    noalloc=True calls cp_prob_backward_noalloc (the library's fixed scratch
    array instead of a workspace it allocates; pass `grad` to allocate nothing)."""
    _planes(params, f.height, f.width, f.param_dtype, "params", f.row_stride)
    _planes(gmin, f.height, f.width, f.out_dtype, "g_min", f.row_stride)
    _planes(gmax, f.height, f.width, f.out_dtype, "g_max", f.row_stride)
    if grad is None:
        grad = torch.empty_like(params)
    _planes(grad, f.height, f.width, f.param_dtype, "grad_params", f.row_stride)
    fn = L.cp_prob_backward_noalloc if noalloc else L.cp_prob_backward
    L.check(fn(f.desc(), _ptr(params), _ptr(gmin), _ptr(gmax), _ptr(grad), _stream(params)))
    return grad


def classify(params: torch.Tensor, f: Field, outputs=("min", "max", "saddle", "regular"),
             terms: bool = False) -> dict:
    """cp_prob_classify: the requested subset of P_min, P_max, P_saddle and
    P_regular (each [H, W]) and, with terms=True, the saddle terms [2, H, W]
    (t1, t2).  Returns a dict keyed by "min", "max", "saddle", "regular",
    "terms"."""
    _planes(params, f.height, f.width, f.param_dtype, "params", f.row_stride)
    if params.shape[0] != f.n_param:
        raise ValueError(f"params needs {f.n_param} planes")
    names = set(outputs)
    if not names <= {"min", "max", "saddle", "regular"}:
        raise ValueError(f"unknown outputs {sorted(names)}")
    out = {k: torch.empty((f.height, f.width), dtype=f.out_dtype, device=params.device) for k in sorted(names)}
    if terms:
        out["terms"] = torch.empty((2, f.height, f.width), dtype=f.out_dtype, device=params.device)
    L.check(L.cp_prob_classify(f.desc(), _ptr(params), _ptr(out.get("min")), _ptr(out.get("max")),
                               _ptr(out.get("saddle")), _ptr(out.get("regular")), _ptr(out.get("terms")),
                               _stream(params)))
    return out


def semianalytical(params: torch.Tensor, f: Field, terms: bool = False) -> dict:
    """cp_prob_semianalytical: Monte Carlo over the vertex histogram with
    closed-form neighbour tails (f.nsamples samples, Philox key f.seed,
    counter word f.field_id).  Returns {"min", "max"} ([H, W]) and, with
    terms=True, "terms" ([2, H, W]: t1, t2)."""
    _planes(params, f.height, f.width, f.param_dtype, "params", f.row_stride)
    if params.shape[0] != f.n_param:
        raise ValueError(f"params needs {f.n_param} planes")
    out = {k: torch.empty((f.height, f.width), dtype=f.out_dtype, device=params.device) for k in ("min", "max")}
    if terms:
        out["terms"] = torch.empty((2, f.height, f.width), dtype=f.out_dtype, device=params.device)
    L.check(L.cp_prob_semianalytical(f.desc(), _ptr(params), _ptr(out["min"]), _ptr(out["max"]),
                                     _ptr(out.get("terms")), _stream(params)))
    return out


def _batch_flags(fwd: bool, bwd: bool, graph: bool = False, per_field: bool = False, tune: bool = False) -> int:
    flags = 0
    if fwd:
        flags |= L.CP_BATCH_FWD
    if bwd:
        flags |= L.CP_BATCH_BWD
    if graph:
        flags |= L.CP_BATCH_GRAPH
    if per_field:
        flags |= L.CP_BATCH_PER_FIELD
    if tune:
        flags |= L.CP_BATCH_TUNE
    return flags


def batched(fields: list[Field], params: list[torch.Tensor], pmin=None, pmax=None, gmin=None, gmax=None,
            grad=None, graph: bool = False, per_field: bool = False, tune: bool = False) -> None:
    """cp_prob_batched over caller-allocated outputs (lists of tensors).
    tune=True autotunes the plan's tile shapes on its first call."""
    n = len(fields)
    flags = _batch_flags(pmin is not None, grad is not None, graph, per_field, tune)
    for i, f in enumerate(fields):
        _planes(params[i], f.height, f.width, f.param_dtype, f"params[{i}]", f.row_stride)
    lst = lambda ts: None if ts is None else [_ptr(t) for t in ts]
    L.check(L.cp_prob_batched(n, [f.desc() for f in fields], lst(params), lst(pmin), lst(pmax), lst(gmin),
                              lst(gmax), lst(grad), flags, _stream(params[0])))


BATCH_PASSES = ("forward", "hist_forward", "adjoint", "hist_adjoint", "hist_gather")


def batched_pin(fields: list[Field], fwd: bool = True, bwd: bool = False, shape: dict | None = None,
                chunk: dict | None = None) -> None:
    """cp_batched_pin: fix the tile shape index / claim chunk of passes of the
    plan used by batched calls over these fields (keys of BATCH_PASSES);
    chunk -1 (or "flat") launches one tile per block."""
    shape, chunk = shape or {}, chunk or {}
    for k in list(shape) + list(chunk):
        if k not in BATCH_PASSES:
            raise ValueError(f"unknown pass {k!r}")
    sh = [int(shape.get(k, -1)) for k in BATCH_PASSES]
    ch = [-1 if chunk.get(k) == "flat" else int(chunk.get(k, 0)) for k in BATCH_PASSES]
    L.check(L.cp_batched_pin(len(fields), [f.desc() for f in fields], _batch_flags(fwd, bwd), sh, ch))


def batched_describe(fields: list[Field], fwd: bool = True, bwd: bool = False) -> str | None:
    """cp_batched_describe: the tile shapes, chunks and grids of the plan used
    by batched calls over these fields (None before the first call)."""
    return L.cp_batched_describe(len(fields), [f.desc() for f in fields], _batch_flags(fwd, bwd))


def philox(counters: torch.Tensor, seed: int) -> torch.Tensor:
    """Raw Philox4x32-10 words for counters [n, 4] (int32 storage of uint32)."""
    out = torch.empty_like(counters)
    L.check(L.cp_philox4x32_10(counters.shape[0], _ptr(counters), seed, _ptr(out), _stream(counters)))
    return out


class CPProb(torch.autograd.Function):
    """(P_min, P_max) = CPProb.apply(params, field); backward through the
    library's adjoint kernel."""

    @staticmethod
    def forward(ctx, params: torch.Tensor, f: Field):
        params = params.contiguous()
        pmin, pmax = forward(params, f)
        ctx.save_for_backward(params)
        ctx.field = f
        return pmin, pmax

    @staticmethod
    def backward(ctx, gmin, gmax):
        (params,) = ctx.saved_tensors
        f = ctx.field
        if gmin is None:
            gmin = torch.zeros((f.height, f.width), dtype=f.out_dtype, device=params.device)
        if gmax is None:
            gmax = torch.zeros((f.height, f.width), dtype=f.out_dtype, device=params.device)
        grad = backward(params, gmin.contiguous(), gmax.contiguous(), f)
        return grad, None


def critical_point_probability(params: torch.Tensor, model, nbins: int = 0, **kw):
    """Differentiable (P_min, P_max) for a parameter field."""
    return CPProb.apply(params, field_of(params, model, nbins, **kw))
