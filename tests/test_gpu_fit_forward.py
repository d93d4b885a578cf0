"""cp_fit_forward (fit and forward in one call) against the two separate
calls, bit for bit, and against the FP64 oracle; fused tiles (uniform,
Epanechnikov with 16-byte aligned rows) and the two-launch path (other
widths and models)."""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_2407_18015_amd as cp
from paper_2407_18015_amd import _lib as L

pytestmark = pytest.mark.gpu

TOL = {torch.float32: 1e-6, torch.float64: 1e-12}


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.load()
    return torch.device("cuda:0")


def note(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def members(seed, H, W, dtype, M=20):
    return torch.as_tensor(workloads.smooth_ensemble(seed, H, W, M), dtype=dtype, device="cuda")


def separate(mem, model, **kw):
    params = cp.fit(mem, model)
    f = cp.field_of(params, model, **kw)
    pmin, pmax = cp.forward(params, f)
    return params, pmin, pmax


def same(a, b, what):
    assert torch.equal(torch.nan_to_num(a, 7.0), torch.nan_to_num(b, 7.0)), what


# (H, W): W a multiple of 4 takes the fused tiles in FP32 and FP64; tall
# grids take the 64 x 12 tiles (1030 x 2112: 33 x 86 tiles, the last rows ragged)
SHAPES = [(1, 4), (3, 8), (5, 68), (67, 132), (131, 196), (1030, 2112)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("model", [L.CP_UNIFORM, L.CP_EPANECHNIKOV])
def test_fused_equals_fit_then_forward(model, dtype, shape):
    H, W = shape
    note("fit_forward", model, dtype, shape)
    mem = members(3, H, W, dtype)
    params, pmin, pmax = cp.fit_forward(mem, model)
    rp, rmin, rmax = separate(mem, model)
    same(params, rp, "params")
    same(pmin, rmin, "P_min")
    same(pmax, rmax, "P_max")


@pytest.mark.parametrize("model", [L.CP_UNIFORM, L.CP_EPANECHNIKOV])
def test_fused_against_oracle(model):
    """37 x 68 FP32 (two tile columns, ragged rows): probabilities of the
    fitted field within 1e-6 of the oracle's on the same parameters, and the
    parameters within the fit tolerances of the oracle's fit."""
    note("fit_forward vs oracle", model)
    H, W = 37, 68
    mem_np = workloads.smooth_ensemble(5, H, W)
    params, pmin, pmax = cp.fit_forward(torch.as_tensor(mem_np, device="cuda"), model)
    ph = params.double().cpu().numpy()
    ref = oracle.fit(model, mem_np.astype(np.float64), single=True)
    if model == L.CP_UNIFORM:  # min / max: exact
        assert np.array_equal(params.cpu().numpy(), ref.astype(np.float32))
    else:  # FP64 sums rounded once to FP32
        np.testing.assert_allclose(params.cpu().numpy(), ref.astype(np.float32), rtol=2.5e-7, atol=0)
    rmin, rmax = oracle.forward(model, ph)
    d = max(np.abs(pmin.double().cpu().numpy() - rmin).max(), np.abs(pmax.double().cpu().numpy() - rmax).max())
    print(f"[parity] fit_forward {model}: max |diff| {d:.3e} (tolerance 1e-06)", flush=True)
    assert d <= 1e-6


@pytest.mark.parametrize("shape", [(9, 131), (4, 3), (2, 1)])
def test_unaligned_width_runs_two_launches(shape):
    """Widths that are not a multiple of 16 bytes take the separate fit and
    forward launches; same results."""
    H, W = shape
    note("fit_forward unaligned", shape)
    mem = members(4, H, W, torch.float32)
    for model in (L.CP_UNIFORM, L.CP_EPANECHNIKOV):
        params, pmin, pmax = cp.fit_forward(mem, model)
        rp, rmin, rmax = separate(mem, model)
        same(params, rp, "params")
        same(pmin, rmin, "P_min")
        same(pmax, rmax, "P_max")


def test_other_models_run_two_launches():
    note("fit_forward histogram / Gaussian / multivariate Gaussian")
    mem = members(6, 33, 40, torch.float32)
    params, pmin, pmax = cp.fit_forward(mem, L.CP_HISTOGRAM, nbins=10)
    rp = cp.fit(mem, L.CP_HISTOGRAM, nbins=10)
    rmin, rmax = cp.forward(rp, cp.field_of(rp, L.CP_HISTOGRAM, 10))
    same(params, rp, "histogram params")
    same(pmin, rmin, "histogram P_min")
    same(pmax, rmax, "histogram P_max")
    params, pmin, pmax = cp.fit_forward(mem, L.CP_GAUSSIAN)
    rp, rmin, rmax = separate(mem, L.CP_GAUSSIAN)
    same(params, rp, "Gaussian params")
    same(pmin, rmin, "Gaussian P_min")
    same(pmax, rmax, "Gaussian P_max")
    params, pmin, pmax = cp.fit_forward(mem, L.CP_MVGAUSS, nsamples=256, seed=5)
    rp = cp.fit(mem, L.CP_MVGAUSS)
    rmin, rmax = cp.forward(rp, cp.field_of(rp, L.CP_MVGAUSS, nsamples=256, seed=5))
    same(params, rp, "multivariate params")
    same(pmin, rmin, "multivariate P_min")
    same(pmax, rmax, "multivariate P_max")


def test_degenerate_and_invalid_members():
    """All-equal members (degenerate widening) and a NaN member in the tile
    halo: identical to the separate calls, NaN pattern included."""
    note("fit_forward degenerate / NaN")
    H, W = 20, 72
    mem = members(7, H, W, torch.float32)
    mem[:, 3:6, 10:14] = 0.25
    mem[4, 15, 63] = float("nan")  # the last column of the first tile: halo of the second
    for model in (L.CP_UNIFORM, L.CP_EPANECHNIKOV):
        params, pmin, pmax = cp.fit_forward(mem, model)
        rp, rmin, rmax = separate(mem, model)
        same(params, rp, "params")
        same(pmin, rmin, "P_min")
        same(pmax, rmax, "P_max")
        assert torch.isnan(pmin[15, 64]) == torch.isnan(rmin[15, 64])
