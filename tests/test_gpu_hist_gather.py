"""The histogram adjoint's gather in its two forms: 16 bytes of vertices per
thread (rows and planes in 16-byte units: four FP32 or two FP64 vertices)
and one vertex per thread (every other width; also the form of the batched
persistent pass).  Both add the five stencils' entries of a mass in the same
order, so the per-field adjoint (vector gather where the layout allows it)
must equal the batched adjoint (scalar gather) bit for bit, and both the
oracle within the gradient tolerance.  Shapes put the row ends, the first
and last rows and single-group rows under the vector form."""
import sys

import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_2407_18015_amd as cp
from paper_2407_18015_amd import _lib as L

pytestmark = pytest.mark.gpu

HST = 2


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.load()
    return torch.device("cuda:0")


def note(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def tol(ref, S, dtype):
    if dtype == torch.float32:
        return 1e-5 * (1 + np.abs(ref)) + 5e-7 * S
    return 1e-10 * (1 + np.abs(ref)) + 1e-13 * S


# (H, W): W = 4, 8, 64, 132 take the vector form in both precisions, 6 and 10
# in FP64 only (two vertices per 16 bytes), 7 in neither
SHAPES = [(5, 4), (1, 8), (7, 8), (3, 64), (9, 132), (6, 6), (4, 10), (5, 7)]


@pytest.mark.parametrize("shape", SHAPES)
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_vector_gather_equals_scalar_gather_and_oracle(dtype, shape):
    H, W = shape
    nb = 5
    note("histogram gather", dtype, shape)
    p = workloads.random_params(HST, 90 + H * W, H, W, nbins=nb, width=0.06)
    pt = torch.as_tensor(p, dtype=dtype, device="cuda")
    gmin, gmax = workloads.upstream(3, H, W, np.float64)
    g1 = torch.as_tensor(gmin, dtype=dtype, device="cuda")
    g2 = torch.as_tensor(gmax, dtype=dtype, device="cuda")
    f = cp.field_of(pt, HST, nb)
    got = cp.backward(pt, g1, g2, f)
    ref_b = torch.empty_like(pt)
    cp.batched([f], [pt], gmin=[g1], gmax=[g2], grad=[ref_b])
    torch.cuda.synchronize()
    assert torch.equal(got, ref_b), "per-field and batched adjoints differ"
    gh = got.cpu().numpy().astype(np.float64)
    args = (HST, pt.cpu().numpy().astype(np.float64), g1.cpu().numpy().astype(np.float64),
            g2.cpu().numpy().astype(np.float64))
    ref, S = oracle.grad(*args), oracle.grad(*args, absolute=True)
    d = np.abs(gh - ref)
    t = tol(ref, S, dtype)
    print(f"[parity] histogram gather {dtype} {shape}: max |diff| {d.max():.3e}, worst |diff|/tolerance "
          f"{(d / t).max():.3g}", flush=True)
    assert np.all(d <= t)


@pytest.mark.parametrize("nb", [1, 2, 32])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_adjoint_bin_count_extremes(dtype, nb):
    """One bin, two bins and the largest count (32: the FP64 sweep then
    takes its two-row tiles): per-field (vector gather) against batched
    (scalar gather) bit for bit, and the oracle within tolerance."""
    H, W = 13, 24
    note("histogram adjoint bins", dtype, nb)
    p = workloads.random_params(HST, 300 + nb, H, W, nbins=nb, width=0.06)
    pt = torch.as_tensor(p, dtype=dtype, device="cuda")
    gmin, gmax = workloads.upstream(5, H, W, np.float64)
    g1 = torch.as_tensor(gmin, dtype=dtype, device="cuda")
    g2 = torch.as_tensor(gmax, dtype=dtype, device="cuda")
    f = cp.field_of(pt, HST, nb)
    got = cp.backward(pt, g1, g2, f)
    ref_b = torch.empty_like(pt)
    cp.batched([f], [pt], gmin=[g1], gmax=[g2], grad=[ref_b])
    torch.cuda.synchronize()
    assert torch.equal(got, ref_b), "per-field and batched adjoints differ"
    gh = got.cpu().numpy().astype(np.float64)
    args = (HST, pt.cpu().numpy().astype(np.float64), g1.cpu().numpy().astype(np.float64),
            g2.cpu().numpy().astype(np.float64))
    ref, S = oracle.grad(*args), oracle.grad(*args, absolute=True)
    d = np.abs(gh - ref)
    t = tol(ref, S, dtype)
    print(f"[parity] histogram adjoint {dtype} {nb} bins: max |diff| {d.max():.3e}, worst |diff|/tolerance "
          f"{(d / t).max():.3g}", flush=True)
    assert np.all(d <= t)
