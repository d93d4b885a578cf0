"""The allocation-free adjoint (cp_prob_backward_noalloc) against
cp_prob_backward, called through the C ABI: bit-identical gradients for the
two models whose adjoints pass partials through scratch memory (histogram,
multivariate Gaussian) and for one that needs none, on two calls in a row of
which the second is smaller (the fixed array keeps the first call's
contents); device memory in use does not change across a call; a field that
needs more scratch than the array holds is refused before any launch."""
import sys

import numpy as np
import pytest
import torch

import workloads
import paper_2407_18015_amd as cp
from paper_2407_18015_amd import _lib as L

pytestmark = pytest.mark.gpu

SCRATCH_BYTES = 64 << 20


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.load()
    return torch.device("cuda:0")


def note(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def case(model, H, W, seed):
    """(params, field, g_min, g_max) of a seeded, fitted field."""
    if model == "mvg":
        p = cp.fit(dev(workloads.correlated_ensemble(seed, H, W)), "mvg")
        f = cp.Field(H, W, L.CP_MVGAUSS, torch.float32, nsamples=192, seed=11 + seed, field_id=seed)
    elif model == "histogram":
        nb = 10 if seed % 2 == 0 else 6
        p = cp.fit(dev(workloads.mixture_ensemble(seed, H, W)), "histogram", nbins=nb)
        f = cp.field_of(p, "histogram", nb)
    else:
        p = cp.fit(dev(workloads.smooth_ensemble(seed, H, W)), model)
        f = cp.field_of(p, model)
    g1, g2 = workloads.upstream(seed, H, W)
    return p, f, dev(g1), dev(g2)


@pytest.mark.parametrize("model", ["histogram", "mvg", "epanechnikov"])
def test_noalloc_matches_backward_on_two_calls(model):
    shapes = [(70, 90, 0), (33, 41, 1)] if model != "mvg" else [(40, 52, 0), (17, 23, 1)]
    for H, W, seed in shapes:
        note("noalloc", model, H, W, seed)
        p, f, g1, g2 = case(model, H, W, seed)
        ref = cp.backward(p, g1, g2, f)
        got = torch.full_like(p, float("nan"))
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        st = L.cp_prob_backward_noalloc(f.desc(), p.data_ptr(), g1.data_ptr(), g2.data_ptr(), got.data_ptr(),
                                        torch.cuda.current_stream().cuda_stream)
        L.check(st)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
        if seed > 0:  # the first call may load the library's code on this device
            assert free1 == free0, f"device memory changed by {free0 - free1} bytes"
        a, b = ref.cpu().numpy(), got.cpu().numpy()
        assert np.array_equal(a, b, equal_nan=True), (
            f"{model} {H}x{W}: {int(np.count_nonzero(a != b))} entries differ, max {np.nanmax(np.abs(a - b))}")
        assert np.isfinite(b).all()


def test_noalloc_python_binding():
    note("noalloc binding")
    p, f, g1, g2 = case("histogram", 21, 35, 2)
    ref = cp.backward(p, g1, g2, f)
    got = cp.backward(p, g1, g2, f, noalloc=True)
    assert torch.equal(ref, got)


def test_noalloc_rejects_fields_beyond_the_array():
    # histogram FP32 with 32 bins: (5 * 32 + 4) * 4 bytes per vertex (the
    # entries and the four tails); no launch happens
    H, W, nb = 512, 256, 32
    need = (5 * nb + 4) * 4 * H * W
    assert need > SCRATCH_BYTES
    p = torch.zeros((2 + nb, H, W), device="cuda")
    g = torch.zeros((H, W), device="cuda")
    f = cp.field_of(p, "histogram", nb)
    st = L.cp_prob_backward_noalloc(f.desc(), p.data_ptr(), g.data_ptr(), g.data_ptr(), p.data_ptr(),
                                    torch.cuda.current_stream().cuda_stream)
    assert st == L.CP_EINVAL
    msg = L.load().cp_last_error().decode()
    assert str(need) in msg and str(SCRATCH_BYTES) in msg
    # the largest multivariate Gaussian field that fits is accepted by the size check
    assert 40 * 1024 * 1024 <= SCRATCH_BYTES
