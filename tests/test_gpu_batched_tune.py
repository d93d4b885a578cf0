"""GPU: tile shapes of the batched launch, pinned one by one and chosen by
the autotuner.  Every shape, claim chunk and the one-tile-per-block form
must give exactly the per-field launches' results (the tile shape changes no per-vertex
arithmetic); the tuner must record its choice and reuse it.
"""
import sys

import numpy as np
import pytest
import torch

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


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def mixed_fields(seed, dtype, n=9, lo=4.0, hi=7.5):
    """n fields of 2^U[lo, hi] per side, models uniform / Epanechnikov /
    histogram (10 bins) in turn."""
    rng = np.random.default_rng(seed)
    fields, params = [], []
    for i in range(n):
        H = int(round(2 ** rng.uniform(lo, hi)))
        W = int(round(2 ** rng.uniform(lo, hi)))
        model = i % 3
        p = dev(workloads.random_params(model, seed * 100 + i, H, W, nbins=10, width=0.05), dtype)
        fields.append(cp.field_of(p, model, 10 if model == HST else 0))
        params.append(p)
    return fields, params


def upstream(fields, dtype):
    g = [workloads.upstream(i, f.height, f.width) for i, f in enumerate(fields)]
    return [dev(a, dtype) for a, _ in g], [dev(b, dtype) for _, b in g]


def outputs(fields, dtype):
    pmin = [torch.full((f.height, f.width), -1.0, dtype=dtype, device="cuda") for f in fields]
    pmax = [torch.full((f.height, f.width), -1.0, dtype=dtype, device="cuda") for f in fields]
    return pmin, pmax


def check_forward(fields, params, pmin, pmax, what):
    torch.cuda.synchronize()
    for i, (f, p) in enumerate(zip(fields, params)):
        a, b = cp.forward(p, f)
        assert torch.equal(a, pmin[i]) and torch.equal(b, pmax[i]), f"{what}: field {i}"


def check_backward(fields, params, gmin, gmax, grad, what):
    torch.cuda.synchronize()
    for i, (f, p) in enumerate(zip(fields, params)):
        assert torch.equal(cp.backward(p, gmin[i], gmax[i], f), grad[i]), f"{what}: field {i}"


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_every_forward_shape_and_chunk(dtype):
    fields, params = mixed_fields(11, dtype)
    for shape in (0, 1, 2):
        for chunk in (1, 3, "flat"):
            note("pinned forward shape", shape, "chunk", chunk, dtype)
            cp.batched_pin(fields, fwd=True, shape={"forward": shape, "hist_forward": min(shape, 1)},
                           chunk={"forward": chunk, "hist_forward": chunk})
            d = cp.batched_describe(fields, fwd=True)
            form = "one tile per block" if chunk == "flat" else f"chunk {chunk}"
            assert d.startswith("pinned") and f"shape {shape}" in d and form in d, d
            pmin, pmax = outputs(fields, dtype)
            cp.batched(fields, params, pmin=pmin, pmax=pmax)
            check_forward(fields, params, pmin, pmax, f"shape {shape} chunk {chunk}")


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_every_adjoint_shape_and_chunk(dtype):
    fields, params = mixed_fields(12, dtype)
    gmin, gmax = upstream(fields, dtype)
    for shape in (0, 1, 2):
        for chunk in (1, 3, "flat"):
            note("pinned adjoint shape", shape, "chunk", chunk, dtype)
            hs = min(shape, 1)
            cp.batched_pin(fields, fwd=False, bwd=True, shape={"adjoint": shape, "hist_adjoint": hs},
                           chunk={"adjoint": chunk, "hist_adjoint": chunk, "hist_gather": chunk})
            grad = [torch.full_like(p, -1.0) for p in params]
            cp.batched(fields, params, None, None, gmin, gmax, grad)
            check_backward(fields, params, gmin, gmax, grad, f"shape {shape} chunk {chunk}")


def test_pin_rejects_unknown_shape():
    fields, _ = mixed_fields(13, torch.float32, n=3)
    with pytest.raises(L.CPError):
        cp.batched_pin(fields, fwd=True, shape={"forward": 3})
    with pytest.raises(ValueError):
        cp.batched_pin(fields, fwd=True, shape={"sideways": 0})


@pytest.mark.parametrize("graph", [False, True])
def test_tuned_forward_backward(graph):
    """fwd + bwd with tuning on the first call; later calls (and graph
    replays) reuse the choice and match the per-field launches."""
    note("tuned fwd+bwd graph", graph)
    dtype = torch.float32
    fields, params = mixed_fields(14 + graph, dtype, n=12, lo=5.0, hi=9.0)
    gmin, gmax = upstream(fields, dtype)
    assert cp.batched_describe(fields, fwd=True, bwd=True) is None
    first = None
    for rep in range(3):
        pmin, pmax = outputs(fields, dtype)
        grad = [torch.full_like(p, -1.0) for p in params]
        cp.batched(fields, params, pmin, pmax, gmin, gmax, grad, graph=graph, tune=True)
        d = cp.batched_describe(fields, fwd=True, bwd=True)
        assert d.startswith("tuned") and " ms" in d, d
        first = first or d
        assert d == first  # tuned once
        check_backward(fields, params, gmin, gmax, grad, f"rep {rep}")
        torch.cuda.synchronize()
        for i, (f, p) in enumerate(zip(fields, params)):
            a, b = cp.forward(p, f)
            assert torch.allclose(a, pmin[i], rtol=0, atol=1e-6, equal_nan=True), (rep, i)
            assert torch.allclose(b, pmax[i], rtol=0, atol=1e-6, equal_nan=True), (rep, i)
    note("tuned plan:", first)


def test_tuned_forward_only():
    note("tuned forward")
    dtype = torch.float32
    fields, params = mixed_fields(16, dtype, n=12, lo=5.0, hi=9.0)
    pmin, pmax = outputs(fields, dtype)
    cp.batched(fields, params, pmin=pmin, pmax=pmax, tune=True)
    d = cp.batched_describe(fields, fwd=True)
    assert d.startswith("tuned") and "histogram forward" in d and "; forward" in d, d
    check_forward(fields, params, pmin, pmax, "tuned")
    pmin, pmax = outputs(fields, dtype)
    cp.batched(fields, params, pmin=pmin, pmax=pmax, graph=True)
    assert cp.batched_describe(fields, fwd=True) == d
    check_forward(fields, params, pmin, pmax, "tuned, graph")
    note("tuned plan:", d)


def test_plan_shared_by_two_streams():
    """Calls with the same shapes on two streams, issued back to back with
    no ordering between the streams: the library orders each call after the
    plan's last use on the other stream, so no tile queue is shared in flight
    and every call matches the per-field launches (forward and adjoint)."""
    note("plan on two streams")
    dtype = torch.float32
    fields, params = mixed_fields(18, dtype, n=9)
    gmin, gmax = upstream(fields, dtype)
    main = torch.cuda.current_stream()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for s in streams:
        s.wait_stream(main)  # inputs were written on the main stream
    results = []
    for k in range(6):
        st = streams[k % 2]
        with torch.cuda.stream(st):
            pmin, pmax = outputs(fields, dtype)
            grad = [torch.full_like(p, -1.0) for p in params]
            cp.batched(fields, params, pmin, pmax, gmin, gmax, grad, graph=(k >= 2))
        results.append((pmin, pmax, grad))
    torch.cuda.synchronize()
    for k, (pmin, pmax, grad) in enumerate(results):
        check_backward(fields, params, gmin, gmax, grad, f"call {k}")
        for i, (f, p) in enumerate(zip(fields, params)):
            a, b = cp.forward(p, f)
            assert torch.allclose(a, pmin[i], rtol=0, atol=1e-6, equal_nan=True), (k, i)
            assert torch.allclose(b, pmax[i], rtol=0, atol=1e-6, equal_nan=True), (k, i)


def test_tuning_table_persists(tmp_path, monkeypatch):
    """With CPCRIT_TUNE_CACHE set, the first tuned call records its choices;
    after cp_release (as in a new process) the same shapes take them from the
    table instead of timing again, and give the per-field results."""
    note("tuning table")
    table = tmp_path / "tune.txt"
    monkeypatch.setenv("CPCRIT_TUNE_CACHE", str(table))
    dtype = torch.float32
    fields, params = mixed_fields(19, dtype, n=7)
    gmin, gmax = upstream(fields, dtype)

    def call():
        pmin, pmax = outputs(fields, dtype)
        grad = [torch.full_like(p, -1.0) for p in params]
        cp.batched(fields, params, pmin, pmax, gmin, gmax, grad, tune=True)
        check_backward(fields, params, gmin, gmax, grad, "table")
        return cp.batched_describe(fields, fwd=True, bwd=True)

    first = call()
    assert first.startswith("tuned;"), first
    lines = table.read_text().splitlines()
    assert len(lines) == 1 and lines[0].startswith("cpcrit-tune-1 ")
    L.check(L.cp_release())
    second = call()
    assert second.startswith("tuned (table);"), second
    # the same shapes and chunks (launch times aside)
    import re
    strip = lambda d: re.sub(r", [0-9.]+ ms", "", d.split(";", 1)[1])
    assert strip(second) == strip(first)
    assert len(table.read_text().splitlines()) == 1  # nothing re-timed, nothing appended
