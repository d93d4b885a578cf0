"""GPU parity: the HIP library (through the C ABI) against the FP64 oracle,
element by element on the same seeded inputs.

Tolerances: probabilities 1e-6 absolute in FP32 and 1e-12 in FP64; gradients
|d| <= 1e-5 (1 + |g|) + 5e-7 S in FP32 and 1e-10 (1 + |g|) + 1e-13 S in FP64,
where S is the sum of the magnitudes of the ten terms the adjoint adds (five
stencils, two sides): the gradient is a sum whose terms scale like 1/width
and cancel, so its rounding error is relative to S, not to g; Monte Carlo: raw
Philox words bit-identical, conditional estimator within 1e-6, hit counts
equal up to samples whose decision margin is below the oracle's ambiguity
threshold; histogram bins (an integer decision) identical.
"""
import os
import sys

import numpy as np
import pytest
import torch

import exact_stencil
import oracle
import workloads
import paper_2407_18015_amd as cp
from paper_2407_18015_amd import _lib as L

pytestmark = pytest.mark.gpu

U, E, HST, MVG = 0, 1, 2, 3
NAMES = {U: "uniform", E: "epanechnikov", HST: "histogram"}


@pytest.fixture(scope="module", autouse=True)
def device():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    L.load()  # fail loudly if the library is missing
    return torch.device("cuda:0")


def note(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def dev(a, dtype):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def fitted_params(model, seed, H, W, nbins=10):
    """Config-shaped parameters: GPU fit of a seeded ensemble (float32)."""
    if model == HST:
        mem = workloads.mixture_ensemble(seed, H, W)
    else:
        mem = workloads.smooth_ensemble(seed, H, W)
    return cp.fit(dev(mem, torch.float32), model, nbins=nbins if model == HST else 0), mem


def gpu_forward(params, model, nbins=0):
    f = cp.field_of(params, model, nbins)
    return cp.forward(params, f)


def report(what, text):
    """One line per checked output (visible with pytest -s): the measured
    error beside its tolerance."""
    print(f"[parity] {what}: {text}", flush=True)


def assert_close(got, ref, atol, what):
    d = np.abs(got - ref)
    i = int(np.nanargmax(d)) if d.size else 0
    if d.size:
        report(what, f"max |diff| {np.nanmax(d):.3e} (tolerance {atol:.0e}, {d.size} values)")
    assert np.all(np.isfinite(got) == np.isfinite(ref)), f"{what}: NaN pattern differs"
    assert np.nanmax(d) <= atol, f"{what}: max |diff| {np.nanmax(d):.3e} at flat {i} (got {got.flat[i]}, ref {ref.flat[i]})"


# ----------------------------------------------------------------------------
# forward
# ----------------------------------------------------------------------------
EXACT_2D = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "exact_2d_stencils.txt")


@pytest.mark.parametrize("case", exact_stencil.load_cases(EXACT_2D), ids=lambda c: c["name"])
@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
def test_exact_2d_stencils(case, dtype):
    """The exact rationals of the 2-D uniform, Epanechnikov and histogram
    stencils (Eq. 3, Sec. 4.3, Sec. 4.4.1 / Eq. 5; fixture re-derived with
    fractions on the CPU): FP64 within 1e-12, FP32 within 1e-6."""
    note("exact 2-D stencil", case["name"], dtype)
    model, nb, grid = exact_stencil.case_grid(case)
    pmin, pmax = gpu_forward(dev(grid, dtype), model, nb)
    tol = 1e-12 if dtype == torch.float64 else 1e-6
    assert abs(host(pmin)[1, 1] - float(case["p_min"])) <= tol
    assert abs(host(pmax)[1, 1] - float(case["p_max"])) <= tol


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_forward_fp64_uniform_64x64(seed):
    """Independent uniform noise on a 64x64 grid in FP64 (1e-12)."""
    note("fp64 uniform 64x64 seed", seed)
    p = workloads.uniform_params_field(seed, 64, 64)
    pmin, pmax = gpu_forward(dev(p, torch.float64), U)
    rmin, rmax = oracle.forward(U, p)
    assert_close(host(pmin), rmin, 1e-12, "P_min")
    assert_close(host(pmax), rmax, 1e-12, "P_max")


@pytest.mark.parametrize("model", [U, E, HST])
@pytest.mark.parametrize("dtype,tol", [(torch.float32, 1e-6), (torch.float64, 1e-12)])
def test_forward_random_fields_ragged(model, dtype, tol):
    """131x197 grid (several tiles, ragged tail in both directions)."""
    note("forward", NAMES[model], dtype, "131x197")
    p = workloads.random_params(model, 3 + model, 131, 197, nbins=7, width=0.06)
    pt = dev(p, dtype)
    pmin, pmax = gpu_forward(pt, model, 7 if model == HST else 0)
    rmin, rmax = oracle.forward(model, host(pt))
    assert_close(host(pmin), rmin, tol, "P_min")
    assert_close(host(pmax), rmax, tol, "P_max")


@pytest.mark.parametrize("model", [U, E, HST])
def test_forward_fitted_fields(model):
    """Parameters fitted on the GPU from config-shaped ensembles."""
    note("forward fitted", NAMES[model], "160x210")
    params, _ = fitted_params(model, 5, 160, 210)
    pmin, pmax = gpu_forward(params, model, 10 if model == HST else 0)
    rmin, rmax = oracle.forward(model, host(params))
    assert_close(host(pmin), rmin, 1e-6, "P_min")
    assert_close(host(pmax), rmax, 1e-6, "P_max")


@pytest.mark.parametrize("shape", [(1, 1), (1, 9), (9, 1), (2, 2), (3, 67), (67, 3), (5, 64), (4, 65)])
@pytest.mark.parametrize("model", [U, E, HST])
def test_forward_edge_shapes(model, shape):
    note("edge shape", NAMES[model], shape)
    H, W = shape
    p = workloads.random_params(model, 17, H, W, nbins=3, width=0.3)
    pt = dev(p, torch.float64)
    pmin, pmax = gpu_forward(pt, model, 3 if model == HST else 0)
    rmin, rmax = oracle.forward(model, p)
    assert_close(host(pmin), rmin, 1e-12, "P_min")
    assert_close(host(pmax), rmax, 1e-12, "P_max")


def test_golden_fixtures_fp64():
    """The fixtures under tests/golden: the Sec. 4.1.1 example (exact
    rational) and the oracle's small fields, through the FP64 kernels."""
    from fractions import Fraction
    from conftest import golden_small_fields, read_golden
    note("golden fixtures")
    g = read_golden("paper_1d_ordering.txt")
    grid = np.array([[[float(v) for v in g["lo"][0].split()]], [[float(v) for v in g["hi"][0].split()]]])
    pmin, pmax = gpu_forward(dev(grid, torch.float64), U)
    k = int(g["vertex"][0])
    assert abs(host(pmin)[0, k] - float(Fraction(g["p_min"][0]))) <= 1e-15
    assert abs(host(pmax)[0, k] - float(Fraction(g["p_max"][0]))) <= 1e-15
    for name, model, H, W, nb, seed, width, rmin, rmax in golden_small_fields():
        p = workloads.random_params(model, seed, H, W, nbins=max(nb, 1), width=width)
        pmin, pmax = gpu_forward(dev(p, torch.float64), model, nb)
        assert_close(host(pmin), rmin, 1e-12, f"{name} P_min")
        assert_close(host(pmax), rmax, 1e-12, f"{name} P_max")


def test_forward_iid_exact():
    """All vertices identical: 1/5 inside, 1/4 on edges, 1/3 at corners."""
    note("iid exact")
    for model, par in [(U, (0.0, 1.0)), (E, (0.5, 0.25)), (HST, (0.0, 1.0, 0.2, 0.5, 0.3))]:
        p = np.broadcast_to(np.array(par)[:, None, None], (len(par), 9, 70)).copy()
        pmin, pmax = gpu_forward(dev(p, torch.float64), model, 3 if model == HST else 0)
        r = oracle.forward(model, p)
        assert_close(host(pmin), r[0], 1e-13, "P_min")
        assert_close(host(pmax), r[1], 1e-13, "P_max")


def test_forward_invalid_parameters_give_nan():
    note("invalid parameters")
    p = workloads.random_params(U, 1, 6, 6, width=0.1)
    p[:, 2, 3] = [0.5, 0.5]  # lo == hi
    pmin, pmax = gpu_forward(dev(p, torch.float32), U)
    a = host(pmin)
    bad = np.zeros((6, 6), bool)
    for dy, dx in [(0, 0), (0, 1), (-1, 0), (0, -1), (1, 0)]:
        bad[2 - dy, 3 - dx] = True  # stencils that contain the bad vertex
    assert np.all(np.isnan(a[bad])) and np.all(np.isfinite(a[~bad]))
    h = workloads.random_params(HST, 1, 6, 6, nbins=3, width=0.1)
    h[2, 1, 1] = -0.1  # negative mass
    pmin, _ = gpu_forward(dev(h, torch.float32), HST, 3)
    assert np.isnan(host(pmin)[1, 1])


def test_row_stride_larger_than_width():
    note("row stride")
    H, W, RS = 37, 50, 64
    p = workloads.random_params(E, 2, H, W, width=0.05)
    big = torch.zeros((2, H, RS), dtype=torch.float32, device="cuda")
    big[:, :, :W] = dev(p, torch.float32)
    view = big[:, :, :W]
    f = cp.Field(H, W, E, torch.float32, row_stride=RS)
    omin = torch.full((H, RS), -7.0, device="cuda")
    omax = torch.full((H, RS), -7.0, device="cuda")
    cp.forward(view, f, omin[:, :W], omax[:, :W])
    r = oracle.forward(E, host(view))
    assert_close(host(omin[:, :W]), r[0], 1e-6, "P_min")
    assert np.all(host(omin[:, W:]) == -7.0)


def test_forward_is_deterministic():
    note("determinism")
    params, _ = fitted_params(HST, 9, 96, 130)
    a = host(gpu_forward(params, HST, 10)[0])
    b = host(gpu_forward(params, HST, 10)[0])
    assert np.array_equal(a, b)


# ----------------------------------------------------------------------------
# fit
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("model", [U, E, HST])
def test_fit_parity(model):
    note("fit", NAMES[model])
    H, W = 97, 131
    mem = workloads.mixture_ensemble(4, H, W) if model == HST else workloads.smooth_ensemble(4, H, W)
    mem[:, 3, 5] = mem[0, 3, 5]  # a degenerate vertex
    got = host(cp.fit(dev(mem, torch.float32), model, nbins=10 if model == HST else 0))
    ref = oracle.fit(model, mem.astype(np.float64), nbins=10 if model == HST else 0, single=True)
    if model == U:
        assert np.array_equal(got, ref)
    elif model == E:
        np.testing.assert_allclose(got, ref.astype(np.float32), rtol=2.5e-7, atol=0)
    else:
        assert np.array_equal(got[:2], ref[:2])
        # masses: identical bin decisions, count/M rounded once to FP32
        np.testing.assert_allclose(got[2:], ref[2:].astype(np.float32), rtol=0, atol=6e-8)


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
@pytest.mark.parametrize("model", [U, E])
def test_fit_vector_loads_equal_scalar_loads(model, dtype):
    """Width a multiple of 4 (FP32) / 2 (FP64): the fit reads 16-byte vectors;
    one more column: 4-byte (8-byte) loads.  The shared columns must agree bit
    for bit, also for degenerate and NaN members."""
    note("fit vector vs scalar", NAMES[model], dtype)
    H, W = 37, 128
    mem = workloads.smooth_ensemble(9, H, W + 1)
    mem[:, 3, 5] = mem[0, 3, 5]
    mem[4, 6, 7] = np.nan
    mem[0, 8, 9] = np.nan
    vec = host(cp.fit(dev(mem[:, :, :W], dtype), model))
    sca = host(cp.fit(dev(mem, dtype), model))[:, :, :W]
    assert np.array_equal(vec, sca, equal_nan=True)


def test_fit_fp64_and_many_members():
    note("fit fp64 / 40 members")
    mem = np.random.default_rng(3).normal(size=(40, 33, 70))
    for model in (U, E, HST):
        got = host(cp.fit(dev(mem, torch.float64), model, nbins=6 if model == HST else 0))
        ref = oracle.fit(model, mem, nbins=6 if model == HST else 0, single=False)
        # 40-term FP64 sums in different orders: rounding ~ M * 2^-53 * max|x|
        np.testing.assert_allclose(got, ref, rtol=1e-12, atol=2e-14)


# ----------------------------------------------------------------------------
# adjoint
# ----------------------------------------------------------------------------
def grad_tol(ref, S, dtype):
    if dtype == torch.float32:
        return 1e-5 * (1 + np.abs(ref)) + 5e-7 * S
    return 1e-10 * (1 + np.abs(ref)) + 1e-13 * S


def assert_grad(g, ref, S, dtype, what="grad"):
    d = np.abs(g - ref)
    tol = grad_tol(ref, S, dtype)
    i = int(np.argmax(d / tol))
    report(what, f"max |diff| {d.max():.3e}, worst |diff|/tolerance {d.flat[i] / tol.flat[i]:.3g} ({d.size} values)")
    assert np.all(d <= tol), f"{what}: worst |d|/tol {d.flat[i] / tol.flat[i]:.3g} (|d| {d.flat[i]:.3e}, g {ref.flat[i]:.4g}, S {S.flat[i]:.3g})"


@pytest.mark.parametrize("model", [U, E, HST])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_backward_parity(model, dtype):
    H, W = (45, 67) if model == HST else (73, 101)
    note("backward", NAMES[model], dtype, (H, W))
    nb = 5
    p = workloads.random_params(model, 40 + model, H, W, nbins=nb, width=0.06)
    pt = dev(p, dtype)
    gmin, gmax = workloads.upstream(1, H, W, np.float64)
    f = cp.field_of(pt, model, nb if model == HST else 0)
    g = host(cp.backward(pt, dev(gmin, dtype), dev(gmax, dtype), f))
    args = (model, host(pt), host(dev(gmin, dtype)), host(dev(gmax, dtype)))
    assert_grad(g, oracle.grad(*args), oracle.grad(*args, absolute=True), dtype)


@pytest.mark.parametrize("model", [U, E, HST])
def test_backward_fitted_fields(model):
    H, W = (40, 44) if model == HST else (96, 70)
    note("backward fitted", NAMES[model], (H, W))
    params, _ = fitted_params(model, 6, H, W)
    gmin, gmax = workloads.upstream(2, H, W)
    f = cp.field_of(params, model, 10 if model == HST else 0)
    g = host(cp.backward(params, dev(gmin, torch.float32), dev(gmax, torch.float32), f))
    args = (model, host(params), gmin.astype(np.float64), gmax.astype(np.float64))
    assert_grad(g, oracle.grad(*args), oracle.grad(*args, absolute=True), torch.float32)


def test_histogram_adjoint_finite_differences_on_crop():
    """The histogram workload's gradient check: on a 32x32 crop (seeded
    offset) of the fitted 2048^2, 10-bin mixture field, the FP64 adjoint with
    respect to the bin masses equals central differences of the FP64 forward
    of L = sum g_min P_min + g_max P_max.  P is linear in each single mass
    (masses are free variables), so the differences are exact up to
    rounding; no oracle involved."""
    note("histogram adjoint vs finite differences, 32x32 crop")
    S, C, nb = 2048, 32, 10
    mem = dev(workloads.mixture_ensemble(0, S, S), torch.float32)
    full = cp.fit(mem, HST, nbins=nb)
    del mem
    rng = np.random.default_rng(17)
    y0, x0 = (int(v) for v in rng.integers(0, S - C, 2))
    par = full[:, y0:y0 + C, x0:x0 + C].to(torch.float64).contiguous()
    del full
    f = cp.field_of(par, HST, nb)
    g1, g2 = (dev(g, torch.float64) for g in workloads.upstream(6, C, C, np.float64))
    grad = host(cp.backward(par, g1, g2, f))

    a0, b0 = cp.forward(par, f)
    h = 1e-3  # one-sided: L is linear in the mass, and a zero mass stays valid
    for _ in range(150):
        y, x, j = int(rng.integers(C)), int(rng.integers(C)), int(rng.integers(nb))
        pp = par.clone()
        pp[2 + j, y, x] += h
        a, b = cp.forward(pp, f)
        # only the five stencils holding (y, x) change: sum the changes alone
        fd = float(((a - a0) * g1 + (b - b0) * g2).sum()) / h
        assert abs(grad[2 + j, y, x] - fd) <= 1e-9 * (1 + abs(fd)), (y, x, j, grad[2 + j, y, x], fd)
    assert np.all(grad[:2] == 0)


def test_epanechnikov_adjoint_finite_differences_on_crop():
    """The quoted workload's gradient, checked without the oracle: on a 32x32
    crop (seeded offset) of the fitted 2048^2 field, the FP64 adjoint with
    respect to centre and half-width against central differences of the FP64
    forward of L = sum g_min P_min + g_max P_max (step 1e-4 of the width;
    the differences of the five stencils that change are summed alone)."""
    note("Epanechnikov adjoint vs finite differences, 32x32 crop")
    S, C = 2048, 32
    mem = dev(workloads.smooth_ensemble(0, S, S), torch.float32)
    full = cp.fit(mem, E)
    del mem
    rng = np.random.default_rng(19)
    y0, x0 = (int(v) for v in rng.integers(0, S - C, 2))
    par = full[:, y0:y0 + C, x0:x0 + C].to(torch.float64).contiguous()
    del full
    f = cp.field_of(par, E)
    g1, g2 = (dev(g, torch.float64) for g in workloads.upstream(7, C, C, np.float64))
    grad = host(cp.backward(par, g1, g2, f))
    for _ in range(120):
        y, x, q = int(rng.integers(C)), int(rng.integers(C)), int(rng.integers(2))
        h = 1e-4 * float(par[1, y, x])
        pp, pm = par.clone(), par.clone()
        pp[q, y, x] += h
        pm[q, y, x] -= h
        (ap, bp), (am, bm) = cp.forward(pp, f), cp.forward(pm, f)
        fd = float(((ap - am) * g1 + (bp - bm) * g2).sum()) / (2 * h)
        assert abs(grad[q, y, x] - fd) <= 1e-6 * (1 + abs(fd)), (y, x, q, grad[q, y, x], fd)


@pytest.mark.parametrize("model", ["uniform", "epanechnikov", "gaussian"])
def test_autograd_function_matches_backward(model):
    """torch.autograd through CPProb gives the adjoint entry point's bits;
    a loss on P_min alone passes zeros for the P_max gradient."""
    note("autograd", model)
    H, W = 40, 50
    if model == "gaussian":
        rng = np.random.default_rng(8)
        base = rng.normal(0, 0.05, (H, W))
        raw = np.stack([base, rng.uniform(0.02, 0.06, (H, W))])
    else:
        raw = workloads.random_params(U if model == "uniform" else E, 8, H, W, width=0.05)
    p = dev(raw, torch.float32).requires_grad_(True)
    pmin, pmax = cp.critical_point_probability(p, model)
    gmin, gmax = workloads.upstream(3, H, W)
    (pmin * dev(gmin, torch.float32) + pmax * dev(gmax, torch.float32)).sum().backward()
    f = cp.field_of(p.detach(), model)
    g = cp.backward(p.detach(), dev(gmin, torch.float32), dev(gmax, torch.float32), f)
    assert torch.equal(p.grad, g)
    q = dev(raw, torch.float32).requires_grad_(True)
    qmin, _ = cp.critical_point_probability(q, model)
    (qmin * dev(gmin, torch.float32)).sum().backward()
    g0 = cp.backward(q.detach(), dev(gmin, torch.float32), torch.zeros_like(qmin), f)
    assert torch.equal(q.grad, g0)


def test_adjoint_buffers_on_two_streams():
    """The histogram and multivariate Gaussian adjoints pass partials through
    a library buffer; issued on two streams at once they give the same bits
    as one after the other on the current stream (one buffer per stream)."""
    note("adjoint on two streams")
    cases = []
    for i, (H, W) in enumerate(((61, 83), (47, 59))):
        p = dev(workloads.random_params(HST, 71 + i, H, W, nbins=6, width=0.06), torch.float32)
        cases.append((p, cp.field_of(p, HST, 6), H, W))
    for i, (H, W) in enumerate(((23, 31), (19, 27))):
        p, _ = mvg_setup(H, W, 11 + i)
        cases.append((p, cp.Field(H, W, MVG, torch.float32, nsamples=128, seed=5 + i, field_id=i), H, W))
    ups = []
    for i, (p, f, H, W) in enumerate(cases):
        gmin, gmax = workloads.upstream(20 + i, H, W)
        ups.append((dev(gmin, torch.float32), dev(gmax, torch.float32)))
    refs = [cp.backward(p, *u, f) for (p, f, _, _), u in zip(cases, ups)]
    torch.cuda.synchronize()
    streams = [torch.cuda.Stream(), torch.cuda.Stream()]
    for rep in range(3):
        outs = []
        for i, ((p, f, _, _), u) in enumerate(zip(cases, ups)):
            with torch.cuda.stream(streams[i % 2]):
                outs.append(cp.backward(p, *u, f))
        torch.cuda.synchronize()
        for i, (o, r) in enumerate(zip(outs, refs)):
            assert torch.equal(o, r), (rep, i)


# ----------------------------------------------------------------------------
# full-size workloads, sampled vertices
# ----------------------------------------------------------------------------
def sample_idx(H, W, n, seed):
    rng = np.random.default_rng(seed)
    idx = set(rng.integers(0, H * W, n).tolist())
    for y, x in [(0, 0), (0, W - 1), (H - 1, 0), (H - 1, W - 1), (0, W // 2), (H // 2, 0), (H - 1, W // 3)]:
        idx.add(y * W + x)
    return np.array(sorted(idx), dtype=np.int64)


@pytest.mark.parametrize("model", [U, E])
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_tall_tiles_ragged(model, dtype):
    """A grid large enough for the 64 x 16 forward and classification tiles
    (1030 x 2113: neither side a multiple of the tile): sampled vertices plus
    every vertex of the last row and column against the oracle, and the
    classification's P_min / P_max equal to the forward's bit for bit."""
    H, W = 1030, 2113
    note("tall tiles ragged", NAMES[model], dtype, (H, W))
    pt = dev(workloads.random_params(model, 90 + model, H, W, width=0.05), dtype)
    f = cp.field_of(pt, model)
    pmin, pmax = cp.forward(pt, f)
    out = cp.classify(pt, f, terms=True)
    assert torch.equal(out["min"], pmin) and torch.equal(out["max"], pmax)
    idx = np.union1d(sample_idx(H, W, 1500, 7),
                     np.concatenate([(H - 1) * W + np.arange(W), np.arange(H) * W + W - 1]))
    ph = host(pt)
    tol = 1e-6 if dtype == torch.float32 else 1e-12
    rmin, rmax = oracle.forward_at(model, ph, idx)
    assert_close(host(pmin).ravel()[idx], rmin, tol, "P_min")
    assert_close(host(pmax).ravel()[idx], rmax, tol, "P_max")
    t1, t2 = oracle.saddle_at(model, ph, idx)
    assert_close(host(out["terms"][0]).ravel()[idx], t1, tol, "t1")
    assert_close(host(out["terms"][1]).ravel()[idx], t2, tol, "t2")


@pytest.mark.parametrize("model,n", [(E, 2048), (HST, 2048), (U, 2048)])
def test_full_size_2048_sampled(model, n):
    """2048^2, 20 members: the benchmark's launch configuration; every output
    plane compared at sampled vertices (borders and corners included)."""
    note("full size 2048^2", NAMES[model])
    H = W = 2048
    params, mem = fitted_params(model, 0, H, W)
    f = cp.field_of(params, model, 10 if model == HST else 0)
    pmin, pmax = cp.forward(params, f)
    gmin, gmax = workloads.upstream(0, H, W)
    grad = cp.backward(params, dev(gmin, torch.float32), dev(gmax, torch.float32), f)
    ph = host(params)
    idx = sample_idx(H, W, n, 1 + model)
    rmin, rmax = oracle.forward_at(model, ph, idx)
    assert_close(host(pmin).ravel()[idx], rmin, 1e-6, "P_min")
    assert_close(host(pmax).ravel()[idx], rmax, 1e-6, "P_max")
    gi = idx[: max(64, n // 16)]
    args = (model, ph, gmin.astype(np.float64), gmax.astype(np.float64), gi)
    g = host(grad).reshape(ph.shape[0], -1)[:, gi].T
    assert_grad(g, oracle.grad_at(*args), oracle.grad_at(*args, absolute=True), torch.float32)
    # the fit itself, at the same vertices
    rfit = oracle.fit(model, mem[:, :64, :].astype(np.float64), nbins=10 if model == HST else 0, single=True)
    gfit = ph[:, :64, :]
    if model == E:
        np.testing.assert_allclose(gfit, rfit.astype(np.float32), rtol=2.5e-7, atol=0)
    else:
        np.testing.assert_allclose(gfit, rfit.astype(np.float32), rtol=0, atol=6e-8)


# ----------------------------------------------------------------------------
# multivariate Gaussian
# ----------------------------------------------------------------------------
def test_philox_bit_identical():
    note("philox")
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2 ** 32, (4096, 4), dtype=np.uint64).astype(np.uint32)
    seed = 0x0123456789ABCDEF
    out = cp.philox(torch.as_tensor(ctr.view(np.int32), device="cuda"), seed)
    got = out.cpu().numpy().view(np.uint32)
    key = [seed & 0xFFFFFFFF, seed >> 32]
    for i in range(0, 4096, 97):
        assert np.array_equal(got[i], oracle.philox4x32_10(ctr[i], key)), i


def assert_mvg_grad(g, ref, slack, what):
    """FP32 samples against FP64 samples: every component within 2e-5 of the
    vertex's largest gradient component (plus 2e-5 absolute), plus the
    oracle's near-tie slack -- the summed magnitude of the sample terms whose
    extreme neighbour lies within rounding of another neighbour, which a
    lower-precision evaluation may route to the other one (0 where no such
    sample occurs).  No vertex is exempt."""
    scale = 1 + np.abs(ref).max(axis=1, keepdims=True)
    d = np.abs(g - ref)
    over = d - (2e-5 * scale + slack)
    i, k = np.unravel_index(int(np.argmax(over)), over.shape)
    r = d / (2e-5 * scale + slack)
    report(what, f"max |diff| {d.max():.3e}, worst |diff|/tolerance {r.max():.3g} ({d.size} values)")
    assert np.all(over <= 0), (f"{what}: vertex {i} component {k}: got {g[i, k]}, ref {ref[i, k]}, "
                               f"slack {slack[i, k]}, vertices with slack {int(np.count_nonzero(slack.any(axis=1)))}")


def mvg_setup(H, W, seed):
    mem = workloads.correlated_ensemble(seed, H, W)
    params = cp.fit(dev(mem, torch.float32), "mvg")
    return params, mem


def test_mvg_fit_parity():
    note("mvg fit")
    params, mem = mvg_setup(37, 53, 1)
    ref = oracle.mvg_fit(mem.astype(np.float64))
    np.testing.assert_allclose(host(params), ref, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("H,W,ns", [(37, 53, 512), (1024, 1024, 4096)])
def test_mvg_forward_parity(H, W, ns):
    note("mvg forward", H, W, ns)
    params, _ = mvg_setup(H, W, 2)
    seed, fid = 1234, 7
    ph = host(params)
    idx = np.arange(H * W) if H * W < 4000 else sample_idx(H, W, 96, 5)
    ref, amb = oracle.mvg_forward_at(ph, idx, ns, seed, fid)
    for est, cols in ((L.CP_MC_CONDITIONAL, (2, 3)), (L.CP_MC_HIT, (0, 1))):
        f = cp.Field(H, W, MVG, torch.float32, nsamples=ns, seed=seed, field_id=fid, estimator=est)
        pmin, pmax = cp.forward(params, f)
        gmin = host(pmin).ravel()[idx]
        gmax = host(pmax).ravel()[idx]
        if est == L.CP_MC_CONDITIONAL:
            assert_close(gmin, ref[:, 2], 1e-6, "conditional P_min")
            assert_close(gmax, ref[:, 3], 1e-6, "conditional P_max")
        else:
            assert np.all(np.abs(gmin * ns - ref[:, 0] * ns) <= amb[:, 0] + 1e-6)
            assert np.all(np.abs(gmax * ns - ref[:, 1] * ns) <= amb[:, 1] + 1e-6)


def test_mvg_backward_parity():
    note("mvg backward")
    H, W, ns = 29, 41, 256
    params, _ = mvg_setup(H, W, 3)
    gmin, gmax = workloads.upstream(5, H, W)
    f = cp.Field(H, W, MVG, torch.float32, nsamples=ns, seed=99, field_id=2)
    g = host(cp.backward(params, dev(gmin, torch.float32), dev(gmax, torch.float32), f))
    idx = np.arange(H * W)
    ref, slack = oracle.mvg_grad_at(host(params), gmin.astype(np.float64), gmax.astype(np.float64), idx, ns, 99,
                                    2, slack=True)
    assert_mvg_grad(g.reshape(16, -1).T, ref, slack, "mvg gradient 29x41")


def test_mvg_diagonal_agrees_with_independent_gaussian():
    """Two device paths that share no code: with a diagonal stencil covariance
    the Monte Carlo model is the independent Gaussian, so its conditional
    estimate (4096 Philox samples) must agree with the deterministic
    quadrature of the independent model within 5 binomial standard errors at
    every vertex (the conditional estimator's spread is below that)."""
    note("mvg diagonal vs independent gaussian")
    H, W, ns = 48, 56, 4096
    rng = np.random.default_rng(23)
    mu = rng.normal(0, 0.03, (H, W))
    sg = rng.uniform(0.01, 0.04, (H, W))
    gp = dev(np.stack([mu, sg]), torch.float32)
    ref = host(cp.forward(gp, cp.field_of(gp, "gaussian"))[0]).astype(np.float64)
    mp = np.zeros((16, H, W))
    mp[0] = gp[0].double().cpu().numpy()
    sgf = gp[1].double().cpu().numpy()
    diag = [1, 3, 6, 10, 15]  # packed positions of L00, L11, L22, L33, L44
    for i, (dy, dx) in enumerate(((0, 1), (-1, 0), (0, -1), (1, 0), (0, 0))):
        sh = np.ones((H, W))
        ys, xs = slice(max(0, -dy), H - max(0, dy)), slice(max(0, -dx), W - max(0, dx))
        yd, xd = slice(max(0, dy), H - max(0, -dy)), slice(max(0, dx), W - max(0, -dx))
        sh[ys, xs] = sgf[yd, xd]
        mp[diag[i]] = sh
    f = cp.Field(H, W, MVG, torch.float32, nsamples=ns, seed=41, field_id=3, estimator=L.CP_MC_CONDITIONAL)
    est = host(cp.forward(dev(mp, torch.float64), f)[0]).astype(np.float64)
    se = np.sqrt(np.clip(ref * (1 - ref), 0, None) / ns)
    assert np.all(np.abs(est - ref) <= 5 * se + 1e-6), float(np.max(np.abs(est - ref) - 5 * se))


def test_mvg_backward_full_size_sampled():
    """1024^2 x 4096 samples (the benchmark's Monte Carlo workload): the
    gathered gradient at sampled vertices, corners and edges included."""
    note("mvg backward full size")
    H, W, ns = 1024, 1024, 4096
    params, _ = mvg_setup(H, W, 2)
    gmin, gmax = workloads.upstream(6, H, W)
    f = cp.Field(H, W, MVG, torch.float32, nsamples=ns, seed=4321, field_id=3)
    g = host(cp.backward(params, dev(gmin, torch.float32), dev(gmax, torch.float32), f)).reshape(16, -1).T
    idx = sample_idx(H, W, 48, 8)
    ref, slack = oracle.mvg_grad_at(host(params), gmin.astype(np.float64), gmax.astype(np.float64), idx, ns, 4321,
                                    3, slack=True)
    assert_mvg_grad(g[idx], ref, slack, "mvg gradient 1024^2 sampled")


# ----------------------------------------------------------------------------
# batched persistent launch
# ----------------------------------------------------------------------------
def batched_fields(seed, n=9, lo=4.0, hi=7.5, dtype=torch.float32):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        H = int(round(2 ** rng.uniform(lo, hi)))
        W = int(round(2 ** rng.uniform(lo, hi)))
        model = i % 3
        p = workloads.random_params(model, seed * 100 + i, H, W, nbins=10, width=0.05)
        out.append((cp.field_of(dev(p, dtype), model, 10 if model == HST else 0), dev(p, dtype)))
    return out


@pytest.mark.parametrize("graph", [False, True])
def test_batched_forward_equals_per_field(graph):
    note("batched forward graph", graph)
    fl = batched_fields(1)
    fields = [f for f, _ in fl]
    params = [p for _, p in fl]
    pmin = [torch.empty((f.height, f.width), device="cuda") for f in fields]
    pmax = [torch.empty((f.height, f.width), device="cuda") for f in fields]
    for rep in range(3):
        for t in pmin + pmax:
            t.fill_(-1.0)
        cp.batched(fields, params, pmin=pmin, pmax=pmax, graph=graph)
        torch.cuda.synchronize()
        for i, (f, p) in enumerate(fl):
            a, b = cp.forward(p, f)
            assert torch.equal(a, pmin[i]) and torch.equal(b, pmax[i]), (rep, i)


@pytest.mark.parametrize("graph", [False, True])
def test_batched_forward_backward(graph):
    note("batched fwd+bwd graph", graph)
    fl = batched_fields(2)
    fields = [f for f, _ in fl]
    params = [p for _, p in fl]
    pmin = [torch.empty((f.height, f.width), device="cuda") for f in fields]
    pmax = [torch.empty((f.height, f.width), device="cuda") for f in fields]
    gmin = [dev(workloads.upstream(i, f.height, f.width)[0], torch.float32) for i, f in enumerate(fields)]
    gmax = [dev(workloads.upstream(i, f.height, f.width)[1], torch.float32) for i, f in enumerate(fields)]
    grad = [torch.empty_like(p) for p in params]
    for rep in range(3 if graph else 1):
        for t in pmin + pmax + grad:
            t.fill_(-1.0)
        torch.cuda.synchronize()
        cp.batched(fields, params, pmin, pmax, gmin, gmax, grad, graph=graph)
        torch.cuda.synchronize()
        for i, (f, p) in enumerate(fl):
            a, b = cp.forward(p, f)
            g = cp.backward(p, gmin[i], gmax[i], f)
            assert_close(host(pmin[i]), host(a), 1e-6, f"P_min field {i}")
            assert_close(host(pmax[i]), host(b), 1e-6, f"P_max field {i}")
            assert torch.equal(g, grad[i]), (rep, i)
    # and the oracle on one field of each model: probabilities and gradients
    for i in range(3):
        f, p = fl[i]
        ph = host(p)
        r = oracle.forward(f.model, ph)
        assert_close(host(pmin[i]), r[0], 1e-6, f"oracle P_min field {i}")
        assert_close(host(pmax[i]), r[1], 1e-6, f"oracle P_max field {i}")
        args = (f.model, ph, host(gmin[i]), host(gmax[i]))
        assert_grad(host(grad[i]), oracle.grad(*args), oracle.grad(*args, absolute=True), torch.float32,
                    f"oracle gradient field {i} ({NAMES[f.model]})")


@pytest.mark.parametrize("graph", [False, True])
def test_batched_many_tiles_back_to_back(graph):
    """24 fields of 2^U[7,10] per side (tens of thousands of tiles, far more
    than resident blocks, so every block claims many tiles from the queue);
    four launches back to back without synchronising (each must start from
    the queue reset by the previous one), then forward and adjoint equal the
    per-field launches bit for bit."""
    note("batched many tiles graph", graph)
    fl = batched_fields(7, n=24, lo=7.0, hi=10.0)
    fields = [f for f, _ in fl]
    params = [p for _, p in fl]
    nt = sum((f.height + 3) // 4 * ((f.width + 63) // 64) for f in fields)
    assert nt > 10000, nt
    pmin = [torch.full((f.height, f.width), -1.0, device="cuda") for f in fields]
    pmax = [torch.full((f.height, f.width), -1.0, device="cuda") for f in fields]
    for _ in range(4):
        cp.batched(fields, params, pmin=pmin, pmax=pmax, graph=graph)
    torch.cuda.synchronize()
    for i, (f, p) in enumerate(fl):
        a, b = cp.forward(p, f)
        assert torch.equal(a, pmin[i]) and torch.equal(b, pmax[i]), i
    gmin = [dev(workloads.upstream(i, f.height, f.width)[0], torch.float32) for i, f in enumerate(fields)]
    gmax = [dev(workloads.upstream(i, f.height, f.width)[1], torch.float32) for i, f in enumerate(fields)]
    grad = [torch.full_like(p, -1.0) for p in params]
    for _ in range(3):
        cp.batched(fields, params, None, None, gmin, gmax, grad, graph=graph)
    torch.cuda.synchronize()
    for i, (f, p) in enumerate(fl):
        assert torch.equal(cp.backward(p, gmin[i], gmax[i], f), grad[i]), i


def test_batched_full_layout_tuned_graph():
    """The benchmark's 64-field layout (sides 2^U[7,11], 47 M vertices),
    autotuned and replayed as a graph, as the benchmark times it: forward
    only equals the per-field forward bit for bit; forward + adjoint gives
    the per-field gradients bit for bit and the probabilities within 1e-6."""
    note("batched full layout")
    fields, params = [], []
    for side, model, seed in workloads.batched_layout(0):
        p = dev(workloads.random_params(model, seed, side, side, nbins=10, width=0.05), torch.float32)
        fields.append(cp.field_of(p, model, 10 if model == HST else 0))
        params.append(p)
    assert sum(f.height * f.width for f in fields) > 40e6
    pmin = [torch.full((f.height, f.width), -1.0, device="cuda") for f in fields]
    pmax = [torch.full((f.height, f.width), -1.0, device="cuda") for f in fields]
    for _ in range(2):
        cp.batched(fields, params, pmin=pmin, pmax=pmax, graph=True, tune=True)
    torch.cuda.synchronize()
    for i, (f, p) in enumerate(zip(fields, params)):
        a, b = cp.forward(p, f)
        assert torch.equal(a, pmin[i]) and torch.equal(b, pmax[i]), i
    gmin = [dev(workloads.upstream(i, f.height, f.width)[0], torch.float32) for i, f in enumerate(fields)]
    gmax = [dev(workloads.upstream(i, f.height, f.width)[1], torch.float32) for i, f in enumerate(fields)]
    grad = [torch.full_like(p, -1.0) for p in params]
    for _ in range(2):
        cp.batched(fields, params, pmin, pmax, gmin, gmax, grad, graph=True, tune=True)
    torch.cuda.synchronize()
    for i, (f, p) in enumerate(zip(fields, params)):
        assert torch.equal(cp.backward(p, gmin[i], gmax[i], f), grad[i]), i
        a, b = cp.forward(p, f)
        assert torch.allclose(a, pmin[i], rtol=0, atol=1e-6) and torch.allclose(b, pmax[i], rtol=0, atol=1e-6), i


def test_batched_pointer_refresh():
    """A second call with the same shapes but new buffers writes the new ones."""
    note("batched pointer refresh")
    fl = batched_fields(3, n=4)
    fields = [f for f, _ in fl]
    params = [p for _, p in fl]
    for _ in range(2):
        pmin = [torch.full((f.height, f.width), -1.0, device="cuda") for f in fields]
        pmax = [torch.full((f.height, f.width), -1.0, device="cuda") for f in fields]
        cp.batched(fields, params, pmin=pmin, pmax=pmax, graph=True)
        torch.cuda.synchronize()
        for i, (f, p) in enumerate(fl):
            a, _ = cp.forward(p, f)
            assert torch.equal(a, pmin[i])


def test_batched_per_field_mode():
    note("batched per-field mode")
    fl = batched_fields(4, n=5)
    fields = [f for f, _ in fl]
    params = [p for _, p in fl]
    pmin = [torch.empty((f.height, f.width), device="cuda") for f in fields]
    pmax = [torch.empty((f.height, f.width), device="cuda") for f in fields]
    cp.batched(fields, params, pmin=pmin, pmax=pmax, per_field=True)
    torch.cuda.synchronize()
    for i, (f, p) in enumerate(fl):
        a, b = cp.forward(p, f)
        assert torch.equal(a, pmin[i]) and torch.equal(b, pmax[i])


# ----------------------------------------------------------------------------
# error-bound uniform model (Sec. 5.3, climate data)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64])
def test_fit_error_bound_bit_exact_and_forward(dtype):
    """240 x 960 (the climate grid's shape): the ends are bit-identical to the
    oracle's, and the probabilities of the resulting uniform field match."""
    note("error-bound fit", dtype)
    H, W = 240, 960
    d = workloads.smooth_ensemble(4, H, W)[0]
    eb = 1e-3 * float(d.max() - d.min())
    dt = dev(d, dtype)
    par = cp.fit_error_bound(dt, eb)
    ref = oracle.fit_error_bound(host(dt), eb, single=dtype == torch.float32)
    assert np.array_equal(host(par), ref)
    pmin, pmax = gpu_forward(par, U)
    rmin, rmax = oracle.forward(U, ref)
    tol = 1e-6 if dtype == torch.float32 else 1e-12
    assert_close(host(pmin), rmin, tol, "P_min")
    assert_close(host(pmax), rmax, tol, "P_max")


def test_fit_error_bound_rejects_bad_bound():
    d = dev(np.zeros((4, 4)), torch.float32)
    for eb in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(L.CPError) as ei:
            cp.fit_error_bound(d, eb)
        assert ei.value.status == L.CP_EDOMAIN
