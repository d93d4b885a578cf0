"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Nothing here compares the oracle with itself: every check uses an
independent route -- a closed form derived by hand from the definition
(Sec. 3 / Eq. 1 / Eq. 3), a library routine (scipy quadrature and scipy.stats
distributions, numpy statistics, rocRAND's Philox), brute-force Monte Carlo,
the paper's literal histogram sum (Eq. 5), the negation argument for maxima
(Sec. 4.1.2), symmetry, or exact linearity.
"""
from fractions import Fraction
import math
import os
import shutil
import subprocess

import numpy as np
import pytest
from scipy import integrate, stats

import exact_stencil
import oracle
import workloads
from conftest import golden_small_fields, read_golden

U, E, HST = oracle.UNIFORM, oracle.EPANECHNIKOV, oracle.HISTOGRAM

# stencil slots in a 3x3 grid around the centre (1, 1): v, e, n, w, s
POS = {"v": (1, 1), "e": (1, 2), "n": (0, 1), "w": (1, 0), "s": (2, 1)}


def stencil_grid(model, dists, nb=0):
    """3x3 parameter grid whose centre stencil holds the given distributions
    (dict name -> parameter tuple); corners get copies of v (unused)."""
    npar = oracle.n_param(model, nb)
    g = np.zeros((npar, 3, 3))
    for y in range(3):
        for x in range(3):
            g[:, y, x] = dists["v"]
    for k, (y, x) in POS.items():
        g[:, y, x] = dists[k]
    return g


def centre(model, grid):
    pmin, pmax = oracle.forward(model, grid)
    return pmin[1, 1], pmax[1, 1]


# ----------------------------------------------------------------------------
# exact values
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("model,par", [
    (U, (0.0, 1.0)), (U, (-3.0, 7.5)),
    (E, (0.0, 1.0)), (E, (0.3, 0.01)),
    (HST, (0.0, 1.0, 0.1, 0.2, 0.3, 0.4)), (HST, (-1.0, 2.0, 0.5, 0.0, 0.5)),
])
def test_iid_stencil_gives_one_over_count(model, par):
    """Identical independent distributions: by exchangeability each of the k
    stencil members is the strict minimum with probability 1/k (5 inside,
    4 on an edge, 3 at a corner)."""
    nb = len(par) - 2 if model == HST else 0
    g = np.broadcast_to(np.array(par)[:, None, None], (len(par), 4, 5)).copy()
    pmin, pmax = oracle.forward(model, g)
    expect = np.full((4, 5), 1 / 5)
    expect[0, :] = expect[-1, :] = expect[:, 0] = expect[:, -1] = 1 / 4
    for y in (0, 3):
        for x in (0, 4):
            expect[y, x] = 1 / 3
    np.testing.assert_allclose(pmin, expect, rtol=0, atol=1e-14)
    np.testing.assert_allclose(pmax, expect, rtol=0, atol=1e-14)


def test_single_vertex_grid():
    """No neighbours: the empty conjunction is certain."""
    for model, par in [(U, (0, 1)), (E, (0, 1)), (HST, (0, 1, 0.5, 0.5))]:
        pmin, pmax = oracle.forward(model, np.array(par, float)[:, None, None])
        assert pmin[0, 0] == pytest.approx(1.0, abs=1e-15) and pmax[0, 0] == pytest.approx(1.0, abs=1e-15)


@pytest.mark.parametrize("c", [0.0, 0.1, 0.25, 0.5, 0.9, 1.0, 1.5])
def test_shifted_uniform_closed_form(c):
    """v = U[0,1], four neighbours U[c, 1+c].  By hand from Eq. 3 with S
    the survival function of U[c, 1+c]:
      P_min = c + (1 - c^5)/5,  P_max = (1 - c)^5 / 5   (0 <= c <= 1),
    and P_min = 1, P_max = 0 once c >= 1."""
    d = {k: (c, 1 + c) for k in POS}
    d["v"] = (0.0, 1.0)
    pmin, pmax = centre(U, stencil_grid(U, d))
    cc = min(c, 1.0)
    assert pmin == pytest.approx(cc + (1 - cc ** 5) / 5, abs=1e-15)
    assert pmax == pytest.approx((1 - cc) ** 5 / 5, abs=1e-15)


def test_paper_one_dimensional_ordering():
    """The running example of Sec. 4.1.1 (ordering a2 < a1 < a3 < b2 < b1 <
    b3), instantiated with uniform densities; the exact values and their
    derivation are in tests/golden/paper_1d_ordering.txt."""
    g = read_golden("paper_1d_ordering.txt")
    assert g["model"] == ["uniform"]
    grid = np.array([[[float(v) for v in g["lo"][0].split()]], [[float(v) for v in g["hi"][0].split()]]])
    pmin, pmax = oracle.forward(U, grid)
    k = int(g["vertex"][0])
    assert pmin[0, k] == pytest.approx(float(Fraction(g["p_min"][0])), abs=1e-15)
    assert pmax[0, k] == pytest.approx(float(Fraction(g["p_max"][0])), abs=1e-15)


def test_oracle_reproduces_its_golden_fields():
    """Regression fixture (tests/golden/oracle_small_fields.txt, written by
    make_oracle_golden.py from the oracle): a change of the oracle's
    arithmetic shows here."""
    for name, model, H, W, nb, seed, width, rmin, rmax in golden_small_fields():
        p = workloads.random_params(model, seed, H, W, nbins=max(nb, 1), width=width)
        pmin, pmax = oracle.forward(model, p)
        np.testing.assert_allclose(pmin, rmin, rtol=0, atol=1e-15, err_msg=name)
        np.testing.assert_allclose(pmax, rmax, rtol=0, atol=1e-15, err_msg=name)


EXACT_2D = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "exact_2d_stencils.txt")


@pytest.mark.parametrize("case", exact_stencil.load_cases(EXACT_2D), ids=lambda c: c["name"])
def test_exact_2d_stencil_values_rederived(case):
    """The fixture's rationals equal an exact Fraction integration of the
    definitions (Eq. 3 and its mirror, densities of Sec. 4.3 / 4.4.1)."""
    pmin, pmax = exact_stencil.case_exact(case)
    assert pmin == case["p_min"] and pmax == case["p_max"], (pmin, pmax)


@pytest.mark.parametrize("case", exact_stencil.load_cases(EXACT_2D), ids=lambda c: c["name"])
def test_oracle_matches_exact_2d_stencils(case):
    """The oracle at 1e-15 on the exact 2-D stencils: tighter than the 1e-12
    the FP64 device path is held to against it (inputs such as 1/10 are
    rounded once to FP64, which moves P by ~1e-16)."""
    model, nb, grid = exact_stencil.case_grid(case)
    pmin, pmax = oracle.forward(model, grid)
    assert abs(pmin[1, 1] - float(case["p_min"])) <= 1e-15, pmin[1, 1]
    assert abs(pmax[1, 1] - float(case["p_max"])) <= 1e-15, pmax[1, 1]


@pytest.mark.parametrize("model", [U, E, HST])
def test_disjoint_supports(model):
    """b_v below every neighbour's support: certain minimum, impossible
    maximum; one neighbour entirely below a_v: P_min = 0 (Sec. 4.1.1,
    the b_min < a_1 case)."""
    def mk(lo, hi):
        if model == U:
            return (lo, hi)
        if model == E:
            return ((lo + hi) / 2, (hi - lo) / 2)
        return (lo, hi, 0.2, 0.5, 0.3)
    nb = 3 if model == HST else 0
    d = {k: mk(2.0, 3.0) for k in POS}
    d["v"] = mk(0.0, 1.0)
    assert centre(model, stencil_grid(model, d, nb)) == (pytest.approx(1.0, abs=1e-15), pytest.approx(0.0, abs=1e-15))
    d["n"] = mk(-2.0, -1.0)
    pmin, pmax = centre(model, stencil_grid(model, d, nb))
    assert pmin == 0.0 and pmax == 0.0
    d = {k: mk(-3.0, -2.0) for k in POS}
    d["v"] = mk(0.0, 1.0)
    assert centre(model, stencil_grid(model, d, nb)) == (pytest.approx(0.0, abs=1e-15), pytest.approx(1.0, abs=1e-15))


# ----------------------------------------------------------------------------
# library quadrature of the definition with scipy.stats distributions
# ----------------------------------------------------------------------------
def scipy_dist(model, par):
    if model == U:
        return stats.uniform(loc=par[0], scale=par[1] - par[0]), [par[0], par[1]]
    if model == E:  # Epanechnikov = Beta(2, 2) on [m - w, m + w]
        m, w = par
        return stats.beta(2, 2, loc=m - w, scale=2 * w), [m - w, m + w]
    lo, hi, *mass = par
    edges = np.linspace(lo, hi, len(mass) + 1)
    return stats.rv_histogram((np.asarray(mass), edges), density=False), list(edges)


def quad_min_max(model, dists):
    """P_min = int pdf_v prod sf_n, P_max = int pdf_v prod cdf_n (scipy)."""
    dv, pts = scipy_dist(model, dists["v"])
    nbr = []
    allpts = list(pts)
    for k in ("e", "n", "w", "s"):
        d, p = scipy_dist(model, dists[k])
        nbr.append(d)
        allpts += p
    lo, hi = pts[0], pts[-1]
    inner = sorted({p for p in allpts if lo < p < hi})
    fmin = lambda x: dv.pdf(x) * np.prod([d.sf(x) for d in nbr])
    fmax = lambda x: dv.pdf(x) * np.prod([d.cdf(x) for d in nbr])
    kw = dict(points=inner or None, limit=400, epsabs=1e-14, epsrel=1e-12)
    return integrate.quad(fmin, lo, hi, **kw)[0], integrate.quad(fmax, lo, hi, **kw)[0]


def random_stencil(model, rng, nb=4):
    d = {}
    for k in POS:
        c = rng.uniform(0, 1)
        w = rng.uniform(0.2, 0.8)
        if model == U:
            d[k] = (c - w, c + w)
        elif model == E:
            d[k] = (c, w)
        else:
            m = rng.dirichlet(np.ones(nb))
            d[k] = (c - w, c + w, *m)
    return d


@pytest.mark.parametrize("model", [U, E, HST])
def test_against_scipy_quadrature(model):
    rng = np.random.default_rng(42 + model)
    nb = 4
    for _ in range(12):
        d = random_stencil(model, rng, nb)
        got = centre(model, stencil_grid(model, d, nb if model == HST else 0))
        ref = quad_min_max(model, d)
        assert got[0] == pytest.approx(ref[0], abs=2e-10)
        assert got[1] == pytest.approx(ref[1], abs=2e-10)


# ----------------------------------------------------------------------------
# brute-force Monte Carlo
# ----------------------------------------------------------------------------
def sample(model, par, n, rng):
    if model == U:
        return rng.uniform(par[0], par[1], n)
    if model == E:
        return par[0] + par[1] * (2.0 * rng.beta(2.0, 2.0, n) - 1.0)
    lo, hi, *mass = par
    mass = np.asarray(mass)
    b = rng.choice(len(mass), size=n, p=mass / mass.sum())
    return lo + (b + rng.random(n)) * (hi - lo) / len(mass)


MIXED_STENCILS = {
    # (v, e, n, w, s)
    U: {"v": (0, 1), "e": (-0.5, 0.5), "n": (0.25, 1.25), "w": (0.5, 2.0), "s": (0.1, 0.9)},
    E: {"v": (0, 1), "e": (0.5, 1), "n": (-0.25, 0.75), "w": (1 / 3, 0.5), "s": (0.1, 2.0)},
}


@pytest.mark.parametrize("model", [U, E, HST])
def test_brute_force_monte_carlo(model):
    """4e6 joint samples of the five independent stencil values; the counted
    frequencies of 'v strictly below / above all neighbours' agree with the
    oracle within 4 binomial standard errors."""
    rng = np.random.default_rng(7 + model)
    nb = 3
    d = MIXED_STENCILS.get(model) or {
        "v": (0, 1, 0.5, 0.25, 0.25), "e": (-0.5, 0.5, 1 / 3, 1 / 3, 1 / 3),
        "n": (0.25, 1.25, 0.1, 0.6, 0.3), "w": (0.5, 2.0, 0.2, 0.3, 0.5), "s": (0.1, 0.9, 0.2, 0.2, 0.6)}
    pmin, pmax = centre(model, stencil_grid(model, d, nb if model == HST else 0))
    N, chunks = 1_000_000, 4
    cmin = cmax = 0
    for _ in range(chunks):
        xs = {k: sample(model, d[k], N, rng) for k in POS}
        nmin = np.minimum.reduce([xs[k] for k in "enws"])
        nmax = np.maximum.reduce([xs[k] for k in "enws"])
        cmin += int(np.count_nonzero(xs["v"] < nmin))
        cmax += int(np.count_nonzero(xs["v"] > nmax))
    n = N * chunks
    for p, c in ((pmin, cmin), (pmax, cmax)):
        se = math.sqrt(max(p * (1 - p), 1e-12) / n)
        assert abs(c / n - p) < 4 * se, (p, c / n, se)


def test_monte_carlo_on_grid():
    """Whole 16x16 grids (boundary stencils included), all three models,
    2e5 samples per vertex: every vertex within 4.5 standard errors."""
    rng = np.random.default_rng(3)
    n = 200_000
    for model in (U, E, HST):
        par = workloads.random_params(model, 11 + model, 16, 16, nbins=3, width=0.05)
        pmin, pmax = oracle.forward(model, par)
        H, W = 16, 16
        cmin = np.zeros((H, W)); cmax = np.zeros((H, W))
        for _ in range(2):
            xs = np.empty((H, W, n // 2))
            for y in range(H):
                for x in range(W):
                    xs[y, x] = sample(model, par[:, y, x], n // 2, rng)
            big = np.inf
            pad_lo = np.pad(xs, ((1, 1), (1, 1), (0, 0)), constant_values=big)
            pad_hi = np.pad(xs, ((1, 1), (1, 1), (0, 0)), constant_values=-big)
            nmin = np.minimum.reduce([pad_lo[1:-1, 2:], pad_lo[:-2, 1:-1], pad_lo[1:-1, :-2], pad_lo[2:, 1:-1]])
            nmax = np.maximum.reduce([pad_hi[1:-1, 2:], pad_hi[:-2, 1:-1], pad_hi[1:-1, :-2], pad_hi[2:, 1:-1]])
            cmin += (xs < nmin).sum(-1)
            cmax += (xs > nmax).sum(-1)
        for p, c in ((pmin, cmin / n), (pmax, cmax / n)):
            se = np.sqrt(np.maximum(p * (1 - p), 1e-10) / n)
            assert np.all(np.abs(c - p) < 4.5 * se + 1e-12), model


# ----------------------------------------------------------------------------
# structure: negation, histogram identities, Eq. 5
# ----------------------------------------------------------------------------
def negate(model, par):
    """Parameters of -X (Sec. 4.1.2: the maximum of X is the minimum of -X)."""
    if model == U:
        return np.stack([-par[1], -par[0]])
    if model == E:
        return np.stack([-par[0], par[1]])
    return np.concatenate([np.stack([-par[1], -par[0]]), par[:1:-1]])


@pytest.mark.parametrize("model", [U, E, HST])
def test_negation_identity(model):
    par = workloads.random_params(model, 5, 12, 9, nbins=4, width=0.04)
    pmin, pmax = oracle.forward(model, par)
    nmin, nmax = oracle.forward(model, negate(model, par))
    np.testing.assert_allclose(pmax, nmin, atol=1e-13, rtol=0)
    np.testing.assert_allclose(pmin, nmax, atol=1e-13, rtol=0)


@pytest.mark.parametrize("nb", [1, 4])
def test_equal_mass_histogram_is_uniform(nb):
    """A histogram with equal masses (or one bin) is the uniform density on
    its range (Sec. 4.4.1: a histogram is a mixture of uniform kernels)."""
    up = workloads.random_params(U, 9, 10, 11, width=0.05)
    hp = np.concatenate([up, np.full((nb,) + up.shape[1:], 1.0 / nb)])
    a = oracle.forward(U, up)
    b = oracle.forward(HST, hp)
    np.testing.assert_allclose(a[0], b[0], atol=1e-13, rtol=0)
    np.testing.assert_allclose(a[1], b[1], atol=1e-13, rtol=0)


@pytest.mark.parametrize("seed", [0, 1])
def test_histogram_equals_literal_eq5_sum(seed):
    """Eq. 5: P_min = sum over all h^5 choices of one uniform kernel per
    stencil member of (product of their masses) x P_min of those uniforms.
    The uniform probabilities come from the oracle's uniform model, which is
    pinned separately by the closed forms above."""
    rng = np.random.default_rng(100 + seed)
    nb = 3
    d = random_stencil(HST, rng, nb)
    pmin, pmax = centre(HST, stencil_grid(HST, d, nb))
    names = ["v", "e", "n", "w", "s"]
    kernels = {}
    for k in names:
        lo, hi, *m = d[k]
        edges = np.linspace(lo, hi, nb + 1)
        kernels[k] = [((edges[j], edges[j + 1]), m[j]) for j in range(nb)]
    smin = smax = 0.0
    import itertools
    for combo in itertools.product(range(nb), repeat=5):
        w = 1.0
        dd = {}
        for k, j in zip(names, combo):
            dd[k], mj = kernels[k][j]
            w *= mj
        a, b = centre(U, stencil_grid(U, dd))
        smin += w * a
        smax += w * b
    assert pmin == pytest.approx(smin, abs=1e-13)
    assert pmax == pytest.approx(smax, abs=1e-13)


def test_single_member_histogram_is_classical_classification():
    """One member per vertex: the fitted histogram is a spike of width
    2 eps |x| around the value, so P_min / P_max reduce to the deterministic
    strict local minimum / maximum (Sec. 3) wherever neighbours differ by more
    than the spike width."""
    rng = np.random.default_rng(5)
    vals = rng.random((1, 17, 13)).astype(np.float32).astype(np.float64)
    par = oracle.fit(HST, vals, nbins=4, single=True)
    pmin, pmax = oracle.forward(HST, par)
    v = vals[0]
    pad_lo = np.pad(v, 1, constant_values=np.inf)
    pad_hi = np.pad(v, 1, constant_values=-np.inf)
    nmin = np.minimum.reduce([pad_lo[1:-1, 2:], pad_lo[:-2, 1:-1], pad_lo[1:-1, :-2], pad_lo[2:, 1:-1]])
    nmax = np.maximum.reduce([pad_hi[1:-1, 2:], pad_hi[:-2, 1:-1], pad_hi[1:-1, :-2], pad_hi[2:, 1:-1]])
    np.testing.assert_array_equal(pmin, (v < nmin).astype(float))
    np.testing.assert_array_equal(pmax, (v > nmax).astype(float))


def test_probabilities_are_probabilities():
    par = workloads.random_params(E, 2, 20, 20, width=0.05)
    pmin, pmax = oracle.forward(E, par)
    assert np.all(pmin >= -1e-15) and np.all(pmax >= -1e-15)
    assert np.all(pmin + pmax <= 1 + 1e-13)


# ----------------------------------------------------------------------------
# gradients
# ----------------------------------------------------------------------------
def fd_stencil_jacobian(model, grid, h):
    """Central differences of the centre probabilities w.r.t. each parameter
    of each stencil member."""
    npar = grid.shape[0]
    jmin = np.zeros((5, npar)); jmax = np.zeros((5, npar))
    for s, k in enumerate(["v", "e", "n", "w", "s"]):
        y, x = POS[k]
        for q in range(npar):
            gp = grid.copy(); gm = grid.copy()
            gp[q, y, x] += h; gm[q, y, x] -= h
            a = centre(model, gp); b = centre(model, gm)
            jmin[s, q] = (a[0] - b[0]) / (2 * h)
            jmax[s, q] = (a[1] - b[1]) / (2 * h)
    return jmin, jmax


@pytest.mark.parametrize("model", [U, E, HST])
def test_jacobian_matches_finite_differences(model):
    rng = np.random.default_rng(21 + model)
    nb = 3
    for _ in range(6):
        d = random_stencil(model, rng, nb)
        g = stencil_grid(model, d, nb if model == HST else 0)
        jmin, jmax = oracle.jacobian_at(model, g, [4])
        fmin, fmax = fd_stencil_jacobian(model, g, 1e-6)
        if model == HST:  # range ends are not differentiated
            fmin[:, :2] = 0; fmax[:, :2] = 0
        np.testing.assert_allclose(jmin[0], fmin, atol=2e-6 * (1 + np.abs(fmin).max()), rtol=0)
        np.testing.assert_allclose(jmax[0], fmax, atol=2e-6 * (1 + np.abs(fmax).max()), rtol=0)


def test_histogram_masses_enter_multilinearly():
    """P is linear in each single mass (Eq. 5 is a multilinear form), so a
    finite step reproduces the derivative exactly."""
    rng = np.random.default_rng(8)
    nb = 4
    d = random_stencil(HST, rng, nb)
    g = stencil_grid(HST, d, nb)
    jmin, jmax = oracle.jacobian_at(HST, g, [4])
    for s, k in enumerate(["v", "e", "n", "w", "s"]):
        y, x = POS[k]
        for q in range(2, 2 + nb):
            step = 0.37
            gp = g.copy(); gp[q, y, x] += step
            a = centre(HST, gp); b = centre(HST, g)
            assert (a[0] - b[0]) / step == pytest.approx(jmin[0, s, q], abs=1e-12)
            assert (a[1] - b[1]) / step == pytest.approx(jmax[0, s, q], abs=1e-12)


def test_gradient_signs():
    """Raising the vertex centre lowers P_min and raises P_max; raising a
    neighbour centre does the opposite (Epanechnikov, random stencils)."""
    rng = np.random.default_rng(12)
    for _ in range(10):
        g = stencil_grid(E, random_stencil(E, rng))
        jmin, jmax = oracle.jacobian_at(E, g, [4])
        assert jmin[0, 0, 0] <= 1e-14 and jmax[0, 0, 0] >= -1e-14
        assert np.all(jmin[0, 1:, 0] >= -1e-14) and np.all(jmax[0, 1:, 0] <= 1e-14)


@pytest.mark.parametrize("model", [U, E, HST])
def test_adjoint_gather_matches_finite_differences(model):
    """grad[k][u] = d/dtheta_k(u) of sum_v g_min(v) P_min(v) + g_max(v) P_max(v),
    by central differences of whole-grid forwards (checks the gather over the
    adjoint stencil, boundary included)."""
    H, W, nb = 6, 7, 3
    par = workloads.random_params(model, 31, H, W, nbins=nb, width=0.06)
    gmin, gmax = workloads.upstream(4, H, W, np.float64)
    grad = oracle.grad(model, par, gmin, gmax)
    rng = np.random.default_rng(0)
    qs = range(2, 2 + nb) if model == HST else range(2)

    def loss(p):
        a, b = oracle.forward(model, p)
        return float((gmin * a).sum() + (gmax * b).sum())

    h = 1e-6
    for _ in range(12):
        y, x = int(rng.integers(H)), int(rng.integers(W))
        for q in qs:
            pp = par.copy(); pm = par.copy()
            pp[q, y, x] += h; pm[q, y, x] -= h
            fd = (loss(pp) - loss(pm)) / (2 * h)
            assert grad[q, y, x] == pytest.approx(fd, abs=1e-5 * (1 + abs(fd)))
    idx = np.array([0, W - 1, 3 * W + 2, H * W - 1])
    np.testing.assert_allclose(oracle.grad_at(model, par, gmin, gmax, idx),
                               grad.reshape(grad.shape[0], -1)[:, idx].T, atol=1e-15, rtol=0)


# ----------------------------------------------------------------------------
# fitting rules
# ----------------------------------------------------------------------------
def test_fit_against_numpy():
    members = workloads.smooth_ensemble(3, 9, 11, M=20).astype(np.float64)
    u = oracle.fit(U, members, single=True)
    np.testing.assert_array_equal(u[0], members.min(0))
    np.testing.assert_array_equal(u[1], members.max(0))
    e = oracle.fit(E, members, single=True)
    np.testing.assert_allclose(e[0], members.mean(0), rtol=1e-14)
    np.testing.assert_allclose(e[1], 1.06 * members.std(0, ddof=1) * 20 ** -0.2, rtol=1e-12)
    h = oracle.fit(HST, members, nbins=10, single=False)
    for y in range(9):
        for x in range(11):
            cnt, _ = np.histogram(members[:, y, x], bins=10, range=(members[:, y, x].min(), members[:, y, x].max()))
            np.testing.assert_allclose(h[2:, y, x], cnt / 20.0, rtol=0, atol=1e-15)


def test_fit_degenerate_range_is_widened():
    members = np.full((5, 2, 2), 0.5)
    u = oracle.fit(U, members, single=False, eps=2.0 ** -30)
    assert np.all(u[0] == 0.5 - 2.0 ** -30) and np.all(u[1] == 0.5 + 2.0 ** -30)
    e = oracle.fit(E, members, single=False, eps=2.0 ** -30)
    assert np.all(e[0] == 0.5) and np.all(e[1] == 2.0 ** -30)


def test_fit_histogram_bins_in_fp32():
    """FP32 fields take the bin decision in FP32; check against numpy's
    float32 arithmetic of the same expression."""
    members = workloads.mixture_ensemble(1, 8, 8, M=20).astype(np.float64)
    h = oracle.fit(HST, members, nbins=10, single=True)
    m32 = members.astype(np.float32)
    lo = m32.min(0); hi = m32.max(0)
    t = ((m32 - lo) / (hi - lo)) * np.float32(10)
    j = np.minimum(t.astype(np.int64), 9)
    for b in range(10):
        np.testing.assert_allclose(h[2 + b], (j == b).sum(0) / 20.0, rtol=0, atol=1e-15)


# ----------------------------------------------------------------------------
# multivariate Gaussian (Monte Carlo)
# ----------------------------------------------------------------------------
@pytest.fixture(scope="module")
def rocrand_philox(tmp_path_factory):
    src = os.path.join(os.path.dirname(__file__), "helpers", "rocrand_philox_ref.cpp")
    if shutil.which("g++") is None or not os.path.exists("/opt/rocm/include/rocrand"):
        pytest.skip("rocRAND headers or g++ not available")
    exe = str(tmp_path_factory.mktemp("philox") / "ref")
    r = subprocess.run(["g++", "-O1", "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", src, "-o", exe],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("could not build the rocRAND reference: " + r.stderr[-300:])
    return exe


def test_philox_matches_rocrand(rocrand_philox):
    rng = np.random.default_rng(2024)
    cases = [([0, 0, 0, 0], [0, 0])]
    for _ in range(60):
        c = [int(v) for v in rng.integers(0, 2 ** 32, 4)]
        c[1] %= 2 ** 30
        cases.append((c, [int(v) for v in rng.integers(0, 2 ** 32, 2)]))
    for c, k in cases:
        out = subprocess.run([rocrand_philox] + [str(v) for v in c + k], capture_output=True, text=True,
                             check=True).stdout.split()
        assert [int(v) for v in out] == [int(v) for v in oracle.philox4x32_10(c, k)], (c, k)


def mvg_grid(mu, L):
    """3x3 grid: mean plane mu (3x3), centre factor L (5x5 over e, n, w, s, v)."""
    par = np.zeros((16, 3, 3))
    par[0] = mu
    eye = np.eye(5)
    for y in range(3):
        for x in range(3):
            LL = L if (y, x) == (1, 1) else eye
            k = 0
            for r in range(5):
                for c in range(r + 1):
                    par[1 + k, y, x] = LL[r, c]
                    k += 1
    return par


def mu_plane(vals):
    mu = np.zeros((3, 3))
    for k, v in zip(["e", "n", "w", "s", "v"], vals):
        mu[POS[k]] = v
    return mu


def test_mvg_diagonal_covariance_matches_quadrature():
    """Diagonal covariance = independent Gaussians: P_min = int phi_v prod sf_n
    by library quadrature; both estimators within 4 standard errors."""
    means = [0.1, -0.2, 0.3, 0.05, 0.0]  # e, n, w, s, v
    sig = [0.3, 0.5, 0.4, 0.2, 0.35]
    par = mvg_grid(mu_plane(means), np.diag(sig))
    ns = 1 << 15
    est, _ = oracle.mvg_forward_at(par, [4], ns, seed=12345)
    dv = stats.norm(means[4], sig[4])
    nb = [stats.norm(m, s) for m, s in zip(means[:4], sig[:4])]
    pmin = integrate.quad(lambda x: dv.pdf(x) * np.prod([d.sf(x) for d in nb]), -np.inf, np.inf, epsabs=1e-13)[0]
    pmax = integrate.quad(lambda x: dv.pdf(x) * np.prod([d.cdf(x) for d in nb]), -np.inf, np.inf, epsabs=1e-13)[0]
    for got, p in ((est[0, 0], pmin), (est[0, 2], pmin), (est[0, 1], pmax), (est[0, 3], pmax)):
        assert abs(got - p) < 4 * math.sqrt(p * (1 - p) / ns), (got, p)


def test_mvg_exchangeable_is_one_fifth():
    rho, s2 = 0.6, 0.04
    C = s2 * ((1 - rho) * np.eye(5) + rho * np.ones((5, 5)))
    par = mvg_grid(np.zeros((3, 3)), np.linalg.cholesky(C))
    ns = 1 << 15
    est, _ = oracle.mvg_forward_at(par, [4], ns, seed=99)
    se = math.sqrt(0.2 * 0.8 / ns)
    assert np.all(np.abs(est[0] - 0.2) < 4 * se)


def test_mvg_corner_vertex_bivariate_orthant():
    """Corner vertex (0,0): neighbours e and s only.  With zero mean
    differences Pr(X_v < X_e, X_v < X_s) = 1/4 + asin(rho_D)/(2 pi), rho_D the
    correlation of the two differences; with means, scipy's bivariate normal
    CDF."""
    rng = np.random.default_rng(3)
    A = rng.normal(size=(3, 3))
    C3 = A @ A.T + 0.2 * np.eye(3)  # over (e, s, v)
    # embed into (e, n, w, s, v): n, w absent -> identity
    C = np.eye(5)
    idx = [0, 3, 4]
    for i in range(3):
        for j in range(3):
            C[idx[i], idx[j]] = C3[i, j]
    L = np.linalg.cholesky(C)
    par = np.zeros((16, 2, 2))
    eye = np.eye(5)
    for y in range(2):
        for x in range(2):
            LL = L if (y, x) == (0, 0) else eye
            k = 0
            for r in range(5):
                for c in range(r + 1):
                    par[1 + k, y, x] = LL[r, c]
                    k += 1
    for mus in ([0.0, 0.0, 0.0], [0.3, -0.2, 0.1]):
        par[0] = 0.0
        par[0, 0, 1], par[0, 1, 0], par[0, 0, 0] = mus  # e, s, v
        ns = 1 << 15
        est, _ = oracle.mvg_forward_at(par, [0], ns, seed=5)
        T = np.array([[1, 0, -1], [0, 1, -1]])  # (X_e - X_v, X_s - X_v)
        SD = T @ C3 @ T.T
        mD = T @ np.array(mus)
        if mus[0] == 0 and mus[1] == 0:
            rho = SD[0, 1] / math.sqrt(SD[0, 0] * SD[1, 1])
            pmin = 0.25 + math.asin(rho) / (2 * math.pi)
        else:
            pmin = stats.multivariate_normal(-mD, SD).cdf([0.0, 0.0])
        pmax = stats.multivariate_normal(mD, SD).cdf([0.0, 0.0])
        se = lambda p: math.sqrt(p * (1 - p) / ns)
        assert abs(est[0, 0] - pmin) < 4 * se(pmin) and abs(est[0, 2] - pmin) < 4 * se(pmin)
        assert abs(est[0, 1] - pmax) < 4 * se(pmax) and abs(est[0, 3] - pmax) < 4 * se(pmax)


def test_mvg_interior_four_dimensional_orthant():
    """Interior vertex with a full covariance: Pr(all four differences > 0) by
    scipy's multivariate normal CDF (Genz integration)."""
    rng = np.random.default_rng(8)
    A = rng.normal(size=(5, 5))
    C = A @ A.T / 5 + 0.3 * np.eye(5)
    mu = [0.05, -0.1, 0.2, 0.0, -0.05]
    par = mvg_grid(mu_plane(mu), np.linalg.cholesky(C))
    ns = 1 << 15
    est, _ = oracle.mvg_forward_at(par, [4], ns, seed=77)
    T = np.hstack([np.eye(4), -np.ones((4, 1))])
    SD = T @ C @ T.T
    mD = T @ np.array(mu)
    pmin = stats.multivariate_normal.cdf(np.zeros(4), -mD, SD, abseps=1e-7, releps=1e-7)
    pmax = stats.multivariate_normal.cdf(np.zeros(4), mD, SD, abseps=1e-7, releps=1e-7)
    se = lambda p: math.sqrt(p * (1 - p) / ns)
    assert abs(est[0, 0] - pmin) < 4 * se(pmin) and abs(est[0, 2] - pmin) < 4 * se(pmin)
    assert abs(est[0, 1] - pmax) < 4 * se(pmax) and abs(est[0, 3] - pmax) < 4 * se(pmax)


def test_mvg_conditional_gradient_matches_finite_differences():
    """Same Philox counters on both sides of the step: the conditional
    estimator is a smooth function of (mu, L), so central differences match
    its pathwise gradient."""
    rng = np.random.default_rng(4)
    H, W = 4, 5
    members = rng.normal(size=(12, H, W)) * 0.3 + rng.normal(size=(1, H, W))
    par = oracle.mvg_fit(members)
    gmin, gmax = workloads.upstream(2, H, W, np.float64)
    ns, seed = 64, 31
    idx = np.arange(H * W)
    gr = oracle.mvg_grad_at(par, gmin, gmax, idx, ns, seed)

    def loss(p):
        est, _ = oracle.mvg_forward_at(p, idx, ns, seed)
        return float((gmin.ravel() * est[:, 2]).sum() + (gmax.ravel() * est[:, 3]).sum())

    h = 1e-7
    for (y, x) in [(0, 0), (1, 2), (3, 4), (2, 1)]:
        for q in [0, 1, 3, 6, 10, 11, 14, 15]:
            pp = par.copy(); pm = par.copy()
            pp[q, y, x] += h; pm[q, y, x] -= h
            fd = (loss(pp) - loss(pm)) / (2 * h)
            assert gr[y * W + x, q] == pytest.approx(fd, abs=2e-6 * (1 + abs(fd)))


def test_mvg_gradient_tie_slack_bounds_a_flipped_tie():
    """The near-tie slack of the gradient: a neighbour (w) that duplicates
    another (e) exactly ties with it in every sample.  Moving mu_w by +-1e-13
    (far below any rounding bound) breaks every tie one way or the other, which
    moves whole sample terms between the two neighbours' gradient slots; the
    slack reported on either side bounds that change component by component,
    and it is exactly 0 for a stencil without ties."""
    rng = np.random.default_rng(12)
    A = rng.normal(size=(5, 5))
    L = np.linalg.cholesky(A @ A.T / 5 + 0.2 * np.eye(5))
    L[2, :] = 0.0
    L[2, 0] = L[0, 0]  # x_w = mu_w + L00 z0 = x_e when mu_w = mu_e
    mu = [0.05, -0.02, 0.05, 0.01, 0.0]  # e, n, w, s, v
    H, W = 3, 3
    gmin, gmax = workloads.upstream(3, H, W, np.float64)
    idx = np.arange(H * W)
    ns, seed = 512, 17
    res = []
    for d in (1e-13, -1e-13):
        m = list(mu)
        m[2] += d
        res.append(oracle.mvg_grad_at(mvg_grid(mu_plane(m), L), gmin, gmax, idx, ns, seed, slack=True))
    (gp, sp), (gm, sm) = res
    diff = np.abs(gp - gm)
    assert diff.max() > 1e-3  # the ties moved terms between e and w
    assert np.all(diff <= sp + 1e-9) and np.all(diff <= sm + 1e-9)
    # the slack sits on the tied neighbours only: mean gradients of e and w
    # (through the centre's stencil) and the centre's L rows of e and w
    rows_e, rows_w = [1], [4, 5, 6]  # packed positions of L_00 and L_20..L_22 (offset 1)
    for flat in range(H * W):
        y, x = divmod(flat, W)
        if (y, x) not in (POS["e"], POS["w"]):
            assert sp[flat, 0] == 0.0 and sm[flat, 0] == 0.0, (y, x)
    centre_slack = sp[4, 1:]
    nz = set(np.nonzero(centre_slack)[0] + 1)
    assert nz <= set(rows_e + rows_w) and nz, nz
    # without the duplicate there is no tie and no slack
    L2 = np.linalg.cholesky(A @ A.T / 5 + 0.2 * np.eye(5))
    _, s0 = oracle.mvg_grad_at(mvg_grid(mu_plane([0.1, -0.2, 0.3, 0.05, 0.0]), L2), gmin, gmax, idx, ns, seed,
                               slack=True)
    assert np.all(s0 == 0.0)


def test_mvg_fit_against_numpy():
    rng = np.random.default_rng(6)
    members = rng.normal(size=(20, 5, 6))
    par = oracle.mvg_fit(members, ddof=1, jitter=1e-6)
    np.testing.assert_allclose(par[0], members.mean(0), rtol=1e-13)
    offs = {"e": (0, 1), "n": (-1, 0), "w": (0, -1), "s": (1, 0), "v": (0, 0)}
    for (y, x) in [(2, 3), (0, 0), (4, 5), (0, 3)]:
        series, present = [], []
        for k in ["e", "n", "w", "s", "v"]:
            yy, xx = y + offs[k][0], x + offs[k][1]
            ok = 0 <= yy < 5 and 0 <= xx < 6
            present.append(ok)
            series.append(members[:, yy, xx] if ok else np.zeros(20))
        C = np.cov(np.array(series), ddof=1) + 1e-6 * np.eye(5)
        for i in range(5):
            for j in range(5):
                if not (present[i] and present[j]):
                    C[i, j] = 1.0 if i == j else 0.0
        L = np.linalg.cholesky(C)
        k = 0
        for r in range(5):
            for c in range(r + 1):
                assert par[1 + k, y, x] == pytest.approx(L[r, c], abs=1e-12)
                k += 1


# ----------------------------------------------------------------------------
# saddle probability (Eq. 2, Eq. 4)
# ----------------------------------------------------------------------------
def saddle_centre(model, grid):
    t1, t2 = oracle.saddle_at(model, grid, [4])
    return t1[0], t2[0]


@pytest.mark.parametrize("model,par", [(U, (0.0, 1.0)), (E, (0.3, 0.01)), (HST, (0.0, 1.0, 0.1, 0.2, 0.3, 0.4))])
def test_saddle_iid_is_one_fifteenth(model, par):
    """Identical independent values: t1 = int F^2 S^2 dF = int_0^1 u^2 (1-u)^2 du
    = 1/30, and t2 likewise, so P_saddle = 1/15 (by exchangeability every one
    of the 5! orders is equally likely and 4 of them put v between e,w and
    n,s in each alternating way)."""
    g = np.broadcast_to(np.array(par)[:, None, None], (len(par), 5, 6)).copy()
    ps = oracle.saddle(model, g)
    np.testing.assert_allclose(ps[1:-1, 1:-1], 1 / 15, atol=1e-14)
    assert np.all(ps[0, :] == 0) and np.all(ps[:, 0] == 0) and np.all(ps[-1, :] == 0) and np.all(ps[:, -1] == 0)


def test_saddle_disjoint_supports():
    """e, w entirely above v and n, s entirely below: a certain saddle of the
    first kind (t1 = 1, t2 = 0)."""
    d = {"v": (0.0, 1.0), "e": (2.0, 3.0), "w": (1.5, 4.0), "n": (-2.0, -1.0), "s": (-3.0, -0.5)}
    t1, t2 = saddle_centre(U, stencil_grid(U, d))
    assert t1 == pytest.approx(1.0, abs=1e-15) and t2 == 0.0
    d["n"] = (3.0, 4.0)  # now n is above v as well: impossible
    t1, t2 = saddle_centre(U, stencil_grid(U, d))
    assert t1 == 0.0 and t2 == 0.0


@pytest.mark.parametrize("model", [U, E, HST])
def test_saddle_against_scipy_quadrature(model):
    rng = np.random.default_rng(71 + model)
    nb = 4
    for _ in range(8):
        d = random_stencil(model, rng, nb)
        t1, t2 = saddle_centre(model, stencil_grid(model, d, nb if model == HST else 0))
        dv, pts = scipy_dist(model, d["v"])
        dist = {}
        allpts = list(pts)
        for k in "enws":
            dist[k], p = scipy_dist(model, d[k])
            allpts += p
        lo, hi = pts[0], pts[-1]
        inner = sorted({p for p in allpts if lo < p < hi})
        kw = dict(points=inner or None, limit=400, epsabs=1e-14, epsrel=1e-12)
        f1 = lambda x: dv.pdf(x) * dist["e"].sf(x) * dist["n"].cdf(x) * dist["w"].sf(x) * dist["s"].cdf(x)
        f2 = lambda x: dv.pdf(x) * dist["e"].cdf(x) * dist["n"].sf(x) * dist["w"].cdf(x) * dist["s"].sf(x)
        assert t1 == pytest.approx(integrate.quad(f1, lo, hi, **kw)[0], abs=2e-10)
        assert t2 == pytest.approx(integrate.quad(f2, lo, hi, **kw)[0], abs=2e-10)


@pytest.mark.parametrize("model", [U, E, HST])
def test_saddle_brute_force_monte_carlo(model):
    rng = np.random.default_rng(17 + model)
    nb = 3
    d = MIXED_STENCILS.get(model) or {
        "v": (0, 1, 0.5, 0.25, 0.25), "e": (-0.5, 0.5, 1 / 3, 1 / 3, 1 / 3),
        "n": (0.25, 1.25, 0.1, 0.6, 0.3), "w": (0.5, 2.0, 0.2, 0.3, 0.5), "s": (0.1, 0.9, 0.2, 0.2, 0.6)}
    t1, t2 = saddle_centre(model, stencil_grid(model, d, nb if model == HST else 0))
    N, chunks, c1, c2 = 1_000_000, 4, 0, 0
    for _ in range(chunks):
        xs = {k: sample(model, d[k], N, rng) for k in POS}
        v = xs["v"]
        c1 += int(np.count_nonzero((v < xs["e"]) & (v > xs["n"]) & (v < xs["w"]) & (v > xs["s"])))
        c2 += int(np.count_nonzero((v > xs["e"]) & (v < xs["n"]) & (v > xs["w"]) & (v < xs["s"])))
    n = N * chunks
    for p, c in ((t1, c1), (t2, c2)):
        se = math.sqrt(max(p * (1 - p), 1e-12) / n)
        assert abs(c / n - p) < 4 * se, (p, c / n, se)


@pytest.mark.parametrize("model", [U, E, HST])
def test_saddle_negation_and_classes(model):
    """Negating every value swaps the two saddle terms (Sec. 4.1.3); minimum,
    maximum and saddle are disjoint events, so their probabilities sum to at
    most 1."""
    par = workloads.random_params(model, 6, 9, 11, nbins=4, width=0.05)
    idx = np.arange(9 * 11)
    t1, t2 = oracle.saddle_at(model, par, idx)
    n1, n2 = oracle.saddle_at(model, negate(model, par), idx)
    np.testing.assert_allclose(t1, n2, atol=1e-13)
    np.testing.assert_allclose(t2, n1, atol=1e-13)
    pmin, pmax = oracle.forward(model, par)
    assert np.all(pmin.ravel() + pmax.ravel() + t1 + t2 <= 1 + 1e-12)


@pytest.mark.parametrize("model", [U, E, HST])
def test_classification_brute_force_monte_carlo(model):
    """The four classes (minimum, maximum, saddle of either kind, regular)
    partition the outcomes of one draw of the stencil; P_regular is the rest,
    1 - P_min - P_max - P_saddle.  All four against the sampled frequencies."""
    rng = np.random.default_rng(29 + model)
    nb = 3
    d = random_stencil(model, rng, nb)
    g = stencil_grid(model, d, nb if model == HST else 0)
    pmin, pmax = oracle.forward_at(model, g, [4])
    t1, t2 = saddle_centre(model, g)
    probs = {"min": pmin[0], "max": pmax[0], "saddle": t1 + t2}
    probs["regular"] = 1.0 - probs["min"] - probs["max"] - probs["saddle"]
    N, chunks = 1_000_000, 3
    counts = dict.fromkeys(probs, 0)
    for _ in range(chunks):
        xs = {k: sample(model, d[k], N, rng) for k in POS}
        v, e, n, w, s = (xs[k] for k in "venws")
        is_min = (v < e) & (v < n) & (v < w) & (v < s)
        is_max = (v > e) & (v > n) & (v > w) & (v > s)
        is_sad = ((v < e) & (v > n) & (v < w) & (v > s)) | ((v > e) & (v < n) & (v > w) & (v < s))
        counts["min"] += int(np.count_nonzero(is_min))
        counts["max"] += int(np.count_nonzero(is_max))
        counts["saddle"] += int(np.count_nonzero(is_sad))
        counts["regular"] += int(np.count_nonzero(~(is_min | is_max | is_sad)))
    n_all = N * chunks
    assert sum(counts.values()) == n_all
    for k, p in probs.items():
        se = math.sqrt(max(p * (1 - p), 1e-12) / n_all)
        assert abs(counts[k] / n_all - p) < 4 * se, (k, p, counts[k] / n_all, se)


# ----------------------------------------------------------------------------
# error-bound uniform model (Sec. 5.3, climate data)
# ----------------------------------------------------------------------------
def test_error_bound_single_close_neighbour():
    """Decompressed centre 0, eb = 1: a neighbour at distance delta < eb gives
    Pr[X_v < X_n] = 1 - (1 - delta)^2 / 2 (two unit-width uniforms); the
    other three neighbours lie more than eb above and never interfere."""
    for delta in (0.0, 0.25, 0.6, 0.999):
        d = np.full((3, 3), 5.0)
        d[1, 1] = 0.0
        d[1, 2] = delta
        par = oracle.fit_error_bound(d, 1.0)
        pmin, _ = oracle.forward_at(U, par, [4])
        assert pmin[0] == pytest.approx(1 - (1 - delta) ** 2 / 2, abs=1e-14)


def test_error_bound_certain_and_equal():
    """Gaps larger than eb give the classical min/max (P in {0, 1}); equal
    decompressed values give identical independent ranges, P = 1/5."""
    d = np.array([[3.0, 2.0, 3.0], [2.0, 0.0, 2.5], [3.0, 1.1, 3.0]])
    par = oracle.fit_error_bound(d, 1.0)
    pmin, pmax = oracle.forward_at(U, par, [4])
    assert pmin[0] == 1.0 and pmax[0] == 0.0
    par = oracle.fit_error_bound(np.full((3, 3), 0.7), 0.01)
    pmin, pmax = oracle.forward_at(U, par, [4])
    assert pmin[0] == pytest.approx(0.2, abs=1e-13) and pmax[0] == pytest.approx(0.2, abs=1e-13)


def test_error_bound_fp32_ends_are_rounded_once():
    """In FP32 each end is the correctly rounded d' -/+ eb/2."""
    from fractions import Fraction
    rng = np.random.default_rng(3)
    d = rng.uniform(-100, 100, 257).astype(np.float32)
    eb = 1e-3
    par = oracle.fit_error_bound(d[None, :], eb, single=True)
    h = Fraction(float(np.float32(eb * 0.5)))
    for i in range(d.size):
        lo_exact = Fraction(float(d[i])) - h
        hi_exact = Fraction(float(d[i])) + h
        assert par[0, 0, i] == float(np.float32(float(lo_exact))) or abs(
            Fraction(par[0, 0, i]) - lo_exact) <= abs(Fraction(float(np.float32(float(lo_exact)))) - lo_exact)
        assert par[1, 0, i] == float(np.float32(float(hi_exact))) or abs(
            Fraction(par[1, 0, i]) - hi_exact) <= abs(Fraction(float(np.float32(float(hi_exact)))) - hi_exact)


# ----------------------------------------------------------------------------
# independent Gaussian model (the parametric comparison model of Sec. 5.2)
# ----------------------------------------------------------------------------
G = oracle.GAUSSIAN


def gauss_grid(vals):
    """3x3 (mu, sigma) grid with the given stencil; other cells far away."""
    par = np.zeros((2, 3, 3))
    par[0] = 50.0
    par[1] = 1.0
    for k, (m, s) in vals.items():
        par[0][POS[k]] = m
        par[1][POS[k]] = s
    return par


def random_gauss_stencil(rng):
    sig = 10 ** rng.uniform(-2, 0.3, 5) if rng.random() < 0.5 else 10 ** rng.uniform(-0.3, 0.3, 5)
    mu = rng.normal(0, 1, 5) * (0.4 if rng.random() < 0.7 else 3)
    return {k: (mu[i], sig[i]) for i, k in enumerate("venws")}


def test_gauss_iid_values():
    """Identical independent Gaussians: every ordering of the five values is
    equally likely, so P_min = P_max = 1/5 and t1 = t2 = 1/30 (4 of 120)."""
    for m, s in ((0.0, 1.0), (3.5, 0.01), (-200.0, 7.0)):
        r = oracle.gauss_at(gauss_grid({k: (m, s) for k in "venws"}), [4])[0]
        np.testing.assert_allclose(r, [0.2, 0.2, 1 / 30, 1 / 30], atol=1e-14)


def test_gauss_single_neighbour_closed_form():
    """1x2 grid: each vertex has one neighbour, and Pr[X_v < X_n] =
    Phi((mu_n - mu_v) / sqrt(sigma_v^2 + sigma_n^2))."""
    from scipy import special
    rng = np.random.default_rng(4)
    for _ in range(20):
        mu = rng.normal(0, 1, 2)
        sg = 10 ** rng.uniform(-2, 0.5, 2)
        p = np.array([[mu], [sg]]).reshape(2, 1, 2)
        r = oracle.gauss_at(p, [0, 1])
        z = (mu[1] - mu[0]) / math.hypot(sg[0], sg[1])
        assert r[0, 0] == pytest.approx(special.ndtr(z), abs=1e-14)
        assert r[0, 1] == pytest.approx(special.ndtr(-z), abs=1e-14)
        assert r[1, 0] == pytest.approx(special.ndtr(-z), abs=1e-14)
        assert r[0, 2] == 0.0 and r[0, 3] == 0.0


def test_gauss_corner_bivariate_orthant():
    """Corner vertex (0,0) with neighbours e, s: (X_e - X_v, X_s - X_v) is
    bivariate normal with covariance [[s_v^2 + s_e^2, s_v^2], [s_v^2,
    s_v^2 + s_s^2]]; P_min is its positive orthant (scipy's bivariate normal
    CDF)."""
    rng = np.random.default_rng(8)
    for _ in range(10):
        mu = rng.normal(0, 0.5, 3)
        sg = 10 ** rng.uniform(-1, 0.3, 3)
        p = np.zeros((2, 2, 2))
        p[1] = 1.0
        p[0, 0, 0], p[0, 0, 1], p[0, 1, 0] = mu  # v, e, s
        p[1, 0, 0], p[1, 0, 1], p[1, 1, 0] = sg
        r = oracle.gauss_at(p, [0])[0]
        dm = np.array([mu[1] - mu[0], mu[2] - mu[0]])
        C = np.array([[sg[0] ** 2 + sg[1] ** 2, sg[0] ** 2], [sg[0] ** 2, sg[0] ** 2 + sg[2] ** 2]])
        # Pr[D > 0] = Pr[-D < 0] with -D ~ N(-dm, C)
        ref = stats.multivariate_normal.cdf(np.zeros(2), -dm, C, abseps=1e-12, releps=1e-12)
        assert r[0] == pytest.approx(ref, abs=1e-9)


def test_gauss_against_scipy_quadrature():
    """Interior stencils with mixed scales: all four integrals against scipy's
    adaptive quadrature of scipy.stats densities and tails."""
    rng = np.random.default_rng(12)
    for _ in range(12):
        d = random_gauss_stencil(rng)
        r = oracle.gauss_at(gauss_grid(d), [4])[0]
        dv = stats.norm(*d["v"])
        nb = {k: stats.norm(*d[k]) for k in "enws"}
        pts = sorted(m + c * s for m, s in d.values() for c in (-3, 0, 3))
        lo, hi = d["v"][0] - 12 * d["v"][1], d["v"][0] + 12 * d["v"][1]
        inner = [p for p in pts if lo < p < hi]
        kw = dict(points=inner or None, limit=500, epsabs=1e-14, epsrel=1e-12)
        fs = [
            lambda x: dv.pdf(x) * np.prod([nb[k].sf(x) for k in "enws"]),
            lambda x: dv.pdf(x) * np.prod([nb[k].cdf(x) for k in "enws"]),
            lambda x: dv.pdf(x) * nb["e"].sf(x) * nb["n"].cdf(x) * nb["w"].sf(x) * nb["s"].cdf(x),
            lambda x: dv.pdf(x) * nb["e"].cdf(x) * nb["n"].sf(x) * nb["w"].cdf(x) * nb["s"].sf(x),
        ]
        for q in range(4):
            assert r[q] == pytest.approx(integrate.quad(fs[q], lo, hi, **kw)[0], abs=1e-11), q


def test_gauss_brute_force_monte_carlo():
    rng = np.random.default_rng(31)
    d = {"v": (0.0, 0.3), "e": (0.2, 0.5), "n": (-0.1, 0.2), "w": (0.05, 0.3), "s": (-0.3, 0.4)}
    r = oracle.gauss_at(gauss_grid(d), [4])[0]
    N, chunks = 1_000_000, 3
    c = np.zeros(4)
    for _ in range(chunks):
        x = {k: rng.normal(m, s, N) for k, (m, s) in d.items()}
        v, e, n, w, s = (x[k] for k in "venws")
        c += [np.count_nonzero((v < e) & (v < n) & (v < w) & (v < s)),
              np.count_nonzero((v > e) & (v > n) & (v > w) & (v > s)),
              np.count_nonzero((v < e) & (v > n) & (v < w) & (v > s)),
              np.count_nonzero((v > e) & (v < n) & (v > w) & (v < s))]
    n_all = N * chunks
    for q in range(4):
        se = math.sqrt(r[q] * (1 - r[q]) / n_all)
        assert abs(c[q] / n_all - r[q]) < 4 * se, (q, r[q], c[q] / n_all)


def test_gauss_negation_and_invariance():
    """Negating every value swaps P_min/P_max and t1/t2 (Sec. 4.1.2, 4.1.3);
    an affine change of units a X + b (a > 0) changes nothing."""
    rng = np.random.default_rng(2)
    par = np.stack([rng.normal(0, 0.1, (7, 9)), 10 ** rng.uniform(-2, -0.5, (7, 9))])
    r = oracle.gauss(par)
    neg = oracle.gauss(np.stack([-par[0], par[1]]))
    np.testing.assert_allclose(r[[1, 0, 3, 2]], neg, atol=1e-13)
    aff = oracle.gauss(np.stack([3.0 * par[0] + 17.0, 3.0 * par[1]]))
    np.testing.assert_allclose(r, aff, atol=1e-12)
    assert np.all(r.sum(0) <= 1 + 1e-12)


def test_gauss_equals_diagonal_multivariate_model():
    """The multivariate Gaussian model with a diagonal covariance is the
    independent model: its conditional Monte Carlo estimate (a separate
    oracle routine, Philox samples) agrees within 4 standard errors."""
    means = [0.1, -0.2, 0.3, 0.05, 0.0]  # e, n, w, s, v
    sig = [0.3, 0.5, 0.4, 0.2, 0.35]
    r = oracle.gauss_at(gauss_grid({k: (means[i], sig[i]) for i, k in enumerate("enwsv")}), [4])[0]
    est, _ = oracle.mvg_forward_at(mvg_grid(mu_plane(means), np.diag(sig)), [4], 1 << 15, seed=777)
    for got, p in ((est[0, 2], r[0]), (est[0, 3], r[1])):
        assert abs(got - p) < 4 * math.sqrt(p * (1 - p) / (1 << 15)), (got, p)


def test_gauss_jacobian_matches_finite_differences():
    """Derivatives of P_min / P_max of a stencil with respect to (mu, sigma)
    of each slot, against central differences of the oracle's forward (an
    independent route: no derivative formula)."""
    rng = np.random.default_rng(21)
    slots = "venws"
    for _ in range(6):
        d = random_gauss_stencil(rng)
        par = gauss_grid(d)
        jm, jx = oracle.gauss_jacobian_at(par, [4])
        for si, k in enumerate(slots):
            for q in range(2):
                h = 1e-5 * d[k][1]
                pp, pm = par.copy(), par.copy()
                pp[q][POS[k]] += h
                pm[q][POS[k]] -= h
                fp, fm = oracle.gauss_at(pp, [4])[0], oracle.gauss_at(pm, [4])[0]
                for j, r in ((0, jm), (1, jx)):
                    fd = (fp[j] - fm[j]) / (2 * h)
                    assert r[0, si, q] == pytest.approx(fd, rel=2e-6, abs=2e-7 / d[k][1]), (k, q, j)


def test_gauss_jacobian_invariances():
    """Translation (sum of the mu-derivatives is 0) and scale about the vertex
    mean (sigma_v dP/dsigma_v + sum_n (mu_n - mu_v) dP/dmu_n + sigma_n
    dP/dsigma_n = 0): the identities the device adjoint uses for the vertex
    slot, checked on the oracle, which integrates that slot directly."""
    rng = np.random.default_rng(23)
    for _ in range(8):
        d = random_gauss_stencil(rng)
        jm, jx = oracle.gauss_jacobian_at(gauss_grid(d), [4])
        for r in (jm[0], jx[0]):
            scale = np.abs(r).sum()
            assert abs(r[:, 0].sum()) <= 1e-11 * scale
            sc = sum((d[k][0] - d["v"][0]) * r[i, 0] + d[k][1] * r[i, 1] for i, k in enumerate("venws"))
            assert abs(sc) <= 1e-11 * (scale * (1 + max(abs(d[k][0] - d["v"][0]) + d[k][1] for k in "venws")))


def test_gauss_jacobian_magnitude_scale():
    """The integrals of the integrands' magnitudes (the rounding scale the
    adjoint tolerances use): a lone vertex has closed forms (the integrals of
    phi(u) |u| and phi(u) |u^2 - 1| are sqrt(2/pi) and 4 phi(1), over
    sigma); in a stencil they bound the signed integrals and equal them
    where the integrand has one sign (the mu-derivatives of the neighbours'
    survival and distribution factors)."""
    sg = 0.37
    par = np.array([[[0.2]], [[sg]]])
    for r in oracle.gauss_jacobian_at(par, [0], absolute=True):
        assert r[0, 0, 0] == pytest.approx(math.sqrt(2 / math.pi) / sg, rel=1e-12)
        assert r[0, 0, 1] == pytest.approx(4 * math.exp(-0.5) / math.sqrt(2 * math.pi) / sg, rel=1e-12)
        assert np.all(r[0, 1:] == 0)
    rng = np.random.default_rng(27)
    for _ in range(6):
        par = gauss_grid(random_gauss_stencil(rng))
        jm, jx = oracle.gauss_jacobian_at(par, [4])
        am, ax = oracle.gauss_jacobian_at(par, [4], absolute=True)
        for j, a in ((jm, am), (jx, ax)):
            assert np.all(a >= np.abs(j) * (1 - 1e-12))
            assert a[0, 1:, 0] == pytest.approx(np.abs(j[0, 1:, 0]), rel=1e-11)


def test_gauss_adjoint_matches_finite_differences_of_the_loss():
    """Gathered adjoint of L = sum g_min P_min + g_max P_max on a 5x6 grid
    (edges, corners) against central differences of L itself."""
    rng = np.random.default_rng(25)
    H, W = 5, 6
    par = np.stack([rng.normal(0, 0.2, (H, W)), 10 ** rng.uniform(-1.3, -0.5, (H, W))])
    g1, g2 = rng.normal(size=(H, W)), rng.normal(size=(H, W))
    idx = np.arange(H * W)
    got = oracle.gauss_grad_at(par, g1, g2, idx)
    def loss(p):
        r = oracle.gauss(p)
        return float((g1 * r[0] + g2 * r[1]).sum())
    for i in idx[::3]:
        y, x = divmod(int(i), W)
        for q in range(2):
            h = 1e-5 * par[1, y, x]
            pp, pm = par.copy(), par.copy()
            pp[q, y, x] += h
            pm[q, y, x] -= h
            fd = (loss(pp) - loss(pm)) / (2 * h)
            assert got[i, q] == pytest.approx(fd, rel=2e-6, abs=1e-6 / par[1, y, x]), (i, q)


def test_gauss_fit_against_numpy():
    mem = workloads.smooth_ensemble(2, 9, 13)
    par = oracle.fit(G, mem.astype(np.float64))
    np.testing.assert_allclose(par[0], mem.astype(np.float64).mean(0), rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(par[1], mem.astype(np.float64).std(0, ddof=1), rtol=1e-12)


# ----------------------------------------------------------------------------
# semianalytical histogram estimator (Sec. 4.4.2)
# ----------------------------------------------------------------------------
def test_semi_sampler_is_the_inverse_histogram_cdf():
    """The estimator's sample positions are the histogram's inverse CDF at
    the Philox uniforms ((word >> 8) + 1/2) 2^-24 of counter
    (i // 4, y*W + x, field_id, 2): recomputed with numpy's piecewise-linear
    interpolation of the cumulative masses."""
    par = workloads.random_params(HST, 5, 4, 5, nbins=7, width=0.1)
    y, x, ns, seed, fid = 2, 3, 64, 0x1234_5678_9ABC, 7
    xs = oracle.semi_samples(par, y, x, ns, seed, fid)
    lo, hi, m = par[0, y, x], par[1, y, x], par[2:, y, x]
    C = np.concatenate([[0.0], np.cumsum(m)])
    edges = lo + (hi - lo) * np.arange(len(m) + 1) / len(m)
    key = np.array([seed & 0xFFFFFFFF, seed >> 32], dtype=np.uint32)
    for i in range(ns):
        w = oracle.philox4x32_10([i // 4, y * 5 + x, fid, 2], key)[i % 4]
        u = ((int(w) >> 8) + 0.5) / 2.0 ** 24
        assert xs[i] == pytest.approx(np.interp(u * C[-1], C, edges), abs=1e-13)


def test_semi_samples_follow_the_histogram():
    """Kolmogorov-Smirnov: 20000 samples against the histogram CDF."""
    par = workloads.random_params(HST, 9, 3, 3, nbins=5, width=0.2)
    xs = oracle.semi_samples(par, 1, 1, 20000, seed=3)
    lo, hi, m = par[0, 1, 1], par[1, 1, 1], par[2:, 1, 1]
    C = np.concatenate([[0.0], np.cumsum(m)]) / m.sum()
    edges = lo + (hi - lo) * np.arange(len(m) + 1) / len(m)
    assert stats.kstest(xs, lambda t: np.interp(t, edges, C)).pvalue > 1e-3


def test_semi_point_mass_vertex():
    """A vertex histogram of width 1e-12 puts every sample at x0, so each
    estimate is the product of the neighbours' tails at x0 (numpy
    interpolation of their cumulative masses)."""
    par = workloads.random_params(HST, 11, 3, 3, nbins=4, width=0.2)
    x0 = par[0, 1, 1] + 0.3 * (par[1, 1, 1] - par[0, 1, 1])
    par[0, 1, 1], par[1, 1, 1] = x0, x0 + 1e-12
    est = oracle.semi_at(par, [4], 64, seed=1)[0]
    S, F = {}, {}
    for k in "enws":
        yy, xx = POS[k]
        lo, hi, m = par[0, yy, xx], par[1, yy, xx], par[2:, yy, xx]
        edges = lo + (hi - lo) * np.arange(len(m) + 1) / len(m)
        F[k] = np.interp(x0, edges, np.concatenate([[0.0], np.cumsum(m)]))
        S[k] = m.sum() - F[k]
    T = par[2:, 1, 1].sum()
    ref = [T * np.prod([S[k] for k in "enws"]), T * np.prod([F[k] for k in "enws"]),
           T * S["e"] * F["n"] * S["w"] * F["s"], T * F["e"] * S["n"] * F["w"] * S["s"]]
    np.testing.assert_allclose(est, ref, atol=1e-9)


@pytest.mark.parametrize("seed", [0, 1])
def test_semi_estimates_are_unbiased(seed):
    """2^15 samples per vertex: every estimate lies within 4 standard errors
    of the closed-form value (Eq. 3, Eq. 4) of the same histograms (each
    sample's product lies in [0, 1], so its variance is at most p(1 - p))."""
    par = workloads.random_params(HST, 20 + seed, 6, 7, nbins=6, width=0.08)
    idx = np.arange(6 * 7)
    ns = 1 << 15
    est = oracle.semi_at(par, idx, ns, seed=seed + 5)
    pmin, pmax = oracle.forward_at(HST, par, idx)
    t1, t2 = oracle.saddle_at(HST, par, idx)
    for q, ref in enumerate((pmin, pmax, t1, t2)):
        se = np.sqrt(np.clip(ref * (1 - ref), 1e-12, None) / ns)
        assert np.all(np.abs(est[:, q] - ref) <= 4 * se + 1e-12), q
