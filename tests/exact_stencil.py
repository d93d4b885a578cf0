"""Exact rational P_min / P_max of one 2-D stencil, for the pins of the
oracle (test infrastructure; shares nothing with the oracle or the HIP path).

P_min(v) = integral of pdf_v(x) prod_n S_n(x) dx and P_max(v) = integral of
pdf_v(x) prod_n F_n(x) dx (Eq. 3 with the inner integrals done; the maximum
by the negation argument of Sec. 4.1.2).  Every density here is piecewise
polynomial with rational breakpoints and coefficients -- uniform and
Epanechnikov (Sec. 4.3), histogram as a mixture of uniform bin kernels
(Sec. 4.4.1) -- so the integral is a finite sum of integrals of polynomial
products, evaluated exactly with fractions.Fraction: no floating point.

A distribution is a list of pieces (x0, x1, c) with pdf(x) = sum_k c[k] x^k on
[x0, x1) and 0 outside the pieces.
"""
from fractions import Fraction as Fr


def pmul(a, b):
    out = [Fr(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        if x:
            for j, y in enumerate(b):
                out[i + j] += x * y
    return out


def pint(c):
    """Antiderivative with zero constant."""
    return [Fr(0)] + [x / (k + 1) for k, x in enumerate(c)]


def peval(c, x):
    r = Fr(0)
    for k in reversed(range(len(c))):
        r = r * x + c[k]
    return r


def uniform(a, b):
    a, b = Fr(a), Fr(b)
    return [(a, b, [1 / (b - a)])]


def epanechnikov(m, w):
    """pdf 3/(4w) (1 - ((x - m)/w)^2) on [m - w, m + w], expanded in x."""
    m, w = Fr(m), Fr(w)
    k = Fr(3) / (4 * w)
    # 1 - (x - m)^2 / w^2 = (1 - m^2/w^2) + (2m/w^2) x - x^2 / w^2
    return [(m - w, m + w, [k * (1 - m * m / (w * w)), k * 2 * m / (w * w), -k / (w * w)])]


def histogram(lo, hi, masses):
    """Equal-width bins over [lo, hi]; pdf = mass_j / Delta on bin j."""
    lo, hi = Fr(lo), Fr(hi)
    h = len(masses)
    d = (hi - lo) / h
    return [(lo + j * d, lo + (j + 1) * d, [Fr(m) / d]) for j, m in enumerate(masses)]


def _cdf_pieces(dist):
    """[(x0, x1, CDF polynomial on the piece)], plus the total mass."""
    acc, out = Fr(0), []
    for x0, x1, c in sorted(dist, key=lambda p: p[0]):
        P = pint(c)
        q = [-peval(P, x0) + acc] + [Fr(0)] * (len(P) - 1)
        cdf = [P[k] + q[k] for k in range(len(P))]
        out.append((x0, x1, cdf))
        acc = peval(cdf, x1)
    return out, acc


def _factor(dist, x0, x1, survival):
    """S (or F) of dist as a polynomial on the sub-interval [x0, x1], which
    lies inside one piece or entirely between / outside the pieces."""
    pieces, total = _cdf_pieces(dist)
    mid = (x0 + x1) / 2
    cdf = [Fr(0)]  # below the support
    for a, b, c in pieces:
        if a <= mid < b:
            cdf = c
            break
        if b <= mid:  # past this piece: the CDF is constant until the next one
            cdf = [peval(c, b)]
    if survival:
        return [total - cdf[0]] + [-x for x in cdf[1:]]
    return list(cdf)


def _pdf_on(dist, x0, x1):
    mid = (x0 + x1) / 2
    for a, b, c in dist:
        if a <= mid < b:
            return c
    return None


def exact_min_max(v, neighbours):
    """(P_min, P_max) as Fractions for the vertex distribution v and a list of
    neighbour distributions (each a list of pieces)."""
    cuts = set()
    for d in [v] + list(neighbours):
        for a, b, _ in d:
            cuts.add(a)
            cuts.add(b)
    cuts = sorted(cuts)
    res = []
    for survival in (True, False):
        total = Fr(0)
        for x0, x1 in zip(cuts[:-1], cuts[1:]):
            pv = _pdf_on(v, x0, x1)
            if pv is None:
                continue
            poly = list(pv)
            for d in neighbours:
                poly = pmul(poly, _factor(d, x0, x1, survival))
            P = pint(poly)
            total += peval(P, x1) - peval(P, x0)
        res.append(total)
    return tuple(res)


# ----------------------------------------------------------------------------
# the fixture tests/golden/exact_2d_stencils.txt
# ----------------------------------------------------------------------------
SLOTS = ("v", "e", "n", "w", "s")
POS = {"v": (1, 1), "e": (1, 2), "n": (0, 1), "w": (1, 0), "s": (2, 1)}
MODELS = {"uniform": 0, "epanechnikov": 1, "histogram": 2}


def load_cases(path):
    """[{name, model, dists: {slot: (numbers, masses or None)}, p_min, p_max}]"""
    cases, cur = [], None
    with open(path) as fh:
        for line in fh:
            line = line.split("#")[0].strip()
            if not line:
                continue
            key, _, rest = line.partition(" ")
            if key == "case":
                cur = {"name": rest.strip(), "dists": {}}
                cases.append(cur)
            elif key == "model":
                cur["model"] = rest.strip()
            elif key in SLOTS:
                head, _, tail = rest.partition(":")
                nums = [Fr(t) for t in head.split()]
                masses = [Fr(t) for t in tail.split()] if tail.strip() else None
                cur["dists"][key] = (nums, masses)
            elif key in ("p_min", "p_max"):
                cur[key] = Fr(rest.strip())
    return cases


def case_dist(model, nums, masses):
    if model == "uniform":
        return uniform(*nums)
    if model == "epanechnikov":
        return epanechnikov(*nums)
    return histogram(nums[0], nums[1], masses)


def case_exact(case):
    d = {k: case_dist(case["model"], *case["dists"][k]) for k in SLOTS}
    return exact_min_max(d["v"], [d[k] for k in SLOTS[1:]])


def case_grid(case):
    """(model id, nbins, parameter planes [n_param][3][3] as floats) with the
    case's stencil around the centre; the corners copy v (they are not in the
    centre's stencil).  Histograms of different bin counts are written with a
    common count (the least common multiple), each bin's mass split equally
    over the finer bins it covers -- the same density."""
    import math

    import numpy as np
    model = MODELS[case["model"]]
    nb = 0
    if model == 2:
        nb = 1
        for _, m in case["dists"].values():
            nb = nb * len(m) // math.gcd(nb, len(m))
    npar = 2 + nb
    g = np.zeros((npar, 3, 3))

    def planes(nums, masses):
        col = [float(nums[0]), float(nums[1])]
        if model == 2:
            r = nb // len(masses)
            col += [float(m / r) for m in masses for _ in range(r)]
        return col

    for y in range(3):
        for x in range(3):
            g[:, y, x] = planes(*case["dists"]["v"])
    for k in SLOTS:
        g[:, POS[k][0], POS[k][1]] = planes(*case["dists"][k])
    return model, nb, g
