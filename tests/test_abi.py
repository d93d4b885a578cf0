"""Host-side checks of the C ABI: the library loads, exports every function
include/cpcrit.h declares, its Gauss-Legendre tables are the textbook rules,
and argument validation answers before anything reaches the device.  No
compute call is made here (no GPU needed)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_2407_18015_amd import _lib as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    text = open(os.path.join(ROOT, "include", "cpcrit.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(c[a-z_0-9]+)\s*\(", text, flags=re.M)))


def test_library_exports_every_declared_function():
    lib = L.load()
    names = header_functions()
    assert set(names) >= {"cpu_fit_params", "cp_prob_forward", "cp_prob_backward", "cp_prob_batched"}
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(L.EXPORTS) == names


def test_struct_layouts_match_header():
    # int32 h, w; int64 row_stride; int32 model, dtype, nbins, nsamples; uint64 seed; uint32 id; int32 est
    assert ctypes.sizeof(L.cp_field_desc_t) == 48
    assert L.cp_field_desc_t.seed.offset == 32
    assert ctypes.sizeof(L.cp_fit_opts_t) == 32


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8, 10])
def test_gauss_legendre_tables(n):
    """The device rules against numpy's Gauss-Legendre (Golub-Welsch)."""
    x, w = L.cp_gauss_legendre(n)
    xr, wr = np.polynomial.legendre.leggauss(n)
    np.testing.assert_allclose(x, xr, atol=1e-15)
    np.testing.assert_allclose(w, wr, atol=1e-15)


@pytest.mark.parametrize("n,rem", [(2, 8 / 45), (4, 128 / 11025), (7, 512 / 2760615)])
def test_gauss_legendre_remainders(n, rem):
    """The remainders the kernels add for a top term y^(2n), 2^(2n+1) (n!)^4 /
    ((2n+1) ((2n)!)^2, against the device rule applied to y^(2n) and to a
    polynomial of degree 2n + 1 with random coefficients."""
    x, w = (np.asarray(v) for v in L.cp_gauss_legendre(n))
    f = math.factorial
    assert rem == pytest.approx(2 ** (2 * n + 1) * f(n) ** 4 / ((2 * n + 1) * f(2 * n) ** 2), rel=1e-15)
    assert 2 / (2 * n + 1) - np.dot(w, x ** (2 * n)) == pytest.approx(rem, rel=1e-12)
    c = np.random.default_rng(n).normal(size=2 * n + 2)
    exact = sum(c[k] * 2 / (k + 1) for k in range(0, 2 * n + 2, 2))
    rule = np.dot(w, np.polynomial.polynomial.polyval(x, c))
    assert rule + rem * c[2 * n] == pytest.approx(exact, rel=1e-13, abs=1e-14)


def test_gauss_legendre_rejects_other_sizes():
    with pytest.raises(L.CPError):
        L.cp_gauss_legendre(9)


def test_n_params():
    assert L.cp_n_params(L.CP_UNIFORM, 0) == 2
    assert L.cp_n_params(L.CP_EPANECHNIKOV, 0) == 2
    assert L.cp_n_params(L.CP_HISTOGRAM, 10) == 12
    assert L.cp_n_params(L.CP_MVGAUSS, 0) == 16
    assert L.cp_n_params(L.CP_HISTOGRAM, 0) == -1
    assert L.cp_n_params(9, 0) == -1


def desc(**kw):
    d = dict(height=4, width=5, row_stride=0, model=L.CP_UNIFORM, dtype=L.CP_F32, nbins=0, nsamples=0, seed=0,
             field_id=0, estimator=0)
    d.update(kw)
    return L.cp_field_desc_t(**d)


FAKE = 0x1000  # never dereferenced: every case below fails validation first


@pytest.mark.parametrize("kw,status", [
    (dict(height=0), L.CP_EINVAL),
    (dict(width=-1), L.CP_EINVAL),
    (dict(model=7), L.CP_EINVAL),
    (dict(dtype=3), L.CP_EINVAL),
    (dict(row_stride=3), L.CP_EINVAL),
    (dict(model=L.CP_HISTOGRAM, nbins=0), L.CP_EINVAL),
    (dict(model=L.CP_HISTOGRAM, nbins=33), L.CP_EINVAL),
    (dict(model=L.CP_MVGAUSS, dtype=L.CP_F64, nsamples=8), L.CP_EUNSUPPORTED),
    (dict(model=L.CP_MVGAUSS, nsamples=0), L.CP_EINVAL),
    (dict(model=L.CP_MVGAUSS, nsamples=8, estimator=5), L.CP_EINVAL),
])
def test_descriptor_validation(kw, status):
    assert L.cp_prob_forward(desc(**kw), FAKE, FAKE, FAKE, None) == status
    assert L.load().cp_last_error().decode() != ""


def test_null_pointers_rejected():
    assert L.cp_prob_forward(desc(), None, FAKE, FAKE, None) == L.CP_EINVAL
    assert L.cp_prob_backward(desc(), FAKE, None, FAKE, FAKE, None) == L.CP_EINVAL
    assert L.cpu_fit_params(desc(), None, 3, None, FAKE, None) == L.CP_EINVAL
    assert L.cpu_fit_params(desc(), FAKE, 0, None, FAKE, None) == L.CP_EINVAL
    assert L.load().cp_prob_forward(None, FAKE, FAKE, FAKE, None) == L.CP_EINVAL


def test_fit_forward_argument_errors():
    """cp_fit_forward rejects what either of cpu_fit_params and cp_prob_forward
    rejects, before anything is launched."""
    assert L.cp_fit_forward(desc(), None, 3, None, FAKE, FAKE, FAKE, None) == L.CP_EINVAL
    assert L.cp_fit_forward(desc(), FAKE, 3, None, None, FAKE, FAKE, None) == L.CP_EINVAL
    assert L.cp_fit_forward(desc(), FAKE, 3, None, FAKE, None, FAKE, None) == L.CP_EINVAL
    assert L.cp_fit_forward(desc(), FAKE, 3, None, FAKE, FAKE, None, None) == L.CP_EINVAL
    assert L.cp_fit_forward(desc(), FAKE, 0, None, FAKE, FAKE, FAKE, None) == L.CP_EINVAL
    assert L.cp_fit_forward(desc(height=0), FAKE, 3, None, FAKE, FAKE, FAKE, None) == L.CP_EINVAL
    bad = L.cp_fit_opts_t(-1, 1.06, 1e-6, 0.0)
    assert L.cp_fit_forward(desc(), FAKE, 3, bad, FAKE, FAKE, FAKE, None) == L.CP_EDOMAIN
    # the Gaussian forward needs samples
    assert L.cp_fit_forward(desc(model=L.CP_MVGAUSS), FAKE, 3, None, FAKE, FAKE, FAKE, None) == L.CP_EINVAL


def test_fit_option_validation():
    bad = L.cp_fit_opts_t(-1, 1.06, 1e-6, 0.0)
    assert L.cpu_fit_params(desc(), FAKE, 3, bad, FAKE, None) == L.CP_EDOMAIN
    bad = L.cp_fit_opts_t(3, 1.06, 1e-6, 0.0)
    assert L.cpu_fit_params(desc(model=L.CP_EPANECHNIKOV), FAKE, 3, bad, FAKE, None) == L.CP_EDOMAIN
    assert L.cpu_fit_params(desc(model=L.CP_MVGAUSS, nsamples=4), FAKE, 1, None, FAKE, None) == L.CP_EDOMAIN


def test_batched_validation():
    d = [desc(), desc(dtype=L.CP_F64)]
    assert L.cp_prob_batched(2, d, [FAKE, FAKE], [FAKE] * 2, [FAKE] * 2, None, None, None, L.CP_BATCH_FWD,
                             None) == L.CP_EINVAL
    d = [desc(model=L.CP_MVGAUSS, nsamples=4)]
    assert L.cp_prob_batched(1, d, [FAKE], [FAKE], [FAKE], None, None, None, L.CP_BATCH_FWD,
                             None) == L.CP_EUNSUPPORTED
    assert L.cp_prob_batched(1, [desc()], [FAKE], [FAKE], [FAKE], None, None, None, 0, None) == L.CP_EINVAL
    assert L.cp_prob_batched(1, [desc()], [FAKE], None, None, None, None, None, L.CP_BATCH_FWD,
                             None) == L.CP_EINVAL
    assert L.cp_prob_batched(1, [desc()], [FAKE], [FAKE], [FAKE], None, None, None, L.CP_BATCH_BWD,
                             None) == L.CP_EINVAL


def test_batched_tune_flag_and_describe_without_a_plan():
    # the tune flag is a known bit (validation stops at the NULL table first)
    assert L.cp_prob_batched(1, [desc()], [FAKE], None, None, None, None, None,
                             L.CP_BATCH_FWD | L.CP_BATCH_TUNE, None) == L.CP_EINVAL
    assert "NULL" in L.load().cp_last_error().decode()
    assert L.cp_prob_batched(1, [desc()], [FAKE], [FAKE], [FAKE], None, None, None, 32 | L.CP_BATCH_FWD,
                             None) == L.CP_EINVAL
    assert "flag" in L.load().cp_last_error().decode()
    # pin: argument checks come before any device call
    sh, ch = [0] * 5, [1] * 5
    assert L.cp_batched_pin(1, [desc()], 0, sh, ch) == L.CP_EINVAL
    assert L.cp_batched_pin(1, [desc(height=0)], L.CP_BATCH_FWD, sh, ch) == L.CP_EINVAL
    assert L.cp_batched_pin(1, [desc(model=L.CP_MVGAUSS, nsamples=4)], L.CP_BATCH_FWD, sh, ch) == L.CP_EUNSUPPORTED
    assert L.load().cp_batched_pin(1, None, L.CP_BATCH_FWD, None, None) == L.CP_EINVAL
    # no plan has been built for these shapes, and bad descriptors give none
    assert L.cp_batched_describe(1, [desc(height=3, width=3)], L.CP_BATCH_FWD) is None
    assert L.cp_batched_describe(1, [desc(height=0)], L.CP_BATCH_FWD) is None


def test_classify_validation():
    lib = L.load()
    assert lib.cp_prob_classify(desc(), None, FAKE, FAKE, FAKE, FAKE, FAKE, None) == L.CP_EINVAL
    assert lib.cp_prob_classify(desc(), FAKE, None, None, None, None, None, None) == L.CP_EINVAL
    assert lib.cp_prob_classify(desc(height=0), FAKE, FAKE, None, None, None, None, None) == L.CP_EINVAL
    assert lib.cp_prob_classify(desc(model=L.CP_MVGAUSS, nsamples=4), FAKE, FAKE, None, None, None, None,
                                None) == L.CP_EUNSUPPORTED
    assert lib.cp_last_error().decode() != ""


def test_error_bound_fit_validation():
    lib = L.load()
    assert lib.cp_fit_error_bound(desc(), None, 1.0, FAKE, None) == L.CP_EINVAL
    assert lib.cp_fit_error_bound(desc(model=L.CP_EPANECHNIKOV), FAKE, 1.0, FAKE, None) == L.CP_EUNSUPPORTED
    for eb in (0.0, -1.0, float("nan"), float("inf"), 1e39):
        assert lib.cp_fit_error_bound(desc(), FAKE, eb, FAKE, None) == L.CP_EDOMAIN


def test_binding_covers_every_call_of_the_torch_layer():
    """Every L.<name> the torch layer calls exists in the binding module."""
    import re
    src = open(os.path.join(ROOT, "paper_2407_18015_amd", "ops.py")).read()
    for name in set(re.findall(r"\bL\.(cp\w+)\(", src)):
        assert callable(getattr(L, name, None)), name
    for name in L.EXPORTS:
        if name not in ("cp_status_string", "cp_last_error"):
            assert callable(getattr(L, name, None)), name


def test_semianalytical_validation():
    lib = L.load()
    h = dict(model=L.CP_HISTOGRAM, nbins=4, nsamples=8)
    assert lib.cp_prob_semianalytical(desc(**h), None, FAKE, FAKE, None, None) == L.CP_EINVAL
    assert lib.cp_prob_semianalytical(desc(**h), FAKE, None, None, None, None) == L.CP_EINVAL
    assert lib.cp_prob_semianalytical(desc(model=L.CP_HISTOGRAM, nbins=4, nsamples=0), FAKE, FAKE, FAKE, None,
                                      None) == L.CP_EINVAL
    assert lib.cp_prob_semianalytical(desc(), FAKE, FAKE, FAKE, None, None) == L.CP_EUNSUPPORTED


def test_status_strings():
    lib = L.load()
    for s in range(6):
        assert lib.cp_status_string(s)


def test_product_package_does_not_reference_the_oracle():
    pkg = os.path.join(ROOT, "paper_2407_18015_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".cpp", ".h")):
                text = open(os.path.join(dirpath, fn)).read()
                assert "import oracle" not in text and "from oracle" not in text and "cp_oracle" not in text, fn
