"""The library's host-callable code under AddressSanitizer and
UndefinedBehaviorSanitizer on the CPU: the per-vertex routines of the
closed-form kernels (vertex_fwd_ue, vertex_jac_vals, hist_vertex_minmax,
hist_stencil_jac) and the gather of their Jacobians, built host-only from the
library's own headers and run on small seeded fields, are compared with the
oracle; the adjoint-buffer bookkeeping (one buffer per device and stream,
grown buffers retired until release) is exercised with a counting
allocator.  A sanitizer report fails the run."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "helpers", "host_checks.cpp")
U, E, HST = oracle.UNIFORM, oracle.EPANECHNIKOV, oracle.HISTOGRAM
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:halt_on_error=1",
           UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    clang = "/opt/rocm/llvm/bin/clang++"
    if not (os.path.exists(hipcc) and os.path.exists(clang)):
        pytest.skip("no HIP compiler")
    d = tmp_path_factory.mktemp("host_checks")
    obj, exe = str(d / "host_checks.o"), str(d / "host_checks")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", os.path.join(ROOT, "paper_2407_18015_amd", "csrc")]
    # host pass only (no device code is built); the sanitizers apply to it
    subprocess.run([hipcc, "-xhip", "--offload-host-only", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
                    "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                    "-Xarch_host", "-fno-sanitize-recover=undefined", *inc, "-c", SRC, "-o", obj], check=True)
    subprocess.run([clang, "-fsanitize=address,undefined", obj, "-o", exe], check=True)
    return exe


def run(exe, *args):
    r = subprocess.run([exe, *args], capture_output=True, text=True, env=ENV, timeout=300)
    assert r.returncode == 0 and "Sanitizer" not in r.stderr and "runtime error" not in r.stderr, r.stderr[-4000:]
    return r


def test_workspace_bookkeeping(checker):
    assert "pool ok" in run(checker, "pool").stdout


@pytest.mark.parametrize("model,nb", [(U, 0), (E, 0), (HST, 5), (HST, 10)])
@pytest.mark.parametrize("dtype", [np.float64, np.float32])
def test_per_vertex_routines_against_oracle(checker, tmp_path, model, nb, dtype):
    H, W = 23, 37
    p = workloads.random_params(model, 70 + model + nb, H, W, nbins=nb, width=0.06).astype(dtype)
    # invalid distributions in two places (NaN stencils must match the oracle's)
    p[0, 5, 7] = np.nan
    if model == E:
        p[1, 11, 0] = 0.0  # zero width
    else:
        p[1, 11, 0] = p[0, 11, 0]  # empty range
    g1, g2 = (g.astype(dtype) for g in workloads.upstream(9, H, W))
    p64, g1, g2 = p.astype(np.float64), g1.astype(np.float64), g2.astype(np.float64)
    fin, fout = tmp_path / "in.bin", tmp_path / "out.bin"
    with open(fin, "wb") as fh:
        fh.write(np.array([model, 1 if dtype == np.float64 else 0, H, W, nb], dtype=np.int32).tobytes())
        fh.write(np.ascontiguousarray(p64).tobytes())
        fh.write(np.ascontiguousarray(g1).tobytes())
        fh.write(np.ascontiguousarray(g2).tobytes())
    run(checker, "field", str(fin), str(fout))
    out = np.fromfile(fout, dtype=np.float64).reshape(2 + p.shape[0], H, W)
    # the stencils that contain an invalid vertex give NaN probabilities; the
    # gradient is NaN wherever one of those stencils contributes (distance 2)
    bad = np.zeros((H, W), bool)
    for y, x in ((5, 7), (11, 0)):
        for dy, dx in ((0, 0), (0, 1), (-1, 0), (0, -1), (1, 0)):
            if 0 <= y + dy < H and 0 <= x + dx < W:
                bad[y + dy, x + dx] = True
    gbad = bad.copy()
    for y, x in np.argwhere(bad):
        for dy, dx in ((0, 1), (-1, 0), (0, -1), (1, 0)):
            if 0 <= y + dy < H and 0 <= x + dx < W:
                gbad[y + dy, x + dx] = True
    assert np.array_equal(np.isnan(out[0]), bad) and np.array_equal(np.isnan(out[1]), bad)
    gplanes = out[2:] if model != HST else out[4:]
    assert np.array_equal(np.isnan(gplanes).any(axis=0), gbad)
    # valid stencils against the oracle, on a copy with the invalid vertices
    # replaced by valid distributions (they only reach the masked outputs)
    q = p64.copy()
    q[:, 5, 7] = q[:, 5, 6]
    q[:, 11, 0] = q[:, 11, 1]
    rmin, rmax = oracle.forward(model, q)
    tol = 1e-12 if dtype == np.float64 else 1e-6
    for got, ref in ((out[0], rmin), (out[1], rmax)):
        assert np.max(np.abs(got - ref)[~bad]) <= tol
    rg = oracle.grad(model, q, g1, g2)
    S = oracle.grad(model, q, g1, g2, absolute=True)
    if dtype == np.float64:
        bound = 1e-10 * (1 + np.abs(rg)) + 1e-13 * S
    else:
        bound = 1e-5 * (1 + np.abs(rg)) + 5e-7 * S
    ok = (np.abs(out[2:] - rg) <= bound) | gbad[None]
    assert np.all(ok), float(np.max((np.abs(out[2:] - rg) - bound)[~ok]))
