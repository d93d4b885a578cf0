"""Host-side pieces of the benchmark: the one-GPU guard and the piece
counts behind the algorithmic FLOP figure of the roofline (no GPU)."""
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_piece_counts_of_hand_cases():
    """Pieces per side follow the started-neighbour structure: a lone vertex
    has only piece 0 on each side; two identical neighbours start together at
    the vertex's lower end, so each side is one piece with one factor; a
    neighbour entirely above the vertex leaves only piece 0 for P_min and no
    piece at all for P_max."""
    lone = np.array([[[0.3]], [[0.1]]])
    assert bench.epa_piece_counts(lone).tolist() == [2, 0, 0, 0, 0]
    pair = np.array([[[0.3, 0.3]], [[0.1, 0.1]]])
    assert bench.epa_piece_counts(pair).tolist() == [0, 4, 0, 0, 0]
    apart = np.array([[[0.0, 1.0]], [[0.1, 0.1]]])
    # vertex 0: min side piece 0 only (neighbour starts above its support);
    # max side empty (the neighbour is always larger).  Vertex 1 mirrors it.
    assert bench.epa_piece_counts(apart).tolist() == [2, 0, 0, 0, 0]


def test_piece_counts_match_a_per_vertex_count():
    """The vectorised count against a plain loop over vertices and sides."""
    rng = np.random.default_rng(3)
    H, W = 7, 9
    p = np.stack([rng.normal(0, 0.05, (H, W)), rng.uniform(0.02, 0.08, (H, W))])
    ref = np.zeros(5, dtype=np.int64)
    for y in range(H):
        for x in range(W):
            m, w = p[0, y, x], p[1, y, x]
            nb = [(y + dy, x + dx) for dy, dx in ((0, 1), (-1, 0), (0, -1), (1, 0))
                  if 0 <= y + dy < H and 0 <= x + dx < W]
            for sign in (1.0, -1.0):
                d = [sign * (p[0, yy, xx] - m) for yy, xx in nb]
                wn = [p[1, yy, xx] for yy, xx in nb]
                bmin = min([w] + [di + wi for di, wi in zip(d, wn)])
                if not bmin > -w:
                    continue
                starts = sorted([min(max(di - wi, -w), bmin) for di, wi in zip(d, wn)] + [bmin] * (4 - len(nb)))
                edges = [-w] + starts + [bmin]
                for k in range(5):
                    ref[k] += edges[k + 1] > edges[k]
    assert bench.epa_piece_counts(p).tolist() == ref.tolist()


def test_uniform_piece_counts_match_a_per_vertex_count():
    """Uniform pieces: vertex support [0, Lv] from its lower end (minimum) or
    reflected from its upper end (maximum), against a plain loop."""
    rng = np.random.default_rng(4)
    H, W = 6, 8
    c = rng.normal(0, 0.05, (H, W))
    hw = rng.uniform(0.02, 0.08, (H, W))
    p = np.stack([c - hw, c + hw])
    ref = np.zeros(5, dtype=np.int64)
    for y in range(H):
        for x in range(W):
            lo, hi = p[0, y, x], p[1, y, x]
            nb = [(y + dy, x + dx) for dy, dx in ((0, 1), (-1, 0), (0, -1), (1, 0))
                  if 0 <= y + dy < H and 0 <= x + dx < W]
            for side in (0, 1):
                if side == 0:
                    ab = [(p[0, yy, xx] - lo, p[1, yy, xx] - lo) for yy, xx in nb]
                else:
                    ab = [(hi - p[1, yy, xx], hi - p[0, yy, xx]) for yy, xx in nb]
                bmin = min([hi - lo] + [b for _, b in ab])
                if not bmin > 0:
                    continue
                starts = sorted([min(max(a, 0.0), bmin) for a, _ in ab] + [bmin] * (4 - len(nb)))
                edges = [0.0] + starts + [bmin]
                for k in range(5):
                    ref[k] += edges[k + 1] > edges[k]
    assert bench.uni_piece_counts(p).tolist() == ref.tolist()


def test_histogram_interval_count_matches_a_per_vertex_count():
    """Sub-intervals of the merged sweep: 1 + distinct bin edges of the five
    histograms strictly inside the vertex range, against a plain loop in
    the same FP32 vertex frame."""
    import workloads
    nb = 4
    p = workloads.random_params(2, 5, 5, 7, nbins=nb).astype(np.float32)
    H, W = p.shape[1:]
    total = 0
    for y in range(H):
        for x in range(W):
            lo = p[0, y, x]
            hv = np.float32(p[1, y, x] - lo)
            edges = {float(np.float32(k) * np.float32(hv * np.float32(1.0 / nb))) for k in range(1, nb)}
            for dy, dx in ((0, 1), (-1, 0), (0, -1), (1, 0)):
                yy, xx = y + dy, x + dx
                if 0 <= yy < H and 0 <= xx < W:
                    a = np.float32(p[0, yy, xx] - lo)
                    b = np.float32(p[1, yy, xx] - lo)
                    d = np.float32((b - a) * np.float32(1.0 / nb))
                    edges |= {float(np.float32(a + np.float32(k) * d)) for k in range(nb + 1)}
            total += 1 + sum(1 for e in edges if 0 < e < hv)
    assert bench.hist_interval_count(p, nb) == total
    # a lone vertex: its own h - 1 interior edges, h intervals
    assert bench.hist_interval_count(np.array([[[0.0]], [[1.0]]] + [[[0.25]]] * 4, dtype=np.float32), 4) == 4
