#!/usr/bin/env python
"""Benchmark of the critical-point probability hot path on one MI355X.

Step (the quoted workload): Epanechnikov model on a 2048 x 2048 grid with 20
ensemble members per vertex (smooth base field + box-smoothed noise): fit the
per-vertex (centre, half-width) from the members, forward P_min / P_max, and
the adjoint dP/dtheta for seeded upstream gradients -- every row of the hot
path for that workload, inputs resident in HBM.

Prints one JSON line.  `value` = grid vertices processed per second by the
whole step.  `detail` carries per-stage and per-model rates (uniform FP64
64^2, uniform / histogram 2048^2, Gaussian Monte Carlo 1024^2 x 4096 samples,
batched 64 fields vs one launch per field); `roofline` describes the
dominant kernel; `cpu_baseline` times the FP64 oracle on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

METRIC = "vertex-probabilities/s (fwd, fwd+bwd) per model; batched vs plain at 1e-6 abs err"
UNIT = "vertex-probabilities/s"
# MI355X published FP32 vector peak.  No packed FP32 instruction is
# generated here, and yet plain FMAs reach it within ~15% when a wave has
# eight or more independent FMAs in flight (the FMA probe of libcpprobes.so,
# measured in every run: `detail.ceilings.fp32_fma_tflops_by_chains`); with
# four or fewer the rate stays near 256 CUs x 64 lanes x 2 x 2.4 GHz =
# 78.6 TFLOP/s, the single-issue rate, reported beside it.
PEAK_FP32 = 157.3e12
RATE_FP32_SINGLE_ISSUE = 256 * 64 * 2 * 2.4e9
PEAK_HBM = 8e12

# HBM bytes of one launch of the Epanechnikov FP32 adjoint at 2048^2, from
# two rocprofv3 --pmc passes (FETCH_SIZE, WRITE_SIZE, KiB per dispatch) over
# `bench.py --profile-only`, each scaled by the same counter on a plain
# 256 MiB copy (FETCH_SIZE read 128 MiB: x2; WRITE_SIZE 256 MiB: x1).  They
# describe the machine code whose instruction hash is recorded here (the
# build writes every closed-form kernel's hash to libcpcrit.isa.json) and are
# reported as null once the built kernel differs.
ADJOINT_PMC = {
    "fetch_kib": 33534.1, "write_kib": 32779.2, "fetch_scale": 2.0, "write_scale": 1.0, "grid": [2048, 2048],
    "kernel": "_ZN2cp8k_bwd_ueIfLi1ELi30ELi30EEEvNS_9FieldPtrsIT_EEii",
    "isa_sha256": "3ba599891565b80b52bf4840d92997bd3d7e72aa5fdc273c503787dbef36e820",
}


def adjoint_traffic(size: int = 2048):
    m = ADJOINT_PMC
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2407_18015_amd", "libcpcrit.isa.json")
    try:
        with open(path) as fh:
            built = json.load(fh).get(m["kernel"])
    except (OSError, ValueError):
        built = None
    if [size, size] != m["grid"] or built != m["isa_sha256"]:
        return None
    return (m["fetch_kib"] * m["fetch_scale"] + m["write_kib"] * m["write_scale"]) * 1024


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # the GPU reaches its sustained clocks only after ~100 ms of load: the
    # default warm-up (~0.1 s of steps) lets the timed steps run at them
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=300)
    ap.add_argument("--size", type=int, default=2048)
    ap.add_argument("--no-detail", action="store_true", help="only the quoted step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--profile-only", action="store_true",
                    help="run the quoted step only (for rocprofv3), no JSON detail")
    ap.add_argument("--profile-histogram", action="store_true",
                    help="for rocprofv3: the 2048^2 x 10-bin histogram forward and adjoint, --steps times after "
                         "--warmup, then a plain copy of known size (no JSON)")
    return ap.parse_args()


# ----------------------------------------------------------------------------
# algorithmic work of the Epanechnikov kernels: FLOPs of the kernels'
# formulation per non-empty piece with k started neighbours at the quadrature
# order n_k (FMA = 2); redundant work (empty pieces, halo ring, masked lanes,
# sorting) is not counted.  Pieces with k = 2 and 4 take n_k = (3k + 2) / 2
# nodes plus the rule's closed-form remainder on the top-degree terms.
#   forward piece k:  setup 6 + 3k; per node 6 + 7k (node, vertex pdf, per
#                     factor u, 4 S(u) and the product); 3 to accumulate;
#                     remainder 3 + 3k.  Piece 0 (vertex CDF in closed
#                     form): 6.
#   adjoint piece k:  setup 6 + 3k; per node 4 + 15k (node, weight x pdf,
#                     per factor u, 4 S(u), prefix / suffix products, the
#                     leave-one-out product times (1 - u^2), two moments);
#                     4k to accumulate; remainder 2 + 4k.  Piece 0 needs no
#                     adjoint work.  Per vertex 8 for the gather of the five
#                     stencils.
# ----------------------------------------------------------------------------
GL_NODES = {1: 3, 2: 4, 3: 6, 4: 7}  # rule for a piece with k started neighbours
GL_REM = {1: False, 2: True, 3: False, 4: True}  # plus the remainder term


def flops_fwd_piece(k):
    if k == 0:
        return 6
    return 9 + 3 * k + GL_NODES[k] * (6 + 7 * k) + (3 + 3 * k if GL_REM[k] else 0)


def flops_bwd_piece(k):
    if k == 0:
        return 0
    return 6 + 7 * k + GL_NODES[k] * (4 + 15 * k) + (2 + 4 * k if GL_REM[k] else 0)


def _torch(a):
    import torch
    return a if isinstance(a, torch.Tensor) else torch.as_tensor(np.asarray(a))


def _nbrs(a, fill=float("nan")):
    """e, n, w, s neighbour planes of a [H, W] tensor (`fill` outside the grid)."""
    import torch
    p = torch.nn.functional.pad(a[None, None], (1, 1, 1, 1), value=fill)[0, 0]
    return [p[1:-1, 2:], p[:-2, 1:-1], p[1:-1, :-2], p[2:, 1:-1]]


def _side_pieces(lower, bmin, starts):
    """Non-empty pieces by started-neighbour count of one side: support from
    `lower`, end bmin, clamped neighbour starts (absent: bmin)."""
    import torch
    c = torch.sort(torch.stack(starts), dim=0).values
    ok = bmin > lower
    edges = torch.cat([lower[None], c, bmin[None]])
    return np.array([int(((edges[k + 1] > edges[k]) & ok).sum()) for k in range(5)], dtype=np.int64)


def epa_piece_counts(params) -> np.ndarray:
    """counts[k] = number of non-empty pieces with k started neighbours over
    all vertices and both sides (minimum, and maximum by reflection)."""
    import torch
    p = _torch(params).to(torch.float64)
    m, w = p[0], p[1]
    mn, wn = _nbrs(m), _nbrs(w)
    counts = np.zeros(5, dtype=np.int64)
    for sign in (1.0, -1.0):
        d = [sign * (x - m) for x in mn]
        bmin = w.clone()
        for di, wi in zip(d, wn):
            bmin = torch.where(torch.isfinite(di), torch.minimum(bmin, di + wi), bmin)
        starts = [torch.where(torch.isfinite(di), torch.minimum(torch.maximum(di - wi, -w), bmin), bmin)
                  for di, wi in zip(d, wn)]
        counts += _side_pieces(-w, bmin, starts)
    return counts


def uni_piece_counts(params) -> np.ndarray:
    """As epa_piece_counts for the uniform model: vertex support [0, Lv]
    from its lower end (minimum) or reflected from its upper end (maximum)."""
    import torch
    p = _torch(params).to(torch.float64)
    lo, hi = p[0], p[1]
    lon, hin = _nbrs(lo), _nbrs(hi)
    zero = torch.zeros_like(lo)
    counts = np.zeros(5, dtype=np.int64)
    for side in (0, 1):
        a = [(ln - lo) if side == 0 else (hi - hn) for ln, hn in zip(lon, hin)]
        b = [(hn - lo) if side == 0 else (hi - ln) for ln, hn in zip(lon, hin)]
        bmin = hi - lo
        for bi in b:
            bmin = torch.where(torch.isfinite(bi), torch.minimum(bmin, bi), bmin)
        starts = [torch.where(torch.isfinite(ai), torch.minimum(torch.maximum(ai, zero), bmin), bmin) for ai in a]
        counts += _side_pieces(zero, bmin, starts)
    return counts


def hist_interval_count(params, nbins: int, rows: int = 128) -> int:
    """Sub-intervals the histogram sweep integrates, over all vertices: per
    vertex 1 + the number of distinct bin edges of the five histograms
    strictly inside the vertex range (vertex frame, FP32 as in the kernel)."""
    import torch
    p = _torch(params).to(torch.float32)
    lo, hi = p[0], p[1]
    lon, hin = _nbrs(lo), _nbrs(hi)
    H = lo.shape[0]
    k = torch.arange(nbins + 1, dtype=torch.float32, device=lo.device)
    kv = torch.arange(1, nbins, dtype=torch.float32, device=lo.device)
    total = 0
    for r0 in range(0, H, rows):
        r1 = min(H, r0 + rows)
        lv, hv = lo[r0:r1].reshape(-1), (hi[r0:r1] - lo[r0:r1]).reshape(-1)
        cols = [kv[None, :] * (hv * (1.0 / nbins))[:, None]]
        for ln, hn in zip(lon, hin):
            a = ln[r0:r1].reshape(-1) - lv
            b = hn[r0:r1].reshape(-1) - lv
            cols.append(a[:, None] + k[None, :] * ((b - a) * (1.0 / nbins))[:, None])
        e = torch.cat(cols, dim=1)
        e = torch.where((e > 0) & (e < hv[:, None]), e, torch.full_like(e, float("inf")))
        e = torch.sort(e, dim=1).values
        fin = torch.isfinite(e)
        new = fin.clone()
        new[:, 1:] &= e[:, 1:] != e[:, :-1]
        valid = hv > 0
        total += int(((new.sum(dim=1) + 1) * valid).sum())
    return total


def epa_flops(params):
    c = epa_piece_counts(params)
    fwd = sum(int(c[k]) * flops_fwd_piece(k) for k in range(5))
    bwd = sum(int(c[k]) * flops_bwd_piece(k) for k in range(5)) + 8 * params.shape[1] * params.shape[2]
    return fwd, bwd, c


# ----------------------------------------------------------------------------
# uniform model, same convention (uni_piece / uni_piece_grad): a piece with k
# started neighbours is integrated exactly with 1, 1, 2, 2 nodes (k = 1..4),
# k = 2 and 4 with the rule's remainder on the top-degree term (k + 1).
#   forward piece k:  setup 4 + 3k (midpoint, half-length, per factor slope
#                     and offset); per node 3k + 1 (k factors, product,
#                     weighted sum); 2 to scale and accumulate.  Piece 0: 0.
#   adjoint piece k:  setup 4 + 3k; per node 7k (factors, prefix and suffix
#                     products, full product, k leave-one-out products
#                     accumulated); 1 + 2k to scale and accumulate.
#   adjoint per vertex: 2 x 27 (each side's sums of the active integrals and
#                     the lo / hi / width partials), 30 to weight the ten
#                     Jacobian entries by g_min / g_max, 8 for the gather.
# ----------------------------------------------------------------------------
UNI_NODES = {1: 1, 2: 1, 3: 2, 4: 2}
UNI_REM = {1: 0, 2: 3, 3: 0, 4: 5}  # remainder FLOPs (k = 2, 4)
UNI_BWD_VERTEX = 2 * 27 + 30 + 8


def flops_uni_fwd_piece(k):
    return 0 if k == 0 else 6 + 3 * k + UNI_NODES[k] * (3 * k + 1) + UNI_REM[k]


def flops_uni_bwd_piece(k):
    return 0 if k == 0 else 5 + 5 * k + UNI_NODES[k] * 7 * k + UNI_REM[k]


def uni_flops(params):
    c = uni_piece_counts(params)
    nv = params.shape[1] * params.shape[2]
    fwd = sum(int(c[k]) * flops_uni_fwd_piece(k) for k in range(5)) + 2 * nv
    bwd = sum(int(c[k]) * flops_uni_bwd_piece(k) for k in range(5)) + UNI_BWD_VERTEX * nv
    return fwd, bwd, c


# ----------------------------------------------------------------------------
# histogram model (cp_hist.hpp, cp_hist_bwd.hpp), per sub-interval of the
# merged sweep (both sides at once):
#   forward 88:  end values of the four survival functions (12) and CDFs
#                (4), interval weight (2), two exact integrals of a product
#                of four linear factors from their end values (2 x 31), two
#                accumulations (4), advancing the edge that ends it (4).
#   adjoint 163: midpoint, half-length, node offset and weight scales (8);
#                per Gauss-Legendre node (2) 60 (node, four S and F values,
#                pair products, vertex-slot sums, upstream-weighted
#                leave-one-out products for both sides and their plain and
#                bin-kernel-weighted sums); the rule's degree-4 remainder
#                from the four slopes (25); 10 to emit the entry of the edge
#                that ends it and advance that edge.  Per vertex 9h: the
#                closing pass over each neighbour's bins and the gather of
#                five stencils' entries.
# ----------------------------------------------------------------------------
HIST_FWD_INTERVAL = 88
HIST_BWD_INTERVAL = 163


def hist_flops(params, nbins: int):
    n = hist_interval_count(params, nbins)
    nv = params.shape[1] * params.shape[2]
    return HIST_FWD_INTERVAL * n, HIST_BWD_INTERVAL * n + 9 * nbins * nv, n


def roofline(bound: str, work: float, seconds: float, peak: float, unit: str, **extra) -> dict:
    """One roofline object: `work` algorithmic FLOPs (or bytes, or samples)
    per launch over the launch time, against `peak` (same unit per second,
    scaled by 1e12 for TFLOP/s and TB/s)."""
    scale = {"TFLOP/s": 1e12, "TB/s": 1e12, "GB/s": 1e9, "G samples/s": 1e9}[unit]
    achieved = work / seconds / scale
    out = {"bound": bound, "achieved": achieved, "peak": peak / scale, "unit": unit, "frac": achieved * scale / peak,
           "work_per_launch": work, "launch_us": seconds * 1e6}
    out.update(extra)
    return out


# ----------------------------------------------------------------------------
def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU: there is no multi-GPU path (a field shards by rows with a "
              "one- or two-row halo, a batch by field with no communication).  Run with --gpus 1.",
              file=sys.stderr)
        sys.exit(2)
    import torch

    import paper_2407_18015_amd as cp
    import workloads

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    S = args.size
    if args.profile_histogram:
        profile_histogram(cp, workloads, torch, dev, S, args.steps, args.warmup)
        return
    t0 = time.time()
    mem_np = workloads.smooth_ensemble(0, S, S)
    gmin_np, gmax_np = workloads.upstream(0, S, S)
    print(f"[bench] inputs generated in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    mem = torch.as_tensor(mem_np, device=dev)
    gmin = torch.as_tensor(gmin_np, device=dev)
    gmax = torch.as_tensor(gmax_np, device=dev)
    E = 1
    f = cp.Field(S, S, E, torch.float32)
    params = torch.empty((2, S, S), device=dev)
    pmin = torch.empty((S, S), device=dev)
    pmax = torch.empty((S, S), device=dev)
    grad = torch.empty((2, S, S), device=dev)

    # the step: fit and forward in one launch (cp_fit_forward), then the adjoint
    def step():
        cp.fit_forward(mem, E, out=params, pmin=pmin, pmax=pmax)
        cp.backward(params, gmin, gmax, f, grad)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # timed region: K steps, each launch bracketed by HIP events on the stream
    # the kernels run on (torch's current stream), so per-kernel durations are
    # measured inside the step sequence (cold caches after the member reads)
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    for e in evs:
        e[0].record()
        cp.fit_forward(mem, E, out=params, pmin=pmin, pmax=pmax)
        e[1].record()
        cp.backward(params, gmin, gmax, f, grad)
        e[2].record()
    torch.cuda.synchronize()
    ms = evs[0][0].elapsed_time(evs[-1][2]) / args.steps
    t_ff, t_bwd = (sum(e[k].elapsed_time(e[k + 1]) for e in evs) / args.steps for k in range(2))
    value = S * S / (ms * 1e-3)
    print(f"[bench] step {ms:.3f} ms (fit + forward {t_ff * 1e3:.1f} us, adjoint {t_bwd * 1e3:.1f} us)",
          file=sys.stderr, flush=True)
    if args.profile_only:
        # a plain copy of known size (256 MiB read + 256 MiB written): the
        # reference that scales the HBM byte counters of the kernels above
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        return

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    reps = min(50, max(5, args.steps))
    # the fit and the forward as separate launches (their own rooflines)
    t_fit = timed(lambda: cp.fit(mem, E, out=params), reps)
    t_fwd = timed(lambda: cp.forward(params, f, pmin, pmax), reps)
    # forward and adjoint in one launch, for callers whose upstream gradients
    # are known before the forward (sensitivity maps of a fixed functional):
    # the adjoint tiles also write P_min / P_max (one-field batched call)
    t_fused = timed(lambda: cp.batched([f], [params], [pmin], [pmax], [gmin], [gmax], [grad], graph=True), reps)
    t_pipe = pipelined_step(cp, torch, mem, E, f, params, pmin, pmax, gmin, gmax, grad, reps)
    t_cls = timed(lambda: cp.classify(params, f), reps)
    t_sad = timed(lambda: cp.classify(params, f, outputs=("saddle",)), reps)
    fl_fwd, fl_bwd, counts = epa_flops(params)
    achieved = fl_bwd / (t_bwd * 1e-3)
    roof = {"bound": "alu", "kernel": "adjoint, Epanechnikov FP32 (k_bwd_ue<float,1,30,30>)",
            "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12, "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP32, "traffic": adjoint_traffic(S),
            "algorithmic_flops_per_launch": fl_bwd, "launch_us": t_bwd * 1e3,
            "single_issue_rate": RATE_FP32_SINGLE_ISSUE / 1e12,
            "frac_of_single_issue_rate": achieved / RATE_FP32_SINGLE_ISSUE,
            "algorithmic_bytes_per_launch": 24 * S * S}
    ceil = probe_ceilings(torch, dev)
    detail = {
        "ceilings": ceil,
        "epanechnikov_2048": {
            "roofline_fwd": roofline("alu", fl_fwd, t_fwd * 1e-3, PEAK_FP32, "TFLOP/s"),
            "roofline_bwd": roofline("alu", fl_bwd, t_bwd * 1e-3, PEAK_FP32, "TFLOP/s"),
            "roofline_fit": roofline("hbm", (20 * 4 + 8) * S * S, t_fit * 1e-3, PEAK_HBM, "TB/s"),
            # the fused fit + forward against both of its bounds at once
            "roofline_fit_forward_hbm": roofline("hbm", (20 * 4 + 8 + 8) * S * S, t_ff * 1e-3, PEAK_HBM, "TB/s"),
            "roofline_fit_forward_alu": roofline("alu", fl_fwd, t_ff * 1e-3, PEAK_FP32, "TFLOP/s"),
            "fit_forward_ms": t_ff, "fit_ms": t_fit, "fwd_ms": t_fwd, "bwd_ms": t_bwd,
            "fit_forward_vs_separate": (t_fit + t_fwd) / t_ff,
            "fwd_vertices_per_s": S * S / (t_fwd * 1e-3),
            "fwd_bwd_vertices_per_s": S * S / ((t_fwd + t_bwd) * 1e-3),
            "fwd_tflops": fl_fwd / (t_fwd * 1e-3) / 1e12, "bwd_tflops": fl_bwd / (t_bwd * 1e-3) / 1e12,
            "fit_hbm_gbs": (20 * 4 + 8) * S * S / (t_fit * 1e-3) / 1e9,
            "classify_ms": t_cls, "saddle_ms": t_sad,
            "fused_fwd_bwd_ms": t_fused, "fused_fwd_bwd_vertices_per_s": S * S / (t_fused * 1e-3),
            "pipelined_step_ms": t_pipe, "pipelined_step_vertices_per_s": S * S / (t_pipe * 1e-3),
            "pieces_by_started_neighbours": counts.tolist(),
        }
    }
    if not args.no_detail:
        detail.update(more_detail(cp, workloads, torch, dev, S, reps, ceil))

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(mem_np, gmin_np, gmax_np)

    out = {
        "metric": METRIC, "value": value, "unit": UNIT, "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"epanechnikov fit+forward (one launch) + adjoint, {S}x{S} grid, 20 members, FP32",
                   "grid": [S, S], "members": 20, "model": "epanechnikov"},
        "roofline": roof, "cpu_baseline": cpu, "detail": detail,
    }
    print(json.dumps(out), flush=True)


def profile_histogram(cp, workloads, torch, dev, S, steps, warmup):
    """The histogram workload alone (fit once, then forward + adjoint), for
    hardware-counter runs, followed by a plain 256 MiB copy (the reference
    that scales the HBM byte counters)."""
    mem = torch.as_tensor(workloads.mixture_ensemble(1, S, S), device=dev)
    params = cp.fit(mem, 2, nbins=10)
    del mem
    f = cp.field_of(params, 2, 10)
    g1, g2 = (torch.as_tensor(x, device=dev) for x in workloads.upstream(1, S, S))
    a, b = torch.empty((S, S), device=dev), torch.empty((S, S), device=dev)
    grad = torch.empty_like(params)
    for _ in range(warmup + steps):
        cp.forward(params, f, a, b)
        cp.backward(params, g1, g2, f, grad)
    src = torch.ones(64 << 20, dtype=torch.float32, device=dev)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    print(f"[bench] histogram profile: {warmup + steps} forward + adjoint launches", file=sys.stderr, flush=True)


def pipelined_step(cp, torch, mem, model, f, params, pmin, pmax, gmin, gmax, grad, reps):
    """A stream of ensembles with the fit as its own launch: the fit of
    ensemble i+1 on a second stream (default priority) while the forward and
    adjoint of ensemble i run, so the HBM-bound fit overlaps the VALU-bound
    kernels.  Two parameter buffers; events order
    each buffer's reuse.  Every step still runs all three kernels."""
    main = torch.cuda.current_stream()
    side = torch.cuda.Stream()
    bufs = [params, torch.empty_like(params)]
    fitted = [torch.cuda.Event() for _ in range(2)]
    used = [torch.cuda.Event() for _ in range(2)]
    for e in used:
        e.record(main)

    def run(n):
        for i in range(n):
            b = i % 2
            with torch.cuda.stream(side):
                side.wait_event(used[b])
                cp.fit(mem, model, out=bufs[b])
                fitted[b].record(side)
            main.wait_event(fitted[b])
            cp.forward(bufs[b], f, pmin, pmax)
            cp.backward(bufs[b], gmin, gmax, f, grad)
            used[b].record(main)

    run(reps)
    torch.cuda.synchronize()
    a, z = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record(main)
    side.wait_event(a)
    run(reps)
    z.record(main)
    torch.cuda.synchronize()
    return a.elapsed_time(z) / reps


def probe_ceilings(torch, dev):
    """Ceilings measured in this run by the probes of libcpprobes.so: the
    random-number and transcendental work of the conditional Monte Carlo
    estimator at its benchmark shape (1024^2 vertices x 4096 samples, one
    wave per vertex), FP32 FMA issue, and a 1 GiB + 1 GiB streaming copy."""
    import ctypes
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "paper_2407_18015_amd", "libcpprobes.so")
    lib = ctypes.CDLL(path)
    P = ctypes.c_void_p
    lib.cpb_mc_ceiling.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_int, P, P]
    lib.cpb_fma_peak.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, P, P]
    lib.cpb_copy.argtypes = [ctypes.c_int64, P, P, P]
    st = torch.cuda.current_stream().cuda_stream
    n, ns = 1024 * 1024, 4096
    out = torch.empty((n, 2), dtype=torch.float64, device=dev)
    t_mc = _timed(torch, lambda: lib.cpb_mc_ceiling(n, ns, 1, 3, 0, out.data_ptr(), st), 3)
    t_mcp = _timed(torch, lambda: lib.cpb_mc_ceiling(n, ns, 1, 3, 1, out.data_ptr(), st), 3)
    blocks, iters = 256 * 32, 2048
    fo = torch.empty(blocks * 256, device=dev)
    fma = {}
    for c in (1, 2, 4, 8, 16):
        t = _timed(torch, lambda: lib.cpb_fma_peak(blocks, iters * 8 // c, c, fo.data_ptr(), st), 5)
        fma[c] = blocks * 256 * 8 * iters * 2 / (t * 1e-3) / 1e12
    src = torch.ones(1 << 28, device=dev)
    dst = torch.empty_like(src)
    t_cp = _timed(torch, lambda: lib.cpb_copy(src.numel() // 4, src.data_ptr(), dst.data_ptr(), st), 10)
    del src, dst
    return {"mc_samples_per_s": n * ns / (t_mc * 1e-3), "mc_ms": t_mc,
            "mc_pdf_samples_per_s": n * ns / (t_mcp * 1e-3), "mc_pdf_ms": t_mcp,
            "fp32_fma_tflops_by_chains": fma, "fp32_fma_tflops": max(fma.values()),
            "copy_tbs": 2 * 4 * (1 << 28) / (t_cp * 1e-3) / 1e12}


def more_detail(cp, workloads, torch, dev, S, reps, ceil):
    res = {}
    # uniform FP64 64x64
    p = torch.as_tensor(workloads.uniform_params_field(0, 64, 64), device=dev)
    f = cp.field_of(p, 0)
    a, b = torch.empty((64, 64), dtype=torch.float64, device=dev), torch.empty((64, 64), dtype=torch.float64,
                                                                                device=dev)
    t = _timed(torch, lambda: cp.forward(p, f, a, b), reps)
    res["uniform_fp64_64"] = {"fwd_ms": t, "fwd_vertices_per_s": 64 * 64 / (t * 1e-3)}
    # uniform and histogram at S^2
    for name, model, gen, nb in (("uniform_2048", 0, workloads.smooth_ensemble, 0),
                                 ("histogram_2048", 2, workloads.mixture_ensemble, 10)):
        mem = torch.as_tensor(gen(1, S, S), device=dev)
        params = cp.fit(mem, model, nbins=nb)
        del mem
        f = cp.field_of(params, model, nb)
        g1, g2 = (torch.as_tensor(x, device=dev) for x in workloads.upstream(1, S, S))
        a, b = torch.empty((S, S), device=dev), torch.empty((S, S), device=dev)
        grad = torch.empty_like(params)
        tf = _timed(torch, lambda: cp.forward(params, f, a, b), reps)
        tb = _timed(torch, lambda: cp.backward(params, g1, g2, f, grad), max(3, reps // 2))
        tc = _timed(torch, lambda: cp.classify(params, f), reps)
        ts = _timed(torch, lambda: cp.classify(params, f, outputs=("saddle",)), reps)
        if model == 2:
            ff, fb, nint = hist_flops(params, nb)
            work = {"intervals": nint}
        else:
            ff, fb, cnt = uni_flops(params)
            work = {"pieces_by_started_neighbours": cnt.tolist()}
        res[name] = {"fwd_ms": tf, "bwd_ms": tb, "classify_ms": tc, "saddle_ms": ts,
                     "fwd_vertices_per_s": S * S / (tf * 1e-3),
                     "fwd_bwd_vertices_per_s": S * S / ((tf + tb) * 1e-3),
                     "roofline_fwd": roofline("alu", ff, tf * 1e-3, PEAK_FP32, "TFLOP/s"),
                     "roofline_bwd": roofline("alu", fb, tb * 1e-3, PEAK_FP32, "TFLOP/s"), **work}
        if model == 2:
            # semianalytical estimator (Sec. 4.4.2), 1000 samples per vertex
            fs = cp.field_of(params, model, nb, nsamples=1000, seed=1)
            tsa = _timed(torch, lambda: cp.semianalytical(params, fs, terms=True), max(3, reps // 4))
            res[name]["semianalytical_1000_ms"] = tsa
            res[name]["semianalytical_1000_samples_per_s"] = S * S * 1000 / (tsa * 1e-3)
        del params, grad
    # independent Gaussian at S^2 (deterministic quadrature: forward = all four classes)
    mem = torch.as_tensor(workloads.smooth_ensemble(1, S, S), device=dev)
    params = cp.fit(mem, "gaussian")
    del mem
    f = cp.field_of(params, "gaussian")
    a, b = torch.empty((S, S), device=dev), torch.empty((S, S), device=dev)
    tf = _timed(torch, lambda: cp.forward(params, f, a, b), reps)
    g1, g2 = (torch.as_tensor(g, device=dev) for g in workloads.upstream(1, S, S))
    grad = torch.empty_like(params)
    tb = _timed(torch, lambda: cp.backward(params, g1, g2, f, grad), max(3, reps // 4))
    res["gaussian_2048"] = {"fwd_ms": tf, "bwd_ms": tb, "fwd_vertices_per_s": S * S / (tf * 1e-3),
                            "fwd_bwd_vertices_per_s": S * S / ((tf + tb) * 1e-3)}
    del params, grad
    # multivariate Gaussian 1024^2, 4096 samples
    n = 1024
    mem = torch.as_tensor(workloads.correlated_ensemble(0, n, n), device=dev)
    params = cp.fit(mem, "mvg")
    del mem
    g1, g2 = (torch.as_tensor(x, device=dev) for x in workloads.upstream(2, n, n))
    a, b = torch.empty((n, n), device=dev), torch.empty((n, n), device=dev)
    grad = torch.empty_like(params)
    fr = cp.Field(n, n, 3, torch.float32, nsamples=4096, seed=1, estimator=0)
    fh = cp.Field(n, n, 3, torch.float32, nsamples=4096, seed=1, estimator=1)
    t_rb = _timed(torch, lambda: cp.forward(params, fr, a, b), 3)
    t_hit = _timed(torch, lambda: cp.forward(params, fh, a, b), 3)
    t_bwd = _timed(torch, lambda: cp.backward(params, g1, g2, fr, grad), 3)
    mc_peak = ceil["mc_samples_per_s"]
    res["mvg_1024_4096"] = {"fwd_conditional_ms": t_rb, "fwd_hit_ms": t_hit, "bwd_ms": t_bwd,
                            "fwd_vertices_per_s": n * n / (t_rb * 1e-3),
                            "fwd_bwd_vertices_per_s": n * n / ((t_rb + t_bwd) * 1e-3),
                            "samples_per_s_conditional": n * n * 4096 / (t_rb * 1e-3),
                            "roofline_fwd": roofline("alu", n * n * 4096, t_rb * 1e-3, mc_peak, "G samples/s",
                                                     ceiling="Philox + Box-Muller + normal CDF probe"),
                            "roofline_bwd": roofline("alu", n * n * 4096, t_bwd * 1e-3, ceil["mc_pdf_samples_per_s"],
                                                     "G samples/s",
                                                     ceiling="Philox + Box-Muller + normal density probe")}
    del params, grad
    res["batched_64_fields"] = batched_detail(cp, workloads, torch, dev)
    return res


def batched_detail(cp, workloads, torch, dev):
    """64 fields, sides round(2^U[7,11]), models cycling uniform /
    Epanechnikov / histogram(10), each fitted from a 20-member ensemble:
    forward + adjoint as one launch per pass, as a replayed graph, and as
    one forward and one adjoint launch per field."""
    t0 = time.time()
    fields, params, pmin, pmax, gmin, gmax, grad = [], [], [], [], [], [], []
    for side, model, seed in workloads.batched_layout(0):
        gen = workloads.mixture_ensemble if model == 2 else workloads.smooth_ensemble
        mem = torch.as_tensor(gen(seed, side, side), device=dev)
        p = cp.fit(mem, model, nbins=10 if model == 2 else 0)
        del mem
        fields.append(cp.field_of(p, model, 10 if model == 2 else 0))
        params.append(p)
        pmin.append(torch.empty((side, side), device=dev))
        pmax.append(torch.empty((side, side), device=dev))
        a, b = workloads.upstream(seed, side, side)
        gmin.append(torch.as_tensor(a, device=dev))
        gmax.append(torch.as_tensor(b, device=dev))
        grad.append(torch.empty_like(p))
    nv = sum(f.height * f.width for f in fields)
    print(f"[bench] batched inputs ({nv / 1e6:.1f} M vertices) in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)
    # algorithmic work of every field, as for the single-field workloads
    fl_f = fl_b = 0
    for f, p in zip(fields, params):
        a, b, _ = (hist_flops(p, f.nbins) if f.model == 2 else uni_flops(p) if f.model == 0 else epa_flops(p))
        fl_f += a
        fl_b += b
    out = {"fields": len(fields), "vertices": nv, "algorithmic_flops_fwd": fl_f, "algorithmic_flops_fwd_bwd": fl_f + fl_b}
    for name, kw in (("per_field", dict(per_field=True)), ("one_launch_per_pass", dict()), ("graph", dict(graph=True))):
        ms = _timed(torch, lambda: cp.batched(fields, params, pmin, pmax, gmin, gmax, grad, **kw), 5)
        out[name + "_fwd_bwd_ms"] = ms
        out[name + "_fwd_bwd_vertices_per_s"] = nv / (ms * 1e-3)
    for name, kw in (("per_field", dict(per_field=True)), ("graph", dict(graph=True))):
        ms = _timed(torch, lambda: cp.batched(fields, params, pmin, pmax, **kw), 5)
        out[name + "_fwd_ms"] = ms
        out[name + "_fwd_vertices_per_s"] = nv / (ms * 1e-3)
    # autotuned plans: the first call times every tile shape and claim chunk of
    # each pass on these fields, later calls (and the graph) reuse the choice
    for tag, g in (("fwd_bwd", (gmin, gmax, grad)), ("fwd", (None, None, None))):
        t0 = time.time()
        cp.batched(fields, params, pmin, pmax, *g, tune=True)
        torch.cuda.synchronize()
        out["tuning_s_" + tag] = time.time() - t0
        ms = _timed(torch, lambda: cp.batched(fields, params, pmin, pmax, *g, graph=True), 5)
        out["tuned_graph_" + tag + "_ms"] = ms
        out["tuned_graph_" + tag + "_vertices_per_s"] = nv / (ms * 1e-3)
        out["tuned_plan_" + tag] = cp.batched_describe(fields, fwd=True, bwd=g[2] is not None)
    out["roofline_tuned_graph_fwd_bwd"] = roofline("alu", fl_f + fl_b, out["tuned_graph_fwd_bwd_ms"] * 1e-3,
                                                   PEAK_FP32, "TFLOP/s")
    out["roofline_tuned_graph_fwd"] = roofline("alu", fl_f, out["tuned_graph_fwd_ms"] * 1e-3, PEAK_FP32,
                                               "TFLOP/s")
    out["roofline_per_field_fwd_bwd"] = roofline("alu", fl_f + fl_b, out["per_field_fwd_bwd_ms"] * 1e-3,
                                                 PEAK_FP32, "TFLOP/s")
    out["speedup_fwd_bwd_graph_vs_per_field"] = out["per_field_fwd_bwd_ms"] / out["graph_fwd_bwd_ms"]
    out["speedup_fwd_bwd_tuned_graph_vs_per_field"] = out["per_field_fwd_bwd_ms"] / out["tuned_graph_fwd_bwd_ms"]
    return out


def _timed(torch, fn, reps):
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def cpu_baseline(mem_np, gmin_np, gmax_np, budget_s=12.0, band=32):
    """The FP64 oracle (C, OpenMP, untuned) on bands of full-width rows of the
    same workload: fit, forward and adjoint per band, bands taken from the top
    until about `budget_s` seconds of work."""
    import oracle
    H, W = mem_np.shape[1], mem_np.shape[2]
    done, dt, y = 0, 0.0, 0
    while dt < budget_s and y + band <= H:
        lo, hi = max(0, y - 1), min(H, y + band + 1)
        sub = mem_np[:, lo:hi, :].astype(np.float64)
        g1 = gmin_np[lo:hi].astype(np.float64)
        g2 = gmax_np[lo:hi].astype(np.float64)
        rows = np.arange(y - lo, y - lo + band)
        idx = (rows[:, None] * W + np.arange(W)[None, :]).ravel().astype(np.int64)
        t = time.time()
        par = oracle.fit(1, sub, single=True)
        oracle.forward_at(1, par, idx)
        oracle.grad_at(1, par, g1, g2, idx)
        dt += time.time() - t
        done += band * W
        y += band
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    out = {"value": done / dt, "unit": UNIT, "cores": cores, "kind": "oracle",
           "sample": f"fit+forward+adjoint of the first {done // W} rows x {W} columns of the same "
                     f"20-member field, in bands of {band} rows", "seconds": dt}
    out["single_core"] = single_core_baseline(mem_np[:, :band + 1], gmin_np[:band + 1], gmax_np[:band + 1])
    out["per_model"] = oracle_per_model(cores)
    return out


def _timed_loop(fn, budget_s):
    n, t = 0, time.time()
    while n == 0 or time.time() - t < budget_s:
        fn()
        n += 1
    return n, time.time() - t


def oracle_per_model(cores, S=2048, budget_s=2.0):
    """The oracle (as above: FP64, untuned, `cores` host threads) on bounded
    samples of the other workloads, each as forward + adjoint in
    vertex-probabilities/s: the uniform 64x64 field whole, a band of rows of
    the histogram and independent-Gaussian 2048^2 fields, sampled vertices of
    the 1024^2 Monte Carlo field."""
    import oracle
    import workloads
    out = {}
    p = workloads.uniform_params_field(0, 64, 64)
    g1, g2 = workloads.upstream(1, 64, 64, np.float64)
    n, dt = _timed_loop(lambda: (oracle.forward(0, p), oracle.grad(0, p, g1, g2)), budget_s)
    out["uniform_fp64_64"] = {"value": n * 64 * 64 / dt, "cores": cores, "seconds": dt,
                              "sample": f"forward+adjoint of the whole 64x64 field, {n} times"}
    band = 4
    g1, g2 = (g[: band + 2].astype(np.float64) for g in workloads.upstream(1, S, S))
    idx = np.arange(S, S * (band + 1), dtype=np.int64)  # rows 1..band of the strip
    mem = workloads.mixture_ensemble(0, S, S)[:, : band + 2].astype(np.float64)
    ph = oracle.fit(2, mem, nbins=10, single=True)
    n, dt = _timed_loop(lambda: (oracle.forward_at(2, ph, idx), oracle.grad_at(2, ph, g1, g2, idx)), budget_s)
    out["histogram_2048"] = {"value": n * idx.size / dt, "cores": cores, "seconds": dt,
                             "sample": f"forward+adjoint of {band} rows x {S} of the 10-bin field, {n} times"}
    mem = workloads.smooth_ensemble(1, S, S)[:, :6].astype(np.float64)
    pg = oracle.fit(4, mem, single=True)
    gi = np.arange(S, S + 256, dtype=np.int64)
    n, dt = _timed_loop(lambda: (oracle.gauss_at(pg, gi), oracle.gauss_grad_at(pg, g1[:6], g2[:6], gi)), budget_s)
    out["gaussian_2048"] = {"value": n * gi.size / dt, "cores": cores, "seconds": dt,
                            "sample": f"forward+adjoint of 256 vertices of row 1 of the fitted field, {n} times"}
    M = 1024
    cm = workloads.correlated_ensemble(2, M, M)[:, :8].astype(np.float64)
    pm = oracle.mvg_fit(cm)
    mi = np.arange(3 * M, 3 * M + 32, dtype=np.int64)
    h1, h2 = (g[:8].astype(np.float64) for g in workloads.upstream(5, M, M))
    n, dt = _timed_loop(lambda: (oracle.mvg_forward_at(pm, mi, 4096, 1234, 7),
                                 oracle.mvg_grad_at(pm, h1, h2, mi, 4096, 1234, 7)), budget_s)
    out["mvg_1024_4096"] = {"value": n * mi.size / dt, "cores": cores, "seconds": dt,
                            "sample": f"forward (both estimators)+adjoint of 32 vertices, 4096 samples each, {n} times"}
    return out


def single_core_baseline(mem_np, gmin_np, gmax_np):
    """The same oracle work on one thread (a child process started with
    OMP_NUM_THREADS=1) for the first band of rows."""
    import subprocess
    import tempfile
    with tempfile.TemporaryDirectory() as d:
        np.save(os.path.join(d, "mem.npy"), mem_np)
        np.save(os.path.join(d, "g.npy"), np.stack([gmin_np, gmax_np]))
        env = dict(os.environ, OMP_NUM_THREADS="1")
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--oracle-band", d], env=env,
                           capture_output=True, text=True, timeout=600)
    if r.returncode != 0:
        return None
    return json.loads(r.stdout.strip().splitlines()[-1])


def oracle_band(d):
    """Child of single_core_baseline: fit + forward + adjoint of all rows but
    the last (its halo row) of the saved band, timed."""
    import oracle
    mem = np.load(os.path.join(d, "mem.npy")).astype(np.float64)
    g = np.load(os.path.join(d, "g.npy")).astype(np.float64)
    H, W = mem.shape[1] - 1, mem.shape[2]
    idx = np.arange(H * W, dtype=np.int64)
    t = time.time()
    par = oracle.fit(1, mem, single=True)
    oracle.forward_at(1, par, idx)
    oracle.grad_at(1, par, g[0], g[1], idx)
    dt = time.time() - t
    print(json.dumps({"value": H * W / dt, "unit": UNIT, "cores": 1, "seconds": dt,
                      "sample": f"fit+forward+adjoint of the first {H} rows x {W} columns"}))


if __name__ == "__main__":
    if len(sys.argv) == 3 and sys.argv[1] == "--oracle-band":
        oracle_band(sys.argv[2])
    else:
        main()
