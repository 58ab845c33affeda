#!/usr/bin/env python3
"""Benchmark: all right generalized eigenvectors of a real Schur pencil of order
m = 32768, robust FP64 (augmented matrices with power-of-two scale exponents), on one
MI355X.

A step is one call of the whole path on inputs already resident in HBM:
pre-processing, every diagonal solve and tile update of the blocked algorithm, and the
consolidation/normalisation pass.  The throughput is FP64-equivalent TFLOP/s with the
algorithmic count F(m) = 2 m^3 / 3 (each eigenvector of order p costs 2 p^2 flops).

Prints one JSON line (rank 0) with the roofline of the dominant kernel (the FP64-MFMA
tile update, timed with HIP events on the stream it runs on) and the CPU oracle timed
on a column sample of the same pencil.  Extra keys time the other configurations: the
mixed-precision mode, left eigenvectors, the back-transformation, a complex pencil of
order m / 2, one pencil of order 8192 (order_8192) and the batch of 512 pencils (batched).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_MFMA_PEAK = 78.6   # TFLOP/s, MI355X dense FP64 matrix
HBM_PEAK = 8000.0       # GB/s
METRIC = "FP64-equiv TFLOP/s + time for all eigvecs at m=32768; mixed/FP64 speedup"


# HBM traffic of the update kernel per launch from two rocprofv3 counter runs (FETCH_SIZE and
# WRITE_SIZE, scaled by what the counters read for a plain 1 GiB device copy), for the default
# workload; valid only while the kernel's sources hash to the value they had when the counters
# were taken (profiles/update_kernel_m32768_fp64_traffic.md).
TRAFFIC = {"sources_sha256_16": "01be4bf30fb4bffd", "bytes_per_launch": 4.403e9,
           "workload": (32768, 128, 4, 1)}   # m, mb, band, schedule


def update_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("update_tile.hpp", "update.hip"):
        with open(os.path.join(ROOT, "paper_2003_04776_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(S, T, blk, m, seconds):
    """The oracle (scalar robust substitution, one eigenvector at a time) on a sample of
    columns spread evenly over the pencil, on the host cores; rate in FP64-equivalent
    TFLOP/s (2 p^2 flops for the eigenvector of column p).  Also returns the sampled
    columns and the oracle's eigenvectors for them."""
    import numpy as np

    import oracle
    threads = max(1, min(16, os.cpu_count() or 1))
    # calibrate one eigenvector at p ~ m/2 on one thread
    p = m // 2
    sel = np.zeros(m, dtype=np.int32)
    sel[p] = 1
    t0 = time.perf_counter()
    oracle.tgevc(S, T, select=sel, threads=1)
    t1 = time.perf_counter() - t0
    rate1 = 2.0 * (p + 1) ** 2 / max(t1, 1e-6)
    avg_cost = 2.0 * m * m / 3.0
    n = int(seconds * threads * rate1 / avg_cost)
    n = max(threads, min(n, m))
    cols = np.unique(np.linspace(0, m - 1, n).astype(np.int64))
    sel = np.zeros(m, dtype=np.int32)
    sel[cols] = 1
    # closure under conjugation: a selected column of a pair brings its partner
    on = sel.astype(bool) | np.roll(sel.astype(bool) & (blk == 1), 1) | np.roll(sel.astype(bool) & (blk == 2), -1)
    idx = np.nonzero(on)[0]
    flops = float(np.sum(2.0 * (idx + 1.0) ** 2))
    t0 = time.perf_counter()
    Zo, _, _ = oracle.tgevc(S, T, select=sel, threads=threads)
    dt = time.perf_counter() - t0
    res = {"value": flops / dt / 1e12, "unit": "TFLOP/s", "cores": threads, "kind": "oracle",
           "sample": f"{len(idx)} of {m} columns evenly spread over the pencil, {flops:.3e} "
                     f"algorithmic flops in {dt:.1f} s; double-precision scalar robust substitution",
           "one_core_value": rate1 / 1e12,
           "one_core_sample": f"the eigenvector of column {p} alone on one thread ({t1:.2f} s)",
           "host_cpu": cpu_model(), "host_cores_total": os.cpu_count()}
    return res, idx, Zo[:, idx]


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def time_calls(fn, steps, warmup):
    """Median and mean device time (ms) of fn() from HIP events recorded on the current
    stream around each call (fn enqueues on that stream), after warmup calls."""
    import numpy as np
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ts = []
    for _ in range(steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn()
        e1.record()
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    return float(np.median(ts)), float(np.mean(ts))


def backward_error_stats(Sd, Td, Z, ar, ai, be, kind):
    """Componentwise backward error of every eigenvector on the GPU in FP64:
    omega_c = ||(beta S - alpha T) z||_1 / ||beta |S||z| + |alpha||T||z| ||_1 (pairs once, with
    |Re| + |Im|); an FP64 substitution keeps it at a few units of roundoff.  Returns
    median, p99 and max."""
    import numpy as np
    import torch
    dev = Z.device
    m = Z.shape[0]
    kind = np.asarray(kind)
    first = np.nonzero(kind != 2)[0]
    pair = kind[first] == 1
    a = torch.from_numpy(ar[first]).to(dev)
    b = torch.from_numpy(np.where(pair, ai[first], 0.0)).to(dev)
    bt = torch.from_numpy(be[first]).to(dev)
    fi = torch.from_numpy(first).to(dev)
    nx = torch.from_numpy(np.where(pair, first + 1, first)).to(dev)
    pm = torch.from_numpy(pair).to(dev)
    SZ = Sd @ Z
    TZ = Td @ Z
    rx = bt * SZ[:, fi] - a * TZ[:, fi] + b * TZ[:, nx]
    ry = torch.where(pm, bt * SZ[:, nx] - b * TZ[:, fi] - a * TZ[:, nx], torch.zeros_like(rx))
    num = rx.abs().sum(dim=0) + ry.abs().sum(dim=0)
    del SZ, TZ, rx, ry
    aZ = Z.abs()
    az = aZ[:, fi] + torch.where(pm, aZ[:, nx], torch.zeros_like(aZ[:, fi]))
    del aZ
    den = bt * (Sd.abs() @ az).sum(dim=0) + (a.abs() + b.abs()) * (Td.abs() @ az).sum(dim=0)
    om = (num / torch.where(den > 0, den, torch.ones_like(den))).cpu().numpy()
    return {"median": float(np.median(om)), "p99": float(np.quantile(om, 0.99)), "max": float(om.max())}


def run_batched(count, mb, band, steps, warmup):
    """The batch workload: `count` pencils of orders U{64..2048} (seed 3999), pencil i from
    seed 3000 + i, all eigenvectors, one rtgevc_batched call captured in a graph; times
    graph replays with events on the replay stream.  Returns (ms per replay, wall ms per
    replay, flops, orders, info nonzero count)."""
    import numpy as np
    import torch

    from paper_2003_04776_amd import pencils
    from paper_2003_04776_amd import rtgevc as rt

    ms = [int(v) for v in pencils.batch_sizes(count)]
    log(f"[bench] generating {len(ms)} pencils, sum m = {sum(ms)}")
    Sd, Td = [], []
    for i, m in enumerate(ms):
        S, T, _ = pencils.schur_pencil(m, 3000 + i)
        Sd.append(rt.colmajor_to_device(S))
        Td.append(rt.colmajor_to_device(T))
    bs = rt.BatchSolver(ms, mb=mb, band=band)
    Z, sc, info = bs.outputs()
    bs.run(Sd, Td, Z, sc, info)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        with torch.cuda.graph(g, stream=st):
            bs.run(Sd, Td, Z, sc, info)
    torch.cuda.synchronize()
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    times = []
    t0 = time.perf_counter()
    for _ in range(steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        g.replay()
        e1.record()
        e1.synchronize()
        times.append(e0.elapsed_time(e1))
    wall = time.perf_counter() - t0
    F = float(sum(2.0 * m ** 3 / 3.0 for m in ms))
    nz = int((info != 0).sum().item())
    del g, bs, Z, sc, info, Sd, Td
    torch.cuda.empty_cache()
    return float(np.median(times)), wall / max(steps, 1) * 1e3, F, ms, nz


def batch_config(ms, mb, band):
    from paper_2003_04776_amd import rtgevc as rt
    return {"workload": f"{len(ms)} independent real Schur pencils, orders U{{64..2048}} (seed 3999), all "
                        f"eigenvectors, robust FP64, one batched call replayed from a graph",
            "sum_m": sum(ms), "mb": mb or "automatic",
            "band": rt.resolve_opts(max(ms), batched=True, mb=mb, band=band)[1]}


def bench_batched(args):
    """--workload batched: the batch as the main line."""
    med, wall, F, ms, nz = run_batched(args.count, args.mb, args.band, args.steps, args.warmup)
    out = {
        "metric": "FP64-equiv TFLOP/s, batch of pencils (graph replay)",
        "value": round(F / (med * 1e-3) / 1e12, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(med, 3), "wall_ms_per_step": round(wall, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": dict(batch_config(ms, args.mb, args.band), flops_per_step=F),
        "info_nonzero": nz,
    }
    print(json.dumps(out), flush=True)


def bench_order(args, m2):
    """One pencil of order m2 (the seeded normal generator, seed + 11), all eigenvectors with
    the automatic options, FP64 and mixed precision (default refinement), timed with events
    around each product call."""
    import torch
    from paper_2003_04776_amd import pencils
    from paper_2003_04776_amd import rtgevc as rt
    log(f"[bench] order {m2}")
    S, T, _ = pencils.schur_pencil(m2, args.seed + 11, threads=16)
    Sd, Td = rt.colmajor_to_device(S), rt.colmajor_to_device(T)
    del S, T
    F = 2.0 * m2 ** 3 / 3.0
    res = {"what": f"all right eigenvectors, order {m2}, automatic options", "flops_per_call": F}
    for name, prec in (("fp64", 0), ("mixed", 1)):
        sv = rt.Solver(m2, precision=prec)
        Z = rt.colmajor_empty(m2)
        info = torch.zeros(1, dtype=torch.int32, device="cuda")
        ms, _ = time_calls(lambda: sv.run(Sd, Td, Z=Z, info=info), max(args.steps, 5), max(args.warmup, 1))
        mb, band, split = rt.resolve_opts(m2, precision=prec, with_split=True)
        res[name] = {"ms_per_call": round(ms, 3), "value": round(F / (ms * 1e-3) / 1e12, 4),
                     "unit": "FP64-equiv TFLOP/s", "mb": mb, "band": band, "split": split,
                     "info": int(info.item())}
        log(f"[bench] order {m2} {name}: {ms:.2f} ms")
        del sv, Z
    del Sd, Td
    torch.cuda.empty_cache()
    return res


def residual_max(Sd, Td, Z, ar, ai, be, kind):
    """max_c ||S Z_c D_c - T Z_c B_c||_1 / ((||S||_1 + ||T||_1) ||Z_c||_1) on the GPU in FP64
    (the eigen-equation of the Schur pencil column by column; a complex pair (p, p+1) in its
    real form, (alpha, beta) scaled so that max(beta, |Re alpha| + |Im alpha|) = 1)."""
    import numpy as np
    import torch
    dev = Z.device
    m = Z.shape[0]
    kind = np.asarray(kind)
    p = np.where(kind == 2, np.arange(m) - 1, np.arange(m))
    a, b, bt = ar[p].astype(float), np.abs(ai[p]).astype(float), be[p].astype(float)
    s = np.maximum(bt, np.abs(a) + b)
    s[s == 0] = 1.0
    A, Bv, BT = (torch.from_numpy(v / s).to(dev) for v in (a, b, bt))
    R = (Sd @ Z) * BT
    TZ = Td @ Z
    TZB = TZ * A
    k1 = torch.from_numpy(np.nonzero(kind == 1)[0]).to(dev)
    if k1.numel():
        TZB[:, k1] = A[k1] * TZ[:, k1] - Bv[k1] * TZ[:, k1 + 1]
        TZB[:, k1 + 1] = Bv[k1] * TZ[:, k1] + A[k1] * TZ[:, k1 + 1]
    del TZ
    R -= TZB
    del TZB
    den = (Sd.abs().sum(dim=0).max() + Td.abs().sum(dim=0).max()) * Z.abs().sum(dim=0)
    eta = R.abs().sum(dim=0) / torch.where(den > 0, den, torch.ones_like(den))
    return float(eta.max().item())


def bench_left(args, m, Sd, Td, F, ms_right):
    """All left eigenvectors of the same pencil (rtgevc_left: the right path on the flipped
    transposed pencil plus the flip and turn passes), timed with events around each call on
    its stream."""
    import torch
    from paper_2003_04776_amd import rtgevc as rt
    solver = rt.Solver(m, mb=args.mb, normalize=True, band=args.band, schedule=args.schedule, left=True)
    Y = rt.colmajor_empty(m)
    ls = torch.empty(m, dtype=torch.int32, device="cuda")
    linfo = torch.zeros(1, dtype=torch.int32, device="cuda")
    for _ in range(max(args.warmup, 1)):
        solver.run(Sd, Td, Z=Y, scales=ls, info=linfo)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        solver.run(Sd, Td, Z=Y, scales=ls, info=linfo)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / max(args.steps, 1)
    log(f"[bench] left eigenvectors: {ms:.1f} ms per call")
    res = {"what": "all left eigenvectors u^H (beta S - alpha T) = 0 of the same pencil, FP64, normalised",
           "ms_per_call": round(ms, 3), "value": round(F / (ms * 1e-3) / 1e12, 4), "unit": "TFLOP/s",
           "time_vs_right": round(ms / ms_right, 4), "info": int(linfo.item())}
    del solver, Y
    return res


def bench_back(args, m, Sd, Zf, scales, blk):
    """The back-transformation X = V Z of the FP64 eigenvectors with a seeded dense V (the
    contraction does not depend on V being orthogonal), timed with events on the stream it
    runs on.  Algorithmic flops: 2 m per stored entry of the quasi-triangular Z."""
    import numpy as np
    import torch
    from paper_2003_04776_amd import rtgevc as rt
    g = torch.Generator(device="cuda")
    g.manual_seed(args.seed + 1)
    V = torch.randn((m, m), dtype=torch.float64, device="cuda", generator=g).t()   # column-major view
    V.mul_(1.0 / np.sqrt(m))
    X = rt.colmajor_empty(m)
    xs = torch.empty(m, dtype=torch.int32, device="cuda")
    binfo = torch.zeros(1, dtype=torch.int32, device="cuda")
    bt = rt.BackTransformer(m, mb=args.mb if args.mb in (64, 128) else 0)
    for _ in range(max(args.warmup, 1)):
        bt.run(Sd, V, Zf, scales, X=X, xscales=xs, info=binfo)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        bt.run(Sd, V, Zf, scales, X=X, xscales=xs, info=binfo)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / max(args.steps, 1)
    npairs = int((np.asarray(blk) == 1).sum())
    flops = 2.0 * m * (m * (m + 1) / 2.0 + npairs)
    ach = flops / (ms * 1e-3) / 1e12
    log(f"[bench] back-transformation: {ms:.1f} ms per call, {ach:.2f} TFLOP/s")
    res = {
        "what": "X = V Z, the eigenvectors of (U S V^T, U T V^T); dense seeded V, normalised output",
        "mb": 128 if (args.mb == 128 or (args.mb not in (64, 128) and m >= 2048)) else 64,
        "ms_per_call": round(ms, 3),
        "flops_per_call": flops,
        "roofline": {"kernel": "whole call (back_gemm_kernel on FP64 MFMA 16x16x4 plus scan, pack and "
                               "normalisation passes)", "bound": "mfma", "achieved": round(ach, 3),
                     "peak": FP64_MFMA_PEAK, "unit": "TFLOP/s", "frac": round(ach / FP64_MFMA_PEAK, 4)},
        "info": int(binfo.item()),
    }
    del V, X, bt
    return res


def bench_complex(args, mc):
    """All eigenvectors of a complex upper-triangular pencil of order mc (rtgevc_complex: the
    real form of order 2 mc through the real path), timed with events around each call.
    Complex-arithmetic flop count 8 mc^3 / 3 (a complex multiply-add is 8 real flops)."""
    import numpy as np
    import torch
    from paper_2003_04776_amd import pencils
    from paper_2003_04776_amd import rtgevc as rt
    log(f"[bench] complex pencil of order {mc}")
    S, T = pencils.complex_schur_pencil(mc, args.seed + 7, threads=16)
    Sd, Td = rt.ccolmajor_to_device(S), rt.ccolmajor_to_device(T)
    del S, T
    sv = rt.ComplexSolver(mc, mb=args.mb, band=args.band)
    Z = torch.empty((mc, mc), dtype=torch.complex128, device="cuda").t()
    sc = torch.empty(mc, dtype=torch.int32, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    ms, _ = time_calls(lambda: sv.run(Sd, Td, Z=Z, scales=sc, info=info), args.steps, args.warmup)
    F = 8.0 * mc ** 3 / 3.0
    res = {"what": f"all eigenvectors of a complex upper-triangular pencil of order {mc}, FP64, normalised "
                   f"(its real form of order {2 * mc} through the real path)",
           "ms_per_call": round(ms, 3), "flops_per_call": F,
           "value": round(F / (ms * 1e-3) / 1e12, 4), "unit": "TFLOP/s (complex-arithmetic count 8 m^3/3)",
           "info": int(info.item())}
    log(f"[bench] complex: {ms:.1f} ms per call")
    del sv, Z, Sd, Td
    torch.cuda.empty_cache()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--m", type=int, default=32768)
    ap.add_argument("--mb", type=int, default=0)
    ap.add_argument("--band", type=int, default=0)
    ap.add_argument("--schedule", type=int, default=0, choices=(0, 1, 2),
                    help="0/1: band wavefront with look-ahead; 2: persistent walker")
    ap.add_argument("--precision", type=int, default=0, choices=(0, 1),
                    help="0: FP64 tile updates; 1: mixed (int8 matrix cores on split operands)")
    ap.add_argument("--no-compare-mixed", dest="compare_mixed", action="store_false",
                    help="skip the mixed-precision run that follows the FP64 one")
    ap.add_argument("--no-residual", dest="residual", action="store_false",
                    help="skip the eigen-equation residuals of the FP64 and mixed results")
    ap.add_argument("--no-left", dest="left", action="store_false",
                    help="skip the left eigenvectors timed after the right ones")
    ap.add_argument("--no-back", dest="back", action="store_false",
                    help="skip the back-transformation X = V Z timed after the eigenvectors")
    ap.add_argument("--no-extra", dest="extra", action="store_false",
                    help="skip the order-8192 pencil and the batch of --count pencils timed after the headline")
    ap.add_argument("--no-complex", dest="complex", action="store_false",
                    help="skip the complex pencil of order m / 2 timed after the real one")
    ap.add_argument("--seed", type=int, default=400)
    ap.add_argument("--kind", default="normal", choices=("normal", "stress", "zeroinf", "degenerate", "general", "unbalanced"))
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--workload", default="single", choices=("single", "batched"),
                    help="single: one pencil of order --m (the headline); batched: --count pencils")
    ap.add_argument("--count", type=int, default=512)
    ap.add_argument("--copy-probe-mb", type=int, default=0,
                    help="before the timed steps, copy this many MiB once with a plain device copy "
                         "(a kernel of known traffic, to calibrate memory counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only: the library has no multi-GPU path (asked for {args.gpus})",
              file=sys.stderr)
        sys.exit(2)
    if args.workload == "batched":
        bench_batched(args)
        return

    import numpy as np
    import torch

    from paper_2003_04776_amd import pencils
    from paper_2003_04776_amd import rtgevc as rt

    rank = int(os.environ.get("RANK", "0"))
    m = args.m
    log(f"[bench] generating pencil m={m} kind={args.kind} seed={args.seed}")
    t0 = time.perf_counter()
    S, T, blk = pencils.schur_pencil(m, args.seed, args.kind, threads=16)
    log(f"[bench] generated in {time.perf_counter() - t0:.1f} s; uploading")
    Sd, Td = rt.colmajor_to_device(S), rt.colmajor_to_device(T)
    solver = rt.Solver(m, mb=args.mb, normalize=True, band=args.band, schedule=args.schedule,
                       precision=args.precision)
    Z = rt.colmajor_empty(m)
    scales = torch.empty(m, dtype=torch.int32, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    if args.copy_probe_mb > 0:
        n = args.copy_probe_mb * (1 << 20) // 8
        src = torch.ones(n, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] copy probe: {n * 8} bytes read and {n * 8} bytes written")
        del src, dst

    # ---- the headline: the product call rtgevc, HIP events around each call on its stream ----
    def call():
        solver.run(Sd, Td, Z=Z, scales=scales, info=info)

    for _ in range(args.warmup):
        call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dev_ms = []
    for k in range(args.steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        call()
        e1.record()
        e1.synchronize()
        dev_ms.append(e0.elapsed_time(e1))
        log(f"[bench] step {k}: {dev_ms[-1]:.1f} ms (rtgevc, device events)")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = wall / max(args.steps, 1) * 1e3
    info_v = int(info.item())
    F = 2.0 * m ** 3 / 3.0
    value = F / (ms_per_step * 1e-3) / 1e12

    # ---- phase split and the update kernel's roofline: rtgevc_timed (events around every launch) ----
    stats = [solver.run_timed(Sd, Td, Z, scales, info) for _ in range(2)]
    for k, st in enumerate(stats):
        log(f"[bench] timed {k}: device {st['total_ms']:.1f} ms (pre {st['pre_ms']:.2f}, solve {st['solve_ms']:.1f}, "
            f"update {st['update_ms']:.1f}, consolidate {st['consolidate_ms']:.2f}, refine {st['refine_ms']:.2f})")
    upd_flops = sum(s["update_flops"] for s in stats)
    upd_ms = sum(s["update_ms"] for s in stats)
    upd_launches = sum(s["n_update"] for s in stats)
    achieved = upd_flops / (upd_ms * 1e-3) / 1e12 if upd_ms > 0 else 0.0
    st0 = stats[-1]
    res_mb, res_band, res_sched = rt.resolve_opts(m, mb=args.mb, band=args.band, schedule=args.schedule,
                                                  precision=args.precision, with_schedule=True)
    out = {
        "metric": METRIC,
        "value": round(value, 4),
        "unit": "TFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i8+f64" if args.precision == 1 else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"all right eigenvectors of a real Schur pencil, m={m}, robust FP64 "
                        f"(power-of-two scale exponents), normalised output",
            "m": m, "mb": res_mb, "band": res_band,
            "schedule": "persistent walker" if res_sched == 2 else "band wavefront", "tiles": int(st0["M"]),
            "seed": args.seed, "generator": args.kind, "flops_per_step": F,
            "timed_call": "rtgevc (the product entry point), HIP events around each call; ms_per_step is the "
                          "host wall clock over the timed calls",
        },
        "device_ms_median": round(float(np.median(dev_ms)), 3),
        "roofline": {
            "kernel": ("walker_kernel (whole task graph: tile updates on FP64 MFMA 16x16x4 and solves; "
                       "update flops over the walker's time)") if res_sched == 2 else
                      "update_kernel (robust tile update, FP64 MFMA 16x16x4)",
            "bound": "mfma",
            "achieved": round(achieved, 3),
            "peak": FP64_MFMA_PEAK,
            "unit": "TFLOP/s",
            "frac": round(achieved / FP64_MFMA_PEAK, 4),
            "traffic": (TRAFFIC["bytes_per_launch"]
                        if (m, res_mb, res_band, res_sched) == TRAFFIC["workload"]
                        and args.precision == 0
                        and update_sources_hash() == TRAFFIC["sources_sha256_16"] else None),
            "traffic_unit": "bytes per launch (HBM read + write)",
            "launches": int(upd_launches),
            "avg_launch_ms": round(upd_ms / max(upd_launches, 1), 4),
            "flops_per_launch": upd_flops / max(upd_launches, 1),
            "measured_with": "rtgevc_timed (HIP events on the stream of every launch), 2 calls",
        },
        # the same kernel's launches on the side stream alone (the updates of the rows above the
        # next band, most of the flops), beside the roofline over every launch
        "side_stream_updates": None if res_sched == 2 else {
            "what": "update_kernel launches of the side stream (the rows above the next band)",
            "launches": int(sum(s["n_side_update"] for s in stats)),
            "share_of_update_flops": round(sum(s["side_update_flops"] for s in stats) / max(upd_flops, 1.0), 4),
            "avg_launch_ms": round(sum(s["side_update_ms"] for s in stats) / max(sum(s["n_side_update"] for s in stats), 1), 4),
            "achieved": round(sum(s["side_update_flops"] for s in stats)
                              / max(sum(s["side_update_ms"] for s in stats) * 1e-3, 1e-12) / 1e12, 3),
            "frac": round(sum(s["side_update_flops"] for s in stats)
                          / max(sum(s["side_update_ms"] for s in stats) * 1e-3, 1e-12) / 1e12 / FP64_MFMA_PEAK, 4),
        },
        "phases_ms": {k: round(st0[k], 3) for k in ("pre_ms", "solve_ms", "update_ms", "consolidate_ms",
                                                     "refine_ms", "total_ms")},
        "info": info_v,
    }
    Zf = Z.clone()
    Zm = None
    if args.compare_mixed and args.precision == 0 and args.schedule != 2:
        # the mixed-precision mode on the same inputs, with its default refinement (one sweep;
        # columns flagged by the backward-error sketch) and without refinement
        mixed = rt.Solver(m, mb=args.mb, normalize=True, band=args.band, precision=1)
        Zm = rt.colmajor_empty(m)
        minfo = torch.zeros(1, dtype=torch.int32, device="cuda")
        mms, _ = time_calls(lambda: mixed.run(Sd, Td, Z=Zm, scales=scales, info=minfo), args.steps, args.warmup)
        m_info = int(minfo.item())
        mst = mixed.run_timed(Sd, Td, Zm, scales, minfo)
        del mixed
        noref = rt.Solver(m, mb=args.mb, normalize=True, band=args.band, precision=1, max_refine=-1)
        Zn = rt.colmajor_empty(m)
        nms, _ = time_calls(lambda: noref.run(Sd, Td, Z=Zn, scales=scales, info=minfo), args.steps, args.warmup)
        nst = noref.run_timed(Sd, Td, Zn, scales, minfo)
        same = bool(torch.equal(Zn, Zm))
        del noref, Zn
        mmb, mband = rt.resolve_opts(m, mb=args.mb, band=args.band, precision=1)
        fp64_ms = float(np.median(dev_ms))
        out["mixed"] = {
            "precision": "tile-update contraction on int8 matrix cores, operands split into 7 x 7-bit slices "
                         "(S/T halves scaled apart per source tile row); FP64 solves, bounds, residual",
            "mb": mmb, "band": mband,
            "ms_per_call": round(mms, 3),
            "value": round(F / (mms * 1e-3) / 1e12, 4),
            "speedup_vs_fp64": round(fp64_ms / mms, 4),
            "refinement": {"max_sweeps": 1, "threshold": "componentwise backward error 64 m 2^-53",
                           "refine_ms": round(mst["refine_ms"], 3),
                           "info_bit_64": bool(m_info & 64),
                           "result_equals_unrefined": same,
                           "ms_per_call_without_refinement": round(nms, 3),
                           "speedup_vs_fp64_without_refinement": round(fp64_ms / nms, 4)},
            "update_achieved_fp64_equiv_tflops": round(mst["update_flops"] / (mst["update_ms"] * 1e-3) / 1e12, 3)
            if mst["update_ms"] > 0 else None,
            "max_abs_diff_vs_fp64": float((Zm - Zf).abs().max().item()),
            "info": m_info,
        }
        log(f"[bench] mixed: {mms:.1f} ms/call (without refinement {nms:.1f}), speed-up {fp64_ms / mms:.3f}")
    if args.residual and args.precision == 0:
        # the eigen-equation residual and the componentwise backward error of the FP64 result
        # and of the mixed one
        are, aim, bet, _ = solver.eigvals(Sd, Td)
        ar, ai, be = (x.cpu().numpy() for x in (are, aim, bet))
        res = {"bound": 64 * m * 2.0 ** -53, "fp64_max": residual_max(Sd, Td, Zf, ar, ai, be, blk),
               "fp64_backward_error": backward_error_stats(Sd, Td, Zf, ar, ai, be, blk)}
        if Zm is not None:
            res["mixed_max"] = residual_max(Sd, Td, Zm, ar, ai, be, blk)
            res["mixed_backward_error"] = backward_error_stats(Sd, Td, Zm, ar, ai, be, blk)
        out["residual"] = res
        log(f"[bench] residuals: {res}")
    del solver
    if args.left and args.precision == 0:
        out["left"] = bench_left(args, m, Sd, Td, F, float(np.median(dev_ms)))
    if args.back:
        out["backtransform"] = bench_back(args, m, Sd, Zf, scales, blk)
    if args.complex and args.precision == 0:
        out["complex"] = bench_complex(args, m // 2)
    if args.extra and args.precision == 0 and m > 8192:
        # the other configurations of the headline: a smaller order and the batch
        out["order_8192"] = bench_order(args, 8192)
        med, wall, Fb, msb, nzb = run_batched(args.count, 0, 0, max(args.steps, 5), max(args.warmup, 2))
        out["batched"] = {"config": batch_config(msb, 0, 0), "ms_per_call": round(med, 3),
                          "wall_ms_per_call": round(wall, 3), "flops_per_call": Fb,
                          "value": round(Fb / (med * 1e-3) / 1e12, 4), "unit": "FP64-equiv TFLOP/s",
                          "info_nonzero": nzb}
        log(f"[bench] batch of {len(msb)}: {med:.2f} ms")
    if rank == 0 and not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a column sample")
        out["cpu_baseline"], idx, Zo = cpu_baseline(S, T, blk, m, args.cpu_seconds)
        if args.precision == 0:
            # e_c = max_i |Z_gpu - Z_oracle| per column on the sample (normalised columns)
            ti = torch.from_numpy(idx).to(Zf.device)
            chk = {}
            for name, ZZ in (("fp64", Zf), ("mixed", Zm)):
                if ZZ is None:
                    continue
                err = np.abs(ZZ[:, ti].cpu().numpy() - Zo).max(axis=0)
                chk[name] = {"columns": int(len(idx)), "median": float(np.median(err)),
                             "p99": float(np.quantile(err, 0.99)), "max": float(err.max()),
                             "columns_above_1e-10": int((err > 1e-10).sum())}
            if Zm is not None:
                # the columns where the mixed result differs most from the FP64 one, against the oracle
                import oracle
                d = (Zm - Zf).abs().amax(dim=0)
                top = torch.topk(d, 8).indices.cpu().numpy()
                sel = np.zeros(m, dtype=np.int32)
                sel[top] = 1
                Zt, _, _ = oracle.tgevc(S, T, select=sel, threads=16)
                et = np.abs(Zm[:, torch.from_numpy(top).to(Zm.device)].cpu().numpy() - Zt[:, top]).max(axis=0)
                chk["mixed_worst_vs_fp64"] = {"columns": [int(c) for c in top], "max": float(et.max())}
            out["oracle_check"] = chk
    if rank == 0:
        print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
