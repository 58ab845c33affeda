"""Autotuner: sweeps the performance parameters of the solver on the GPU and writes the
table the library compiles in.

Parameters are performance choices only — tile size mb, update band R, schedule (band
wavefront or persistent walker) and the tiles per launch of a band's update of the rows above
it (split) for single pencils in FP64, tile size, band and split for the mixed-precision mode,
tile size per order bucket for batches — never bounds: every choice computes the same
eigenvectors, so a table from another machine is safe, merely slower.

    python -m paper_2003_04776_amd.autotune [--out-dir DIR] [--quick] [--splits-only]

(--splits-only keeps the tile sizes, bands and schedules of the table the library was built
with and sweeps only the splits.)

writes DIR/tuning.json (every timing of the sweep) and DIR/tuning_table.inc (the chosen
entries, in the form csrc/tuning_table.inc expects); copy both into the package (the
.inc into csrc/) and rebuild.  Inputs are the seeded synthetic pencils of
``pencils.schur_pencil``.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

SINGLE_SIZES = (256, 1024, 4096, 8192, 16384, 32768)
SPLITS = (0, 1024, 2048, 4096, 8192)   # 0: one launch per band
BATCH_BUCKETS = ((64, 128), (128, 256), (256, 512), (512, 1024), (1024, 2048))
MBS = (32, 64, 128)
BANDS = (1, 2, 4, 8)


def single_candidates(m):
    """(mb, band, schedule) candidates: the band wavefront with every band size, and the
    persistent walker (one source row per update) up to m = 8192 (beyond, its workspace of
    every tile's W grows past 1 GB and it has never been competitive)."""
    for mb in MBS:
        if m >= 8192 and mb == 32:
            continue       # thousands of tile rows: never competitive, and slow to sweep
        if mb > 2 * m:
            continue
        for band in BANDS:
            yield mb, band, 1
        if m <= 8192:
            yield mb, 1, 2


def mixed_candidates(m):
    """(mb, band) candidates of the mixed-precision mode (band wavefront only)."""
    for mb in MBS:
        if mb == 32 or mb > 2 * m:
            continue
        for band in BANDS:
            yield mb, band


def time_single(m, mb, band, schedule, Sd, Td, Z, sc, info, reps, precision=0, split=0):
    """Best of `reps` product calls (rtgevc), HIP events around each call on the stream it
    runs on (per-launch events would perturb the overlap of the two streams)."""
    import torch
    from paper_2003_04776_amd import rtgevc as rt
    solver = rt.Solver(m, mb=mb, band=band, schedule=schedule, precision=precision, split=split if split else -1)
    solver.run(Sd, Td, Z=Z, scales=sc, info=info)   # warm-up (first launch of each kernel)
    torch.cuda.synchronize()
    best = math.inf
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        solver.run(Sd, Td, Z=Z, scales=sc, info=info)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


def time_batch(ms, mb, Sd, Td, reps):
    import torch
    from paper_2003_04776_amd import rtgevc as rt
    bs = rt.BatchSolver(ms, mb=mb)
    Z, sc, info = bs.outputs()
    bs.run(Sd, Td, Z, sc, info)
    torch.cuda.synchronize()
    best = math.inf
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        bs.run(Sd, Td, Z, sc, info)
        e1.record()
        e1.synchronize()
        best = min(best, e0.elapsed_time(e1))
    return best


SPLIT_GAIN = 0.01   # a split must beat one launch per band by this fraction to be chosen


def choose_split(times, tiles=None):
    """{split: ms} -> the split to tabulate: the fastest, unless it is within SPLIT_GAIN of
    one launch per band (split 0), which then stays (fewer launches at the same time).
    Splits of at least `tiles` (the tile count of the pencil, more than any band update has)
    issue the same launches as split 0 and are not candidates."""
    if not times:
        return 0
    times = {s: t for s, t in times.items() if s == 0 or tiles is None or s < tiles}
    best, t = min(times.items(), key=lambda kv: kv[1])
    if 0 in times and t >= (1.0 - SPLIT_GAIN) * times[0]:
        return 0
    return best


def choose_single(results, mixed=None, splits=None):
    """results: {m: {(mb, band, schedule): ms}}, mixed: {m: {(mb, band): ms}}, splits:
    {m: {"fp64": {split: ms}, "mixed": {split: ms}}} -> table entries (m_max, mb, band,
    schedule, split, mb_mixed, band_mixed, split_mixed), sizes ascending; each measured size's
    best choice covers up to the geometric midpoint to the next.  Without mixed timings the
    mixed columns repeat the FP64 tile size and band; without split timings a band's update
    is one launch (split 0)."""
    sizes = sorted(results)
    out = []
    for i, m in enumerate(sizes):
        (mb, band, schedule), _ = min(results[m].items(), key=lambda kv: kv[1])
        if mixed and mixed.get(m):
            (mbx, bandx), _ = min(mixed[m].items(), key=lambda kv: kv[1])
        else:
            mbx, bandx = mb, band
        sp = (splits or {}).get(m, {})
        split = choose_split(sp.get("fp64"), ((m + mb - 1) // mb) ** 2)
        splitx = choose_split(sp.get("mixed"), ((m + mbx - 1) // mbx) ** 2)
        m_max = int(math.sqrt(m * sizes[i + 1])) if i + 1 < len(sizes) else None
        out.append((m_max, mb, band, schedule, split, mbx, bandx, splitx))
    return out


def choose_batch(results):
    """results: {(lo, hi): {mb: ms}} -> entries (m_max, mb), buckets ascending.  One tile size
    for every bucket, the one with the least summed time over the buckets (that every bucket
    timed): a batch runs its pencils in groups by tile size, one group after the other, so
    mixing tile sizes adds whole lock-step sequences (per-bucket choices measured 44.0 ms on
    the 512-pencil batch of orders U{64..2048} against 41.7 ms with tile 64 throughout)."""
    buckets = sorted(results)
    if not buckets:
        return []
    common = set.intersection(*(set(results[b]) for b in buckets))
    if common:
        mb = min(sorted(common), key=lambda t: sum(results[b][t] for b in buckets))
        return [(hi if i + 1 < len(buckets) else None, mb) for i, (lo, hi) in enumerate(buckets)]
    out = []
    for i, (lo, hi) in enumerate(buckets):
        mbi, _ = min(results[(lo, hi)].items(), key=lambda kv: kv[1])
        out.append((hi if i + 1 < len(buckets) else None, mbi))
    return out


def record_timings(rec):
    """The timings of a tuning.json record in the form the choose_ functions take."""
    def kv(key):
        return dict(p.split("=") for p in key.split(","))
    single = {int(m): {(int(kv(k)["mb"]), int(kv(k)["band"]), int(kv(k)["schedule"])): t for k, t in d.items()}
              for m, d in rec.get("single", {}).items()}
    mixed = {int(m): {(int(kv(k)["mb"]), int(kv(k)["band"])): t for k, t in d.items()}
             for m, d in rec.get("mixed", {}).items()}
    # sizes whose splits were swept on the tile size and band of a built table
    for m, base in rec.get("split_base", {}).items():
        b, x = kv(base["fp64"]), kv(base["mixed"])
        single.setdefault(int(m), {(int(b["mb"]), int(b["band"]), int(b["schedule"])): 0.0})
        mixed.setdefault(int(m), {(int(x["mb"]), int(x["band"])): 0.0})
    splits = {}
    for m, d in rec.get("split", {}).items():
        for k, t in d.items():
            prec, sp = k.split(",")
            splits.setdefault(int(m), {}).setdefault(prec, {})[int(sp.split("=")[1])] = t
    batch = {}
    for b, d in rec.get("batch", {}).items():
        lo, hi = (int(x) for x in b.split("-"))
        batch[(lo, hi)] = {int(k.split("=")[1]): t for k, t in d.items()}
    return single, mixed, splits, batch


def render_inc(single, batch, source):
    lines = [
        "// Performance parameters chosen per problem size (never bounds: every choice computes",
        "// the same eigenvectors).  Written by paper_2003_04776_amd/autotune.py from a sweep on",
        f"// the GPU ({source}).",
        "// Single pencils: the first entry with m <= m_max applies: {m_max, mb, band, schedule, split}",
        "// for FP64, then {mb, band, split} for mixed precision (split: tiles per launch of a band's",
        "// update of the rows above it, 0 = one launch).",
        "static const TuneSingle kTuneSingle[] = {",
    ]
    for m_max, mb, band, schedule, split, mbx, bandx, splitx in single:
        lines.append(f"    {{{m_max if m_max is not None else 'INT64_MAX'}, {mb}, {band}, {schedule}, {split}, "
                     f"{mbx}, {bandx}, {splitx}}},")
    lines += ["};", "// Pencils of a batch (tile size per order bucket).", "static const TuneBatch kTuneBatch[] = {"]
    for m_max, mb in batch:
        lines.append(f"    {{{m_max if m_max is not None else 'INT64_MAX'}, {mb}}},")
    lines.append("};")
    return "\n".join(lines) + "\n"


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--out-dir", default=HERE)
    ap.add_argument("--quick", action="store_true", help="smaller sweep (sizes up to 8192)")
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--batch-count", type=int, default=64)
    ap.add_argument("--splits-only", action="store_true",
                    help="keep the built table's tile sizes, bands and schedules; sweep the splits")
    ap.add_argument("--rechoose", metavar="JSON",
                    help="no sweep: choose the entries again from the timings of a tuning.json")
    args = ap.parse_args()
    if args.rechoose:
        with open(args.rechoose) as f:
            rec = json.load(f)
        single, mixed, splits, batch = record_timings(rec)
        os.makedirs(args.out_dir, exist_ok=True)
        with open(os.path.join(args.out_dir, "tuning_table.inc"), "w") as f:
            f.write(render_inc(choose_single(single, mixed, splits), choose_batch(batch),
                               f"{rec.get('device', '?')}, timings of {os.path.basename(args.rechoose)}"))
        return

    import numpy as np
    import torch

    from paper_2003_04776_amd import pencils
    from paper_2003_04776_amd import rtgevc as rt

    dev = torch.cuda.get_device_properties(0)
    record = {"device": dev.name, "gcn_arch": getattr(dev, "gcnArchName", ""), "single": {}, "batch": {}}
    single, mixed, splits = {}, {}, {}
    sizes = [m for m in SINGLE_SIZES if not (args.quick and m > 8192)]
    for m in sizes:
        S, T, _ = pencils.schur_pencil(m, 500 + m, threads=16)
        Sd, Td = rt.colmajor_to_device(S), rt.colmajor_to_device(T)
        del S, T
        Z = rt.colmajor_empty(m)
        sc = torch.empty(m, dtype=torch.int32, device="cuda")
        info = torch.zeros(1, dtype=torch.int32, device="cuda")
        single[m], mixed[m] = {}, {}
        if args.splits_only:
            single[m][rt.resolve_opts(m, with_schedule=True)] = 0.0
            mixed[m][rt.resolve_opts(m, precision=1)] = 0.0
        else:
            for mb, band, schedule in single_candidates(m):
                t = time_single(m, mb, band, schedule, Sd, Td, Z, sc, info, args.reps)
                single[m][(mb, band, schedule)] = t
                record["single"].setdefault(str(m), {})[f"mb={mb},band={band},schedule={schedule}"] = round(t, 4)
                print(f"[tune] single m={m} mb={mb} band={band} schedule={schedule}: {t:.3f} ms", flush=True)
            for mb, band in mixed_candidates(m):
                t = time_single(m, mb, band, 1, Sd, Td, Z, sc, info, args.reps, precision=1)
                mixed[m][(mb, band)] = t
                record.setdefault("mixed", {}).setdefault(str(m), {})[f"mb={mb},band={band}"] = round(t, 4)
                print(f"[tune] mixed m={m} mb={mb} band={band}: {t:.3f} ms", flush=True)
        # the splits of the chosen tile size and band (the walker has no band updates)
        (mb, band, schedule), _ = min(single[m].items(), key=lambda kv: kv[1])
        (mbx, bandx), _ = min(mixed[m].items(), key=lambda kv: kv[1])
        record.setdefault("split_base", {})[str(m)] = {"fp64": f"mb={mb},band={band},schedule={schedule}",
                                                       "mixed": f"mb={mbx},band={bandx}"}
        splits[m] = {"fp64": {}, "mixed": {}}
        for split in SPLITS if schedule == 1 else (0,):
            t = time_single(m, mb, band, schedule, Sd, Td, Z, sc, info, args.reps, split=split)
            splits[m]["fp64"][split] = t
            record.setdefault("split", {}).setdefault(str(m), {})[f"fp64,split={split}"] = round(t, 4)
            print(f"[tune] split m={m} mb={mb} band={band} split={split}: {t:.3f} ms", flush=True)
        for split in SPLITS:
            t = time_single(m, mbx, bandx, 1, Sd, Td, Z, sc, info, args.reps, precision=1, split=split)
            splits[m]["mixed"][split] = t
            record.setdefault("split", {}).setdefault(str(m), {})[f"mixed,split={split}"] = round(t, 4)
            print(f"[tune] split mixed m={m} mb={mbx} band={bandx} split={split}: {t:.3f} ms", flush=True)
        del Sd, Td, Z
        torch.cuda.empty_cache()
    batch = {}
    for bi, (lo, hi) in enumerate(BATCH_BUCKETS):
        if args.splits_only:
            batch[(lo, hi)] = {rt.resolve_opts(hi, batched=True)[0]: 0.0}
            continue
        rng = np.random.default_rng(7000 + bi)
        ms = [int(v) for v in rng.integers(lo, hi, size=args.batch_count)]
        Sd, Td = [], []
        for i, m in enumerate(ms):
            S, T, _ = pencils.schur_pencil(m, 7100 + 100 * bi + i)
            Sd.append(rt.colmajor_to_device(S))
            Td.append(rt.colmajor_to_device(T))
        batch[(lo, hi)] = {}
        for mb in MBS:
            if mb > 2 * hi:
                continue
            t = time_batch(ms, mb, Sd, Td, args.reps)
            batch[(lo, hi)][mb] = t
            record["batch"].setdefault(f"{lo}-{hi}", {})[f"mb={mb}"] = round(t, 4)
            print(f"[tune] batch [{lo},{hi}) x{len(ms)} mb={mb}: {t:.3f} ms", flush=True)
        del Sd, Td
        torch.cuda.empty_cache()
    ch_single, ch_batch = choose_single(single, mixed, splits), choose_batch(batch)
    record["chosen_single"] = [{"m_max": a, "mb": b, "band": c, "schedule": d, "split": e, "mb_mixed": f,
                                "band_mixed": g, "split_mixed": h} for a, b, c, d, e, f, g, h in ch_single]
    record["chosen_batch"] = [{"m_max": a, "mb": b} for a, b in ch_batch]
    os.makedirs(args.out_dir, exist_ok=True)
    prev = os.path.join(args.out_dir, "tuning.json")
    if args.splits_only and os.path.exists(prev):
        # keep the timings of the sweep that chose the tile sizes, bands and schedules
        with open(prev) as f:
            old = json.load(f)
        for key in ("single", "mixed", "batch"):
            if key in old:
                record[key] = old[key]
    with open(os.path.join(args.out_dir, "tuning.json"), "w") as f:
        json.dump(record, f, indent=1)
    with open(os.path.join(args.out_dir, "tuning_table.inc"), "w") as f:
        f.write(render_inc(ch_single, ch_batch, f"{dev.name}, {time.strftime('%Y-%m-%d')}"))
    print(json.dumps({"chosen_single": record["chosen_single"], "chosen_batch": record["chosen_batch"]}), flush=True)


if __name__ == "__main__":
    main()
