"""Autotuner host logic (no GPU): choosing table entries from timings, rendering the
compiled-in table, and the library resolving automatic options from the table it was
built with."""
from __future__ import annotations

import os
import re

from paper_2003_04776_amd import autotune
from paper_2003_04776_amd import rtgevc as rt

HERE = os.path.dirname(os.path.abspath(autotune.__file__))


def test_choose_single_and_batch():
    res = {256: {(64, 1, 1): 2.0, (128, 4, 1): 1.0}, 4096: {(64, 2, 1): 5.0, (128, 1, 2): 4.0},
           32768: {(128, 4, 1): 9.0}}
    mixed = {256: {(64, 2): 3.0, (128, 1): 2.0}, 32768: {(128, 8): 7.0, (128, 4): 8.0}}
    splits = {32768: {"fp64": {0: 9.0, 1024: 9.5}, "mixed": {0: 7.0, 2048: 6.5, 4096: 6.8}}}
    ch = autotune.choose_single(res, mixed, splits)
    # sizes without mixed timings repeat the FP64 tile size and band in the mixed columns;
    # sizes without split timings take one launch per band (0)
    assert ch == [(1024, 128, 4, 1, 0, 128, 1, 0), (11585, 128, 1, 2, 0, 128, 1, 0),
                  (None, 128, 4, 1, 0, 128, 8, 2048)]
    # one tile size for every bucket: the least summed time over the buckets that timed it
    chb = autotune.choose_batch({(64, 128): {32: 1.0, 64: 2.0}, (128, 256): {32: 5.0, 64: 1.0, 128: 3.0}})
    assert chb == [(128, 64), (None, 64)]
    assert autotune.choose_batch({(64, 128): {32: 1.0}, (128, 256): {64: 1.0}}) == [(128, 32), (None, 64)]
    text = autotune.render_inc(ch, chb, "test")
    assert "{INT64_MAX, 128, 4, 1, 0, 128, 8, 2048}" in text and "{128, 64}" in text


def test_choose_split_keeps_one_launch_within_noise():
    """A split is tabulated only when it beats one launch per band by more than 1 %, and
    splits at least as large as the pencil's tile count (the same launches as one per band)
    are not candidates."""
    assert autotune.choose_split({0: 100.0, 1024: 99.5, 4096: 101.0}, 10 ** 6) == 0
    assert autotune.choose_split({0: 100.0, 1024: 90.0, 4096: 95.0}, 10 ** 6) == 1024
    assert autotune.choose_split({0: 100.0, 8192: 90.0}, 16) == 0
    assert autotune.choose_split({}, 16) == 0 and autotune.choose_split(None) == 0


def test_rechoose_from_recorded_timings():
    """record_timings reads back what a sweep records (tile sizes, bands, schedules, the split
    sweep on a built table's choices, batches), and choosing from it gives the same table."""
    rec = {"single": {"4096": {"mb=64,band=2,schedule=1": 5.0, "mb=128,band=1,schedule=2": 4.0}},
           "mixed": {"4096": {"mb=64,band=8": 6.0}},
           "split_base": {"32768": {"fp64": "mb=128,band=4,schedule=1", "mixed": "mb=128,band=8"}},
           "split": {"32768": {"fp64,split=0": 500.0, "fp64,split=1024": 600.0, "mixed,split=0": 400.0,
                               "mixed,split=1024": 360.0}},
           "batch": {"64-128": {"mb=32": 1.0, "mb=64": 2.0}}}
    single, mixed, splits, batch = autotune.record_timings(rec)
    assert single == {4096: {(64, 2, 1): 5.0, (128, 1, 2): 4.0}, 32768: {(128, 4, 1): 0.0}}
    assert mixed == {4096: {(64, 8): 6.0}, 32768: {(128, 8): 0.0}}
    assert splits == {32768: {"fp64": {0: 500.0, 1024: 600.0}, "mixed": {0: 400.0, 1024: 360.0}}}
    assert batch == {(64, 128): {32: 1.0, 64: 2.0}}
    assert autotune.choose_single(single, mixed, splits) == [(11585, 128, 1, 2, 0, 64, 8, 0),
                                                            (None, 128, 4, 1, 0, 128, 8, 1024)]


def _parse_inc():
    text = open(os.path.join(HERE, "csrc", "tuning_table.inc")).read()
    single_txt = text.split("kTuneSingle[] = {")[1].split("};")[0]
    batch_txt = text.split("kTuneBatch[] = {")[1].split("};")[0]
    single = [tuple(x.strip() for x in e.split(",")) for e in re.findall(r"\{([^{}]*)\}", single_txt)]
    batch = [tuple(x.strip() for x in e.split(",")) for e in re.findall(r"\{([^{}]*)\}", batch_txt)]
    return single, batch


def test_compiled_table_is_well_formed_and_used():
    single, batch = _parse_inc()
    assert single[-1][0] == "INT64_MAX" and batch[-1][0] == "INT64_MAX"
    bounds = [int(e[0]) for e in single[:-1]]
    assert bounds == sorted(bounds)
    for m_max, mb, band, schedule, split, mbx, bandx, splitx in single:
        assert int(mb) in (32, 64, 128) and 1 <= int(band) <= 8 and int(schedule) in (1, 2)
        assert int(mbx) in (32, 64, 128) and 1 <= int(bandx) <= 8
        assert int(split) >= 0 and int(splitx) >= 0
    for m_max, mb in batch:
        assert int(mb) in (32, 64, 128)
    # the library resolves automatic options from this table
    lo = 1
    for m_max, mb, band, schedule, split, mbx, bandx, splitx in single:
        for m in {lo, (lo + int(m_max)) // 2 if m_max != "INT64_MAX" else lo + 1000}:
            sp = int(split) if int(split) > 0 else -1
            assert rt.resolve_opts(m, with_schedule=True, with_split=True) == (int(mb), int(band), int(schedule),
                                                                                  sp), (m, mb, band)
            # mixed precision: its own tile size, band and split, always the band schedule
            spx = int(splitx) if int(splitx) > 0 else -1
            assert rt.resolve_opts(m, precision=1, with_schedule=True, with_split=True) == (int(mbx), int(bandx),
                                                                                             1, spx)
            # a split of the caller's overrides the table; a tile size or band other than the
            # table's takes one launch unless a split is given
            assert rt.resolve_opts(m, split=333, with_split=True)[-1] == 333
            assert rt.resolve_opts(m, split=-1, with_split=True)[-1] == -1
            other = 32 if int(mb) != 32 else 64
            assert rt.resolve_opts(m, mb=other, with_split=True)[-1] == -1
        if m_max != "INT64_MAX":
            lo = int(m_max) + 1
    lo = 1
    for m_max, mb in batch:
        assert rt.resolve_opts(lo, batched=True) == (int(mb), 3)   # lock-step band
        if m_max != "INT64_MAX":
            lo = int(m_max) + 1
    # explicit options win
    assert rt.resolve_opts(5000, mb=32, band=3) == (32, 3)
