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
    ch = autotune.choose_single(res, mixed)
    # sizes without mixed timings repeat the FP64 tile size and band in the mixed columns
    assert ch == [(1024, 128, 4, 1, 128, 1), (11585, 128, 1, 2, 128, 1), (None, 128, 4, 1, 128, 8)]
    chb = autotune.choose_batch({(64, 128): {32: 1.0, 64: 2.0}, (128, 256): {64: 1.0, 128: 3.0}})
    assert chb == [(128, 32), (None, 64)]
    text = autotune.render_inc(ch, chb, "test")
    assert "{INT64_MAX, 128, 4, 1, 128, 8}" in text and "{128, 32}" in text


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
    for m_max, mb, band, schedule, mbx, bandx in single:
        assert int(mb) in (32, 64, 128) and 1 <= int(band) <= 8 and int(schedule) in (1, 2)
        assert int(mbx) in (32, 64, 128) and 1 <= int(bandx) <= 8
    for m_max, mb in batch:
        assert int(mb) in (32, 64, 128)
    # the library resolves automatic options from this table
    lo = 1
    for m_max, mb, band, schedule, mbx, bandx in single:
        for m in {lo, (lo + int(m_max)) // 2 if m_max != "INT64_MAX" else lo + 1000}:
            assert rt.resolve_opts(m, with_schedule=True) == (int(mb), int(band), int(schedule)), (m, mb, band)
            # mixed precision: its own tile size and band, always the band schedule
            assert rt.resolve_opts(m, precision=1, with_schedule=True) == (int(mbx), int(bandx), 1)
        if m_max != "INT64_MAX":
            lo = int(m_max) + 1
    lo = 1
    for m_max, mb in batch:
        assert rt.resolve_opts(lo, batched=True) == (int(mb), 2)   # lock-step band
        if m_max != "INT64_MAX":
            lo = int(m_max) + 1
    # explicit options win
    assert rt.resolve_opts(5000, mb=32, band=3) == (32, 3)
