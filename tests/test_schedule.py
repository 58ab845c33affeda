"""Host-side replay of the band wavefront schedule under stream and event semantics.

The schedule (``csrc/schedule.hpp``, the enqueue order of the tile solves and updates of
Algorithm 1 on two streams) is compiled with g++ into a small driver
(``tests/sched_check.cpp``) that replays it with vector clocks.  No GPU is used."""
from __future__ import annotations

import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2003_04776_amd", "csrc")


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    exe = str(tmp_path_factory.mktemp("sched") / "sched_check")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, os.path.join(HERE, "sched_check.cpp"), "-o", exe],
                   check=True)
    return exe


def _run(exe, rows, band, drop=-1, split=0):
    r = subprocess.run([exe, str(rows), str(band), str(drop), str(split)], capture_output=True, text=True)
    return r.returncode, r.stdout.strip()


@pytest.mark.parametrize("band", [1, 2, 3, 4, 5, 8])
def test_band_schedule_orders_every_conflict(checker, band):
    """Every pair of launches that touch the same tiles or W slots is ordered, every update
    term is applied once, sources are solved before use, targets are complete before their
    solve, and a tile's sources come in descending order: for tile counts 1 .. 70 and the
    256 tiles of order 32768 with tile 128."""
    for rows in list(range(1, 71)) + [129, 256]:
        rc, out = _run(checker, rows, band)
        assert rc == 0 and out.startswith("OK"), (rows, band, out)


@pytest.mark.parametrize("split", [1, 7, 64, 1024, 4096])
@pytest.mark.parametrize("band", [1, 4, 8])
def test_split_updates_keep_every_order(checker, band, split):
    """The update of the rows above a band in several launches of about `split` tiles: the
    same checks, and more launches than with one launch per band where a band's update has
    more tiles than that."""
    for rows in list(range(1, 41)) + [128, 256]:
        rc, out = _run(checker, rows, band, split=split)
        assert rc == 0 and out.startswith("OK"), (rows, band, split, out)
        n_split = int(out.split()[1])
        n_one = int(_run(checker, rows, band)[1].split()[1])
        assert n_split >= n_one
        if split == 1 and rows > 2 * band + 1:
            assert n_split > n_one


def test_replay_detects_a_missing_wait(checker):
    """Dropping the wait that orders U1(b) after U2(b + 1) (both read-modify-write the tiles
    of band b - 1) is reported as a race, band by band: the replay would have caught the
    schedule without that wait."""
    rows, band = 20, 3
    rc, out = _run(checker, rows, band)
    n_wait = int(out.split()[-2])
    races = []
    for d in range(n_wait):
        rc, out = _run(checker, rows, band, d)
        if rc != 0:
            assert out.startswith("RACE"), out
            races.append(out)
    u1_u2 = [r for r in races if r.count("update(") == 2]
    # bands 5 .. 1 each have a U1 that must wait for the previous band's U2
    assert len(u1_u2) == 5, races


def _run_batch(exe, rows, band, steps, cr, drop=-1):
    r = subprocess.run([exe, "batch", str(rows), str(band), str(steps), str(cr), str(drop)], capture_output=True,
                       text=True)
    return r.returncode, r.stdout.strip()


@pytest.mark.parametrize("cr", [0, 1, 3])
@pytest.mark.parametrize("band", [1, 2, 3, 4])
def test_batch_schedule_orders_every_conflict(checker, band, cr):
    """The batch lock-step schedule as each pencil of a group sees it (its own tile rows,
    inside a group whose largest pencil has up to three bands more): the same checks as for
    one pencil, with the update of the rows above a band in one launch or in launches of
    cr tile rows."""
    for rows in range(1, 41):
        nb = (rows + band - 1) // band
        for steps in (nb, nb + 1, nb + 3):
            rc, out = _run_batch(checker, rows, band, steps, cr)
            assert rc == 0 and out.startswith("OK"), (rows, band, steps, cr, out)


def test_batch_replay_detects_a_missing_wait(checker):
    """Dropping any one of the batch schedule's waits that order two streams is reported as
    a race for a pencil with enough bands (each wait is the only order between some pair)."""
    rows, band = 20, 2
    steps = (rows + band - 1) // band
    rc, out = _run_batch(checker, rows, band, steps, 0)
    assert rc == 0, out
    n_wait = int(out.split()[-2])
    raced = 0
    for d in range(n_wait):
        rc, out = _run_batch(checker, rows, band, steps, 0, d)
        if rc != 0:
            assert out.startswith("RACE"), out
            raced += 1
    # every wait is needed but the side stream's start, the first step's wait for a U2 that
    # does not exist, and the final join (the last U2 is already ordered before the last U1)
    assert raced == n_wait - 3, (raced, n_wait)
