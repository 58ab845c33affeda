"""Refinement of the mixed-precision eigenvectors against an FP64 residual (max_refine,
refine_bits), through the C ABI.

The measure is the componentwise backward error omega_c = ||(beta S - alpha T) z||_1 /
||beta |S||z| + |alpha||T||z| ||_1 of each eigenvector (helpers.backward_errors, exact, in
FP64): an FP64 substitution keeps it at a few units of roundoff (pinned on the oracle).  The
library estimates it with a sketch, refines the columns whose estimate is above the
threshold and reports (info bit 64) the columns still above it after the last sweep.
Every result is also compared with the CPU oracle (1e-10 on well-conditioned columns)."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from helpers import backward_errors, left_residuals
from paper_2003_04776_amd import pencils

pytestmark = pytest.mark.gpu

U = 2.0 ** -53
TOL = 1e-10
WELL = 1e-12
INFO_REFINE = 64


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _pencil(kind, m, seed):
    return pencils.schur_pencil(m, seed, kind=kind)


def _run(S, T, left=False, select=None, **kw):
    torch = _torch()
    from paper_2003_04776_amd import rtgevc as rt
    m = S.shape[0]
    Sd, Td = rt.colmajor_to_device(S), rt.colmajor_to_device(T)
    res = rt.Solver(m, left=left, **kw).run(Sd, Td, select=select)
    torch.cuda.synchronize()
    return res.Z.cpu().numpy(), res.scales.cpu().numpy(), int(res.info.item())


def _omega(S, T, Z):
    ar, ai, be, _ = oracle.eigvals(S, T)
    return np.array(list(backward_errors(S, T, Z, ar, ai, be).values()))


def _oracle_err(S, T, Z, select=None):
    Zo, _, _ = oracle.tgevc(S, T, select=select)
    Zl, _, _ = oracle.tgevc(S, T, select=select, precision="ld")
    well = np.max(np.abs(Zo - Zl), axis=0) <= WELL
    err = np.max(np.abs(Z - Zo), axis=0)
    return float(np.max(err[well])), int(well.sum())


CASES = [("normal", 1000, 64, 4, 601), ("normal", 700, 128, 2, 602), ("stress", 600, 64, 8, 603),
         ("unbalanced", 800, 64, 4, 610), ("unbalanced", 600, 128, 8, 611),
         ("general", 500, 32, 2, 604), ("general_stress", 450, 64, 1, 605)]


@pytest.mark.parametrize("kind,m,mb,band,seed", CASES)
def test_default_threshold(kind, m, mb, band, seed):
    """With the default threshold (the residual bound 64 m u on omega) the mixed results of
    these pencils need no sweep: the refined call returns the unrefined result bit for bit."""
    _say(f"refine default: {kind} m={m} mb={mb} band={band}")
    S, T, _ = _pencil(kind, m, seed)
    Z0, s0, i0 = _run(S, T, mb=mb, band=band, precision=1, max_refine=-1)
    Z3, s3, i3 = _run(S, T, mb=mb, band=band, precision=1)
    om = _omega(S, T, Z0)
    _say(f"  omega mixed: median {np.median(om):.2e} max {om.max():.2e}; bound {64 * m * U:.2e}")
    assert om.max() <= 64 * m * U
    assert i3 == i0 and not (i3 & INFO_REFINE)
    assert np.array_equal(Z0, Z3) and np.array_equal(s0, s3)


@pytest.mark.parametrize("kind,m,mb,band,seed", CASES)
def test_refinement_to_fp64_level(kind, m, mb, band, seed):
    """Threshold 2^-50: the sweeps bring every column to the backward error of the FP64
    path, and the eigenvectors to the oracle at least as closely as before."""
    _say(f"refine 2^-50: {kind} m={m} mb={mb} band={band}")
    S, T, _ = _pencil(kind, m, seed)
    Zm, _, im = _run(S, T, mb=mb, band=band, precision=1, max_refine=-1)
    Zr, _, ir = _run(S, T, mb=mb, band=band, precision=1, refine_bits=50)
    Zf, _, i_f = _run(S, T, mb=mb, band=band)
    om_m, om_r, om_f = _omega(S, T, Zm), _omega(S, T, Zr), _omega(S, T, Zf)
    em, _ = _oracle_err(S, T, Zm)
    er, nw = _oracle_err(S, T, Zr)
    ef, _ = _oracle_err(S, T, Zf)
    _say(f"  omega max: mixed {om_m.max():.2e} refined {om_r.max():.2e} fp64 {om_f.max():.2e}; "
         f"oracle err: mixed {em:.2e} refined {er:.2e} fp64 {ef:.2e} ({nw} cols); info {im} {ir} {i_f}")
    assert om_r.max() <= 16 * U
    assert om_r.max() <= max(om_m.max(), 16 * U)
    assert er <= TOL and er <= max(2 * em, 1e-13)
    assert (ir & ~INFO_REFINE) == im


def test_unreachable_threshold_sets_info_bit():
    """Threshold 2^-100 (below what FP64 can reach): every sweep refines every column, the
    last estimate reports them (info bit 64), and the vectors stay correct."""
    S, T, _ = _pencil("normal", 400, 606)
    Z, _, info = _run(S, T, mb=64, band=4, precision=1, refine_bits=100)
    assert info & INFO_REFINE
    err, _ = _oracle_err(S, T, Z)
    assert err <= TOL
    assert _omega(S, T, Z).max() <= 16 * U


def test_refinement_unnormalised_and_selected():
    """Unnormalised output (mantissa and exponent) and a selection: the refined columns keep
    their exponents, unselected columns stay zero, represented vectors match the oracle."""
    m = 600
    S, T, blk = _pencil("stress", m, 607)
    rng = np.random.default_rng(607)
    sel = (rng.random(m) < 0.3).astype(np.int32)
    Zm, sm, _ = _run(S, T, mb=64, band=2, precision=1, max_refine=-1, normalize=False, select=sel)
    Zr, sr, _ = _run(S, T, mb=64, band=2, precision=1, refine_bits=50, normalize=False, select=sel)
    assert np.array_equal(sm, sr)
    Zo, _, _ = oracle.tgevc(S, T, select=sel)
    from helpers import normalized_columns
    chosen = [c for c in range(m) if np.any(Zo[:, c] != 0.0)]
    nr = normalized_columns(Zr, blk, chosen)
    err = max(float(np.max(np.abs(nr[c] - Zo[:, c]))) for c in chosen)
    assert err <= TOL
    off = [c for c in range(m) if c not in set(chosen)]
    assert not np.any(Zr[:, off])


def test_left_refinement():
    S, T, _ = _pencil("normal", 500, 608)
    Y, _, info = _run(S, T, left=True, mb=64, band=4, precision=1, refine_bits=50)
    Yo, _, _ = oracle.tgevc_left(S, T)
    assert float(np.max(np.abs(Y - Yo))) <= TOL
    ar, ai, be, _ = oracle.eigvals(S, T)
    eta = left_residuals(S, T, Y, ar, ai, be)
    assert max(eta.values()) <= 64 * 500 * U


def test_timed_reports_refinement():
    torch = _torch()
    from paper_2003_04776_amd import rtgevc as rt
    m = 800
    S, T, _ = _pencil("normal", m, 609)
    Sd, Td = rt.colmajor_to_device(S), rt.colmajor_to_device(T)
    sv = rt.Solver(m, mb=64, band=4, precision=1, refine_bits=50)
    Z = rt.colmajor_empty(m)
    sc = torch.empty(m, dtype=torch.int32, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    st = sv.run_timed(Sd, Td, Z, sc, info)
    assert st["sweeps"] == 1 and st["refine_ms"] > 0.0
    Zr, _, _ = _run(S, T, mb=64, band=4, precision=1, refine_bits=50)
    assert np.array_equal(Z.cpu().numpy(), Zr)


@pytest.mark.parametrize("kind,m,seed", [("normal", 1000, 620), ("general", 600, 621), ("unbalanced", 700, 623)])
def test_forced_sweep_reaches_fp64_forward_error(kind, m, seed):
    """The mixed result's backward error is already at the FP64 level, but its error against
    the oracle is larger; one forced sweep (threshold 2^-100, every column refined) brings that
    error to the FP64 path's level: the correction works on every column."""
    _say(f"forced sweep: {kind} m={m}")
    S, T, _ = _pencil(kind, m, seed)
    Zm, _, _ = _run(S, T, mb=64, band=4, precision=1, max_refine=-1)
    Zr, _, ir = _run(S, T, mb=64, band=4, precision=1, refine_bits=100, max_refine=1)
    Zf, _, _ = _run(S, T, mb=64, band=4)
    em, _ = _oracle_err(S, T, Zm)
    er, _ = _oracle_err(S, T, Zr)
    ef, _ = _oracle_err(S, T, Zf)
    _say(f"  oracle err: mixed {em:.2e} forced {er:.2e} fp64 {ef:.2e}; info {ir}")
    assert ir & INFO_REFINE
    assert er <= max(4 * ef, 1e-13)
    assert _omega(S, T, Zr).max() <= 16 * U


def test_columns_beyond_the_double_range_are_not_refined():
    """Overflow-stress eigenvectors span far more than the double range; normalised, their
    smallest segments are flushed to zero and an FP64 residual cannot refine them.  A forced
    threshold leaves them as they are and reports them (info bit 64)."""
    S, T, _ = _pencil("stress", 700, 622)
    Zm, _, im = _run(S, T, mb=64, band=4, precision=1, max_refine=-1)
    Zr, _, ir = _run(S, T, mb=64, band=4, precision=1, refine_bits=100, max_refine=1)
    assert ir & INFO_REFINE and (ir & ~INFO_REFINE) == im
    err, _ = _oracle_err(S, T, Zr)
    assert err <= TOL
    # only the few eigenvectors near the top (a handful of rows) fit the double range
    changed = np.any(Zr != Zm, axis=0)
    assert changed.mean() < 0.05, changed.sum()
