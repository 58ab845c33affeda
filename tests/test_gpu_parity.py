"""Parity of the HIP path (through the C ABI) with the CPU oracle, element by element
on seeded inputs, plus the residual of S V D - T V B = 0 (Section 2.2), the overflow-
stress invariants and the edge cases.

Bar: normalised eigenvectors within 1e-10 of the double-precision oracle on every
well-conditioned column (a column whose double and extended-precision oracle results
agree to 1e-12); the normwise residual eta_c <= 64 m 2^-53 on every column."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from helpers import block_kinds_from_S, residuals, residuals_torch
from paper_2003_04776_amd import pencils

pytestmark = pytest.mark.gpu

U = 2.0 ** -53
TOL = 1e-10
WELL = 1e-12


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def run_gpu(S, T, mb=0, select=None, normalize=True, ld=None, band=0, precision=0, split=0, schedule=0):
    torch = _torch()
    from paper_2003_04776_amd import rtgevc as rt
    m = S.shape[0]
    Sd = rt.colmajor_to_device(S, ld=ld)
    Td = rt.colmajor_to_device(T, ld=ld)
    solver = rt.Solver(m, mb=mb, normalize=normalize, band=band, precision=precision, split=split,
                       schedule=schedule)
    res = solver.run(Sd, Td, select=select)
    torch.cuda.synchronize()
    return res.Z.cpu().numpy(), res.scales.cpu().numpy(), int(res.info.item())


def compare(S, T, Zg, select=None, cols=None, tol=TOL):
    """Max error over well-conditioned columns; also returns the per-column errors."""
    Zo, _, _ = oracle.tgevc(S, T, select=select)
    Zl, _, _ = oracle.tgevc(S, T, select=select, precision="ld")
    m = S.shape[0]
    cols = range(m) if cols is None else cols
    errs, worst, nill = [], 0.0, 0
    for c in cols:
        e = float(np.max(np.abs(Zg[:, c] - Zo[:, c]))) if m else 0.0
        errs.append(e)
        if np.max(np.abs(Zo[:, c] - Zl[:, c])) <= WELL:
            worst = max(worst, e)
        else:
            nill += 1
    return worst, np.array(errs), nill


SMALL = [(1, 32, 0), (2, 32, 1), (3, 32, 2), (5, 32, 3), (17, 32, 4), (31, 32, 5), (32, 32, 6),
         (33, 32, 7), (64, 32, 8), (65, 64, 9), (100, 32, 10), (129, 64, 11), (200, 64, 12),
         (256, 0, 0), (257, 128, 13), (300, 128, 14), (513, 128, 15), (700, 64, 16), (1000, 128, 17)]


@pytest.mark.parametrize("m,mb,seed", SMALL)
def test_parity_small(m, mb, seed):
    _say(f"[parity] m={m} mb={mb} seed={seed}")
    S, T, blk = pencils.schur_pencil(m, seed)
    Zg, sc, info = run_gpu(S, T, mb=mb)
    assert info == 0, info
    assert np.isfinite(Zg).all()
    assert (sc == 0).all()
    worst, errs, nill = compare(S, T, Zg)
    _say(f"   max err {worst:.3e} (median {np.median(errs):.1e}, ill {nill})")
    assert worst <= TOL
    ar, ai, be, _ = oracle.eigvals(S, T)
    eta = residuals(S, T, Zg, ar, ai, be)
    assert max(eta.values()) <= 64 * m * U


@pytest.mark.parametrize("seed", [0, 1, 2, 3, 4])
def test_order_256_seeds(seed):
    """The order-256 workload on its five seeds: every column against the oracle, the
    normwise residual and the componentwise backward error of every column."""
    from helpers import backward_errors
    S, T, blk = pencils.schur_pencil(256, seed)
    Zg, sc, info = run_gpu(S, T)
    assert info == 0
    worst, errs, nill = compare(S, T, Zg)
    assert worst <= TOL and nill <= 2
    ar, ai, be, _ = oracle.eigvals(S, T)
    assert max(residuals(S, T, Zg, ar, ai, be).values()) <= 64 * 256 * U
    assert max(backward_errors(S, T, Zg, ar, ai, be).values()) <= 16 * U


@pytest.mark.parametrize("m,mb,seed,kind,precision", [(300, 64, 40, "zeroinf", 0), (700, 128, 41, "zeroinf", 0),
                                                      (701, 128, 42, "zeroinf", 1), (1000, 64, 43, "degenerate", 0),
                                                      (1000, 128, 44, "degenerate", 1)])
def test_zero_and_infinite_eigenvalues(m, mb, seed, kind, precision):
    """Zero (s_jj = 0) and infinite (t_jj = 0, beta = 0) eigenvalues, as in the pencils of
    the paper's experiments: one of each (distinct eigenvalues), or about 1 percent of each
    (repeated: their singular pivots are perturbed, info bit 16, and the columns whose
    double and extended-precision oracles disagree are left out of the comparison)."""
    torch = _torch()
    from paper_2003_04776_amd import rtgevc as rt
    _say(f"[zero/inf] m={m} mb={mb} seed={seed} kind={kind} precision={precision}")
    S, T, blk = pencils.schur_pencil(m, seed, kind)
    Sd, Td = rt.colmajor_to_device(S), rt.colmajor_to_device(T)
    r = rt.Solver(m, mb=mb, precision=precision).run(Sd, Td)
    torch.cuda.synchronize()
    Zg, info = r.Z.cpu().numpy(), int(r.info.item())
    if kind == "zeroinf":
        assert info == 0, info
    else:
        assert info & ~16 == 0, info
    assert np.isfinite(Zg).all()
    worst, errs, nill = compare(S, T, Zg)
    _say(f"   max err {worst:.3e} (ill {nill})")
    assert worst <= TOL
    ar, ai, be, _ = oracle.eigvals(S, T)
    assert (be == 0).sum() >= 1 and ((ar == 0) & (ai == 0)).sum() >= 1
    eta = residuals(S, T, Zg, ar, ai, be)
    assert max(eta.values()) <= 64 * m * U


@pytest.mark.parametrize("m,mb,band,seed", [(300, 32, 1, 30), (301, 32, 2, 31), (333, 32, 3, 32),
                                             (450, 32, 4, 33), (1000, 64, 3, 34), (1100, 128, 4, 35),
                                             (700, 64, 1, 36)])
def test_parity_bands(m, mb, band, seed):
    """Every band size applies the same updates (grouped differently): same eigenvectors.  The
    band wavefront is asked for by name (the automatic choice for orders up to 512 is the
    walker, which has no bands), so bands of more than one row run as chain launches."""
    _say(f"[band] m={m} mb={mb} band={band} seed={seed}")
    S, T, blk = pencils.schur_pencil(m, seed)
    Zg, sc, info = run_gpu(S, T, mb=mb, band=band, schedule=1)
    assert info == 0
    worst, errs, nill = compare(S, T, Zg)
    assert worst <= TOL
    Zs, scs, _ = run_gpu(pencils.schur_pencil(m, seed + 100, "stress")[0],
                         pencils.schur_pencil(m, seed + 100, "stress")[1], mb=mb, band=band, normalize=False,
                         schedule=1)
    assert np.isfinite(Zs).all() and (scs >= 0).all()


@pytest.mark.parametrize("m,mb,seed", [(60, 32, 200), (300, 64, 201), (521, 128, 202)])
def test_parity_stress(m, mb, seed):
    """Overflow-stress pencils: unscaled substitution overflows within a few rows."""
    _say(f"[stress] m={m} mb={mb} seed={seed}")
    S, T, blk = pencils.schur_pencil(m, seed, "stress")
    Zg, sc, info = run_gpu(S, T, mb=mb, normalize=False)
    assert info & ~16 == 0, info
    assert np.isfinite(Zg).all()
    assert (sc >= 0).all() and sc.max() > 1000
    assert np.abs(Zg).max() <= 2.0 ** 1020
    Zn, _, _ = run_gpu(S, T, mb=mb)
    worst, errs, nill = compare(S, T, Zn)
    _say(f"   max err {worst:.3e} ill {nill} max scale {sc.max()}")
    assert worst <= TOL
    ar, ai, be, _ = oracle.eigvals(S, T)
    eta = residuals(S, T, Zn, ar, ai, be)
    assert max(eta.values()) <= 64 * m * U


def test_unnormalised_representation():
    """2^scales[c] * Z[:, c] represents the eigenvector: normalising it gives the
    oracle's normalised eigenvector."""
    m = 700
    S, T, blk = pencils.schur_pencil(m, 21)
    Zu, sc, info = run_gpu(S, T, mb=64, normalize=False)
    assert info == 0 and (sc >= 0).all()
    Zo, _, _ = oracle.tgevc(S, T)
    for c in range(m):
        p = c - 1 if blk[c] == 2 else c
        if blk[p] == 1:
            n = (np.abs(Zu[:, p]) + np.abs(Zu[:, p + 1])).max()
        else:
            n = np.abs(Zu[:, p]).max()
        assert sc[c] == sc[p]
        assert np.max(np.abs(Zu[:, c] / n - Zo[:, c])) <= TOL


@pytest.mark.parametrize("mb,precision", [(64, 0), (128, 1)])
def test_leading_dimension_padding(mb, precision):
    m = 301
    S, T, blk = pencils.schur_pencil(m, 22, ld=m + 7)
    Zg, sc, info = run_gpu(S, T, mb=mb, ld=m + 7, precision=precision)
    assert info == 0
    worst, _, _ = compare(np.asfortranarray(S), np.asfortranarray(T), Zg)
    assert worst <= TOL


@pytest.mark.parametrize("mb,precision", [(64, 0), (128, 1)])
def test_select_subset(mb, precision):
    m = 400
    S, T, blk = pencils.schur_pencil(m, 23)
    rng = np.random.default_rng(0)
    sel = (rng.random(m) < 0.2).astype(np.int32)
    pairs = np.nonzero(blk == 1)[0]
    sel[pairs[0]] = 1
    sel[pairs[0] + 1] = 0           # closure needed
    Zg, sc, info = run_gpu(S, T, mb=mb, select=sel, precision=precision)
    assert info == 32
    Zo, _, io = oracle.tgevc(S, T, select=sel)
    assert io == 32
    assert np.max(np.abs(Zg - Zo)) <= TOL
    on = sel.astype(bool) | np.roll(sel.astype(bool) & (blk == 1), 1) | np.roll(sel.astype(bool) & (blk == 2), -1)
    assert not Zg[:, ~on].any()


@pytest.mark.parametrize("normalize", [True, False])
def test_select_consolidation_ld(normalize):
    """Consolidation with a selection and a padded output: five groups of 256 columns and a tail
    (the rescaling workgroups take their columns in runs of 32 per XCD), unselected columns and
    the rows below each eigenvalue's tile zero, the padding rows of Z untouched."""
    torch = _torch()
    from paper_2003_04776_amd import rtgevc as rt
    m, ldz = 1300, 1303
    S, T, blk = pencils.schur_pencil(m, 29)
    rng = np.random.default_rng(5)
    sel = (rng.random(m) < 0.3).astype(np.int32)
    Sd, Td = rt.colmajor_to_device(S), rt.colmajor_to_device(T)
    Zbuf = torch.full((m, ldz), 7.0, dtype=torch.float64, device="cuda")   # column-major, ld = ldz
    Z = Zbuf.t()[:m]
    r = rt.Solver(m, mb=64, band=2, schedule=1, normalize=normalize).run(
        Sd, Td, select=sel, Z=Z)
    torch.cuda.synchronize()
    Zg = Z.cpu().numpy()
    assert (Zbuf[:, m:].cpu().numpy() == 7.0).all()
    Zo, _, io = oracle.tgevc(S, T, select=sel)
    assert int(r.info.item()) == io
    on = sel.astype(bool) | np.roll(sel.astype(bool) & (blk == 1), 1) | np.roll(sel.astype(bool) & (blk == 2), -1)
    assert not Zg[:, ~on].any()
    if normalize:
        assert np.max(np.abs(Zg - Zo)) <= TOL
    else:   # 2^scales[c] Z[:, c] represents the eigenvector: normalised, it is the oracle's
        for c in np.nonzero(on)[0]:
            p = c - 1 if blk[c] == 2 else c
            n = (np.abs(Zg[:, p]) + np.abs(Zg[:, p + 1])).max() if blk[p] == 1 else np.abs(Zg[:, p]).max()
            assert np.max(np.abs(Zg[:, c] / n - Zo[:, c])) <= TOL


def test_eigvals_entry_point():
    torch = _torch()
    from paper_2003_04776_amd import rtgevc as rt
    m = 500
    S, T, blk = pencils.schur_pencil(m, 24)
    solver = rt.Solver(m)
    ar, ai, be, info = solver.eigvals(rt.colmajor_to_device(S), rt.colmajor_to_device(T))
    torch.cuda.synchronize()
    oa, oi, ob, _ = oracle.eigvals(S, T)
    assert int(info.item()) == 0
    for x, y in ((ar, oa), (ai, oi), (be, ob)):
        x = x.cpu().numpy()
        assert np.allclose(x, y, rtol=1e-14, atol=1e-15)
    assert np.all(ob >= 0)
    s = np.maximum(ob, np.abs(oa) + np.abs(oi))
    assert np.all((s > 0.5) & (s <= 1.0))


def _all_pairs(m, seed):
    rng = np.random.default_rng(seed)
    S = np.triu(rng.standard_normal((m, m)))
    T = np.triu(rng.standard_normal((m, m)))
    for p in range(0, m - 1, 2):
        a, b, c, t = rng.standard_normal(), rng.uniform(0.5, 2), -rng.uniform(0.5, 2), rng.uniform(0.5, 2)
        S[p:p + 2, p:p + 2] = [[a, b], [c, a]]
        T[p:p + 2, p:p + 2] = [[t, 0], [0, t]]
    if m % 2:
        T[m - 1, m - 1] = rng.uniform(0.5, 2)
    return np.asfortranarray(S), np.asfortranarray(T)


@pytest.mark.parametrize("m,mb", [(130, 32), (256, 64), (383, 128)])
def test_all_pairs_and_all_real(m, mb):
    S, T = _all_pairs(m, m)
    Zg, sc, info = run_gpu(S, T, mb=mb)
    assert info == 0
    worst, _, _ = compare(S, T, Zg)
    assert worst <= TOL
    rng = np.random.default_rng(m)
    S2 = np.asfortranarray(np.triu(rng.standard_normal((m, m))))
    T2 = np.asfortranarray(np.triu(rng.standard_normal((m, m))))
    T2[np.diag_indices(m)] = rng.uniform(0.5, 2, m)
    Zg, sc, info = run_gpu(S2, T2, mb=mb)
    assert info == 0
    worst, _, _ = compare(S2, T2, Zg)
    assert worst <= TOL


def test_pair_on_every_tile_boundary():
    """A 2x2 block straddles every nominal boundary, so every tile is MB - 1 rows."""
    m, mb = 320, 32
    S, T = _all_pairs(m, 5)
    # shift the pair pattern by one so the pairs sit at (31, 32), (63, 64), ...
    S = np.asfortranarray(np.pad(S, ((1, 0), (1, 0)))[: m, : m])
    T = np.asfortranarray(np.pad(T, ((1, 0), (1, 0)))[: m, : m])
    S[0, 0], T[0, 0] = 0.3, 1.1
    kind = block_kinds_from_S(S)
    assert kind[31] == 1 and kind[63] == 1
    Zg, sc, info = run_gpu(S, T, mb=mb)
    assert info == 0
    worst, _, _ = compare(S, T, Zg)
    assert worst <= TOL


def test_info_bits():
    m = 50
    S, T, blk = pencils.schur_pencil(m, 25)
    S2 = S.copy(order="F")
    S2[3, 7] = np.nan
    _, _, info = run_gpu(S2, T, mb=32)
    assert info & 1
    S3 = S.copy(order="F")
    k = int(np.nonzero(blk == 1)[0][0])
    if k + 2 < m:
        S3[k + 2, k + 1] = 0.7
        _, _, info = run_gpu(S3, T, mb=32)
        assert info & 2


def test_common_power_of_two_prescale():
    """Entries near the top of the range: S and T are scaled by a common power of
    two (eigenvectors unchanged) and the prescale bit is set."""
    m = 200
    S, T, blk = pencils.schur_pencil(m, 26)
    f = 2.0 ** 1010
    Zg, sc, info = run_gpu(np.asfortranarray(S * f), np.asfortranarray(T * f), mb=64)
    assert info == 256
    Zr, _, _ = run_gpu(S, T, mb=64)
    assert np.max(np.abs(Zg - Zr)) <= 1e-14


@pytest.mark.parametrize("precision,kind", [(0, "normal"), (0, "stress"), (1, "normal")])
def test_split_updates_bitwise(precision, kind):
    """The update of the rows above a band in launches of 1, 40 or 500 tiles, against one
    launch per band: the same eigenvectors, scales and info bit for bit (tile 32, band 2, 40
    tile rows)."""
    m = 1270
    S, T, _ = pencils.schur_pencil(m, 28, kind=kind)
    ref = run_gpu(S, T, mb=32, band=2, precision=precision, split=-1, normalize=False)
    for split in (1, 40, 500):
        got = run_gpu(S, T, mb=32, band=2, precision=precision, split=split, normalize=False)
        _say("split", split, "precision", precision, kind)
        assert np.array_equal(got[0], ref[0]) and np.array_equal(got[1], ref[1]) and got[2] == ref[2]


def test_timed_with_many_launches():
    """The timed entry point with one launch per tile row of each band update (split 1, tile
    32, band 1: thousands of launches, each bracketed by events): no error, and the same
    eigenvectors as the untimed call."""
    torch = _torch()
    from paper_2003_04776_amd import rtgevc as rt
    m = 1270
    S, T, _ = pencils.schur_pencil(m, 29)
    Sd, Td = rt.colmajor_to_device(S), rt.colmajor_to_device(T)
    sv = rt.Solver(m, mb=32, band=1, split=1)
    Z = rt.colmajor_empty(m)
    sc = torch.zeros(m, dtype=torch.int32, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    st = sv.run_timed(Sd, Td, Z, sc, info)
    torch.cuda.synchronize()
    assert st["total_ms"] > 0 and st["update_ms"] > 0
    ref = sv.run(Sd, Td)
    torch.cuda.synchronize()
    assert torch.equal(Z, ref.Z)


def test_timed_side_stream_updates():
    """The timed entry point's side-stream figures: one launch per band with rows above the next
    band (one launch per band update, split 0), most of the update flops, never more than all."""
    torch = _torch()
    from paper_2003_04776_amd import rtgevc as rt
    m, band = 2000, 2
    S, T, _ = pencils.schur_pencil(m, 31)
    Sd, Td = rt.colmajor_to_device(S), rt.colmajor_to_device(T)
    sv = rt.Solver(m, mb=64, band=band, split=-1, schedule=1)
    Z = rt.colmajor_empty(m)
    sc = torch.zeros(m, dtype=torch.int32, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    st = sv.run_timed(Sd, Td, Z, sc, info)
    torch.cuda.synchronize()
    M = int(st["M"])
    _say(f"[timed side] M={M} side launches {st['n_side_update']:.0f}, flops {st['side_update_flops']:.3e} "
         f"of {st['update_flops']:.3e}")
    assert int(st["n_side_update"]) == max(0, (M - 1) // band - 1)
    assert 0.5 * st["update_flops"] < st["side_update_flops"] <= st["update_flops"]
    assert 0.0 < st["side_update_ms"] <= st["update_ms"]


def test_repeat_is_deterministic():
    m = 600
    S, T, _ = pencils.schur_pencil(m, 27)
    Z1, _, _ = run_gpu(S, T, mb=128)
    Z2, _, _ = run_gpu(S, T, mb=128)
    assert np.array_equal(Z1, Z2)


# ------------------------------------------------------------- full sizes --

def _full_size(m, seed, kind, nsample, mb=0, precision=0):
    torch = _torch()
    from paper_2003_04776_amd import rtgevc as rt
    _say(f"[full] m={m} kind={kind} seed={seed} precision={precision}: generating")
    S, T, blk = pencils.schur_pencil(m, seed, kind, threads=16)
    Sd, Td = rt.colmajor_to_device(S), rt.colmajor_to_device(T)
    solver = rt.Solver(m, mb=mb, precision=precision)
    _say("   running")
    res = solver.run(Sd, Td)
    torch.cuda.synchronize()
    info = int(res.info.item())
    assert info & ~16 == 0, info
    Z = res.Z
    assert bool(torch.isfinite(Z).all())
    _say("   residuals")
    ar, ai, be, _ = oracle.eigvals(S, T)
    eta = residuals_torch(Sd, Td, Z, ar, ai, be, blk)
    _say(f"   max eta {eta.max():.3e} bound {64 * m * U:.3e}")
    assert eta.max() <= 64 * m * U
    # the componentwise backward error of every column (a check that the normwise residual,
    # dominated by the largest entries of S and T, cannot make): an FP64 substitution keeps
    # it at a few units of roundoff
    from helpers import backward_errors_torch
    om = backward_errors_torch(Sd, Td, Z, ar, ai, be, blk)
    _say(f"   backward error: median {np.median(om):.2e} max {om.max():.2e}")
    assert om.max() <= 16 * U
    # oracle on a deterministic sample of columns spread over the range
    cols = sorted(set(np.linspace(0, m - 1, nsample).astype(int).tolist()))
    if precision == 1:
        # plus the columns where the mixed result differs most from the FP64 one
        Zf = rt.Solver(m, mb=mb).run(Sd, Td).Z
        torch.cuda.synchronize()
        top = torch.topk((Z - Zf).abs().amax(dim=0), 8).indices.cpu().numpy()
        del Zf
        cols = sorted(set(cols) | set(int(c) for c in top))
    sel = np.zeros(m, dtype=np.int32)
    sel[cols] = 1
    Zo, _, _ = oracle.tgevc(S, T, select=sel)
    Zl, _, _ = oracle.tgevc(S, T, select=sel, precision="ld")
    cols = np.nonzero(sel | np.roll(sel & (blk == 1), 1) | np.roll(sel & (blk == 2), -1))[0]
    Zs = Z[:, torch.from_numpy(cols).to(Z.device)].cpu().numpy()
    worst, nill = 0.0, 0
    for i, c in enumerate(cols):
        e = np.max(np.abs(Zs[:, i] - Zo[:, c]))
        if np.max(np.abs(Zo[:, c] - Zl[:, c])) <= WELL:
            worst = max(worst, e)
        else:
            nill += 1
    _say(f"   sampled {len(cols)} columns: max err {worst:.3e} ill {nill}")
    assert worst <= TOL


def test_full_size_8192():
    _full_size(8192, 100, "normal", 48)


def test_full_size_stress_8192():
    _full_size(8192, 200, "stress", 32)


def test_full_size_32768():
    _full_size(32768, 400, "normal", 12)


def test_full_size_mixed_8192():
    _full_size(8192, 100, "normal", 48, precision=1)


def test_full_size_mixed_stress_8192():
    _full_size(8192, 200, "stress", 32, precision=1)


def test_full_size_mixed_32768():
    _full_size(32768, 400, "normal", 12, precision=1)


# ---- persistent walker (schedule 2) ----

@pytest.mark.parametrize("m,mb,seed", [(1, 32, 400), (33, 32, 401), (200, 64, 402), (300, 128, 403),
                                       (700, 64, 404), (1000, 128, 405), (1500, 32, 406)])
def test_walker_parity(m, mb, seed):
    """The persistent walker against the oracle, and bit for bit against the band schedule
    with one row per band (same updates in the same order per tile)."""
    torch = _torch()
    from paper_2003_04776_amd import rtgevc as rt
    _say(f"[walker] m={m} mb={mb} seed={seed}")
    S, T, blk = pencils.schur_pencil(m, seed)
    Sd, Td = rt.colmajor_to_device(S), rt.colmajor_to_device(T)
    rw = rt.Solver(m, mb=mb, schedule=rt.SCHEDULE_WALKER).run(Sd, Td)
    rb = rt.Solver(m, mb=mb, band=1, schedule=1).run(Sd, Td)
    torch.cuda.synchronize()
    assert int(rw.info.item()) == 0
    Zw = rw.Z.cpu().numpy()
    assert np.array_equal(Zw, rb.Z.cpu().numpy())
    worst, errs, nill = compare(S, T, Zw)
    _say(f"   max err {worst:.3e} ill {nill}")
    assert worst <= TOL


def test_walker_stress_unnormalised():
    torch = _torch()
    from paper_2003_04776_amd import rtgevc as rt
    m, mb = 400, 64
    S, T, blk = pencils.schur_pencil(m, 410, "stress")
    Sd, Td = rt.colmajor_to_device(S), rt.colmajor_to_device(T)
    r = rt.Solver(m, mb=mb, normalize=False, schedule=rt.SCHEDULE_WALKER).run(Sd, Td)
    rb = rt.Solver(m, mb=mb, normalize=False, band=1, schedule=1).run(Sd, Td)
    torch.cuda.synchronize()
    Z, sc = r.Z.cpu().numpy(), r.scales.cpu().numpy()
    assert int(r.info.item()) & ~16 == 0
    assert np.isfinite(Z).all() and (sc >= 0).all() and sc.max() > 1000
    assert np.array_equal(Z, rb.Z.cpu().numpy()) and np.array_equal(sc, rb.scales.cpu().numpy())


def test_walker_repeat_is_deterministic():
    torch = _torch()
    from paper_2003_04776_amd import rtgevc as rt
    m = 900
    S, T, _ = pencils.schur_pencil(m, 411)
    Sd, Td = rt.colmajor_to_device(S), rt.colmajor_to_device(T)
    sol = rt.Solver(m, mb=32, schedule=rt.SCHEDULE_WALKER)
    a = sol.run(Sd, Td).Z.clone()
    for _ in range(3):
        b = sol.run(Sd, Td).Z
        torch.cuda.synchronize()
        assert torch.equal(a, b)


@pytest.mark.parametrize("grid", [1, 7, 64])
def test_walker_grid_counts(grid):
    """opts->grid: the walker with fewer workgroups than fit (one workgroup takes every task in
    ticket order) gives the automatic count's eigenvectors bit for bit."""
    torch = _torch()
    from paper_2003_04776_amd import rtgevc as rt
    m = 900
    S, T, _ = pencils.schur_pencil(m, 413)
    Sd, Td = rt.colmajor_to_device(S), rt.colmajor_to_device(T)
    _say(f"[walker grid] m={m} grid={grid}")
    a = rt.Solver(m, mb=64, schedule=rt.SCHEDULE_WALKER).run(Sd, Td)
    b = rt.Solver(m, mb=64, schedule=rt.SCHEDULE_WALKER, grid=grid).run(Sd, Td)
    torch.cuda.synchronize()
    assert int(a.info.item()) == 0 and int(b.info.item()) == 0
    assert torch.equal(a.Z, b.Z)


def test_walker_watchdog_bit():
    """A dependency-wait bound of one polling round (set from the host) makes waits give
    up: the launch still drains and reports the watchdog bit."""
    torch = _torch()
    from paper_2003_04776_amd import rtgevc as rt
    m = 1200
    S, T, _ = pencils.schur_pencil(m, 412)
    Sd, Td = rt.colmajor_to_device(S), rt.colmajor_to_device(T)
    r = rt.Solver(m, mb=32, schedule=rt.SCHEDULE_WALKER, watchdog=1).run(Sd, Td)
    torch.cuda.synchronize()
    assert int(r.info.item()) & rt.INFO_WATCHDOG
    r2 = rt.Solver(m, mb=32, schedule=rt.SCHEDULE_WALKER).run(Sd, Td)
    torch.cuda.synchronize()
    assert int(r2.info.item()) == 0


# ---- mixed precision (tile-update contraction on the int8 matrix cores) ----

@pytest.mark.parametrize("m,mb,band,seed", [(1, 32, 0, 500), (100, 32, 2, 501), (300, 64, 4, 502),
                                            (700, 128, 4, 503), (1000, 128, 1, 504), (1100, 64, 8, 505)])
def test_mixed_parity(m, mb, band, seed):
    """Mixed precision against the oracle (same bar as FP64) and against the FP64 path."""
    torch = _torch()
    from paper_2003_04776_amd import rtgevc as rt
    _say(f"[mixed] m={m} mb={mb} band={band} seed={seed}")
    S, T, blk = pencils.schur_pencil(m, seed)
    Sd, Td = rt.colmajor_to_device(S), rt.colmajor_to_device(T)
    rx = rt.Solver(m, mb=mb, band=band, precision=rt.PRECISION_MIXED).run(Sd, Td)
    rd = rt.Solver(m, mb=mb, band=band).run(Sd, Td)
    torch.cuda.synchronize()
    assert int(rx.info.item()) == 0
    Zx = rx.Z.cpu().numpy()
    assert np.isfinite(Zx).all()
    d = float(np.max(np.abs(Zx - rd.Z.cpu().numpy()))) if m else 0.0
    worst, errs, nill = compare(S, T, Zx)
    _say(f"   max err {worst:.3e} ill {nill}; mixed vs FP64 {d:.2e}")
    assert worst <= TOL
    ar, ai, be, _ = oracle.eigvals(S, T)
    eta = residuals(S, T, Zx, ar, ai, be)
    assert max(eta.values()) <= 64 * m * U


def test_mixed_stress_unnormalised():
    torch = _torch()
    from paper_2003_04776_amd import rtgevc as rt
    m, mb = 521, 128
    S, T, blk = pencils.schur_pencil(m, 510, "stress")
    Sd, Td = rt.colmajor_to_device(S), rt.colmajor_to_device(T)
    r = rt.Solver(m, mb=mb, normalize=False, precision=rt.PRECISION_MIXED).run(Sd, Td)
    torch.cuda.synchronize()
    Z, sc = r.Z.cpu().numpy(), r.scales.cpu().numpy()
    assert int(r.info.item()) & ~16 == 0
    assert np.isfinite(Z).all() and (sc >= 0).all() and sc.max() > 1000
    Zn, _, _ = run_gpu(S, T, mb=mb)
    rn = rt.Solver(m, mb=mb, precision=rt.PRECISION_MIXED).run(Sd, Td)
    torch.cuda.synchronize()
    worst, errs, nill = compare(S, T, rn.Z.cpu().numpy())
    _say(f"   mixed stress: max err {worst:.3e} ill {nill} max scale {sc.max()}")
    assert worst <= TOL
