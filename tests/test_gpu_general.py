"""GPU parity on the general real Schur form (Section 2): 2x2 diagonal blocks whose T part
has t11 != t22 (with t12 = 0 and t12 != 0) and whose S part is a general 2x2 matrix, from
the "general" generator kinds and from LAPACK's QZ reduction of seeded dense pencils
(Section 1), through the C ABI: FP64, mixed precision, the persistent walker, left
eigenvectors, batches, full size on sampled columns, and the whole chain
(A, B) -> QZ -> rtgevc -> rtgevc_backtransform against LAPACK's eigenvectors of (A, B).

Bar: normalised eigenvectors within 1e-10 of the double-precision oracle on every
well-conditioned column (double and extended-precision oracle agree to 1e-12), and the
normwise residual within 64 m 2^-53 on every column."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from helpers import left_residuals, residuals, residuals_torch
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


def _pencil(src, m, seed):
    if src == "qz":
        return pencils.qz_pencil(m, seed)[:3]
    return pencils.schur_pencil(m, seed, src)


def _worst(Zg, Zo, Zl):
    worst, nill = 0.0, 0
    for c in range(Zg.shape[1]):
        if np.max(np.abs(Zo[:, c] - Zl[:, c]), initial=0.0) <= WELL:
            worst = max(worst, float(np.max(np.abs(Zg[:, c] - Zo[:, c]), initial=0.0)))
        else:
            nill += 1
    return worst, nill


@pytest.mark.parametrize("src,m,mb,seed,precision", [
    ("general", 300, 64, 80, 0), ("general", 1000, 128, 81, 0), ("general", 1000, 64, 82, 1),
    ("general_stress", 300, 64, 83, 0), ("general_stress", 521, 128, 84, 1),
    ("qz", 300, 64, 85, 0), ("qz", 1000, 128, 86, 0), ("qz", 300, 32, 87, 1), ("qz", 1000, 64, 88, 1)])
def test_general_parity(src, m, mb, seed, precision):
    torch = _torch()
    from paper_2003_04776_amd import rtgevc as rt
    _say(f"[general] src={src} m={m} mb={mb} seed={seed} precision={precision}")
    S, T, blk = _pencil(src, m, seed)
    Sd, Td = rt.colmajor_to_device(S), rt.colmajor_to_device(T)
    r = rt.Solver(m, mb=mb, precision=precision).run(Sd, Td)
    torch.cuda.synchronize()
    Zg, info = r.Z.cpu().numpy(), int(r.info.item())
    Zo, _, io = oracle.tgevc(S, T)
    Zl, _, _ = oracle.tgevc(S, T, precision="ld")
    assert info & ~16 == io & ~16, (info, io)
    assert np.isfinite(Zg).all()
    worst, nill = _worst(Zg, Zo, Zl)
    _say(f"   max err {worst:.3e} (ill {nill})")
    assert worst <= TOL
    ar, ai, be, _ = oracle.eigvals(S, T)
    eta = residuals(S, T, Zg, ar, ai, be)
    assert max(eta.values()) <= 64 * m * U
    if src == "general_stress":
        ru = rt.Solver(m, mb=mb, precision=precision, normalize=False).run(Sd, Td)
        torch.cuda.synchronize()
        sc = ru.scales.cpu().numpy()
        assert np.isfinite(ru.Z.cpu().numpy()).all() and (sc >= 0).all() and sc.max() > 1000


def test_general_eigenvalues_entry_point():
    """rtgevc_eigvals on general blocks (the -s21 t12 term, separate t11, t22 scalings)."""
    torch = _torch()
    from paper_2003_04776_amd import rtgevc as rt
    for src, m, seed in (("general", 500, 89), ("qz", 200, 90)):
        S, T, blk = _pencil(src, m, seed)
        ar, ai, be, info = rt.Solver(m).eigvals(rt.colmajor_to_device(S), rt.colmajor_to_device(T))
        torch.cuda.synchronize()
        oa, oi, ob, _ = oracle.eigvals(S, T)
        assert int(info.item()) == 0
        for x, y in ((ar, oa), (ai, oi), (be, ob)):
            assert np.allclose(x.cpu().numpy(), y, rtol=1e-14, atol=1e-15)


@pytest.mark.parametrize("src,m,mb,seed", [("general", 700, 64, 91), ("qz", 300, 128, 92)])
def test_general_walker(src, m, mb, seed):
    """The persistent walker: against the oracle and bit for bit against one row per band."""
    torch = _torch()
    from paper_2003_04776_amd import rtgevc as rt
    _say(f"[general walker] src={src} m={m} mb={mb}")
    S, T, blk = _pencil(src, m, seed)
    Sd, Td = rt.colmajor_to_device(S), rt.colmajor_to_device(T)
    rw = rt.Solver(m, mb=mb, schedule=rt.SCHEDULE_WALKER).run(Sd, Td)
    rb = rt.Solver(m, mb=mb, band=1, schedule=1).run(Sd, Td)
    torch.cuda.synchronize()
    Zw = rw.Z.cpu().numpy()
    assert int(rw.info.item()) == 0
    assert np.array_equal(Zw, rb.Z.cpu().numpy())
    worst, _ = _worst(Zw, oracle.tgevc(S, T)[0], oracle.tgevc(S, T, precision="ld")[0])
    assert worst <= TOL


@pytest.mark.parametrize("src,m,mb,seed,precision", [("general", 400, 64, 93, 0), ("qz", 300, 32, 94, 0),
                                                     ("general", 700, 128, 95, 1)])
def test_general_left(src, m, mb, seed, precision):
    torch = _torch()
    from paper_2003_04776_amd import rtgevc as rt
    _say(f"[general left] src={src} m={m} mb={mb} precision={precision}")
    S, T, blk = _pencil(src, m, seed)
    r = rt.tgevc_left(rt.colmajor_to_device(S), rt.colmajor_to_device(T), mb=mb, precision=precision)
    torch.cuda.synchronize()
    Yg = r.Z.cpu().numpy()
    assert int(r.info.item()) == 0
    Yo, _, _ = oracle.tgevc_left(S, T)
    Yl, _, _ = oracle.tgevc_left(S, T, precision="ld")
    worst, nill = _worst(Yg, Yo, Yl)
    _say(f"   max err {worst:.3e} (ill {nill})")
    assert worst <= TOL
    ar, ai, be, _ = oracle.eigvals(S, T)
    assert max(left_residuals(S, T, Yg, ar, ai, be).values()) <= 64 * m * U


def test_general_batched():
    """A batch mixing general, QZ and normal pencils: every pencil against the oracle."""
    torch = _torch()
    from paper_2003_04776_amd import rtgevc as rt
    specs = [("general", 97, 96), ("qz", 150, 97), ("normal", 300, 98), ("general_stress", 260, 99),
             ("qz", 64, 100), ("general", 700, 101)]
    batch = [_pencil(src, m, seed) for src, m, seed in specs]
    Z, sc, info = rt.tgevc_batched([rt.colmajor_to_device(S) for S, _, _ in batch],
                                   [rt.colmajor_to_device(T) for _, T, _ in batch])
    torch.cuda.synchronize()
    info = info.cpu().numpy()
    for i, (S, T, blk) in enumerate(batch):
        Zg = Z[i].cpu().numpy()
        Zo, _, io = oracle.tgevc(S, T)
        worst, nill = _worst(Zg, Zo, oracle.tgevc(S, T, precision="ld")[0])
        _say(f"   pencil {i} {specs[i]}: max err {worst:.2e} ill {nill} info {info[i]}")
        assert info[i] == io
        assert worst <= TOL


def _match_lapack(A, B, X, blk, ar, ai, be):
    """Largest distance of each eigenvector column (pair: x + i y) from the span of the
    LAPACK eigenvector of the same eigenvalue, relative to its norm."""
    import scipy.linalg
    w, V = scipy.linalg.eig(A, B)
    lam = np.where(be != 0, (ar + 1j * ai) / np.where(be != 0, be, 1), np.inf)
    used, worst = set(), 0.0
    for p in range(A.shape[0]):
        if blk[p] == 2:
            continue
        j = int(np.argmin(np.where(np.isfinite(w), np.abs(w - lam[p]), np.inf)))
        assert j not in used
        used.add(j)
        v = V[:, j]
        z = X[:, p] + (1j * X[:, p + 1] if blk[p] == 1 else 0)
        c = np.vdot(v, z) / np.vdot(v, v)
        worst = max(worst, np.linalg.norm(z - c * v) / np.linalg.norm(z))
    return worst


@pytest.mark.parametrize("m,seed", [(300, 102), (1000, 103)])
def test_qz_end_to_end(m, seed):
    """(A, B) -> QZ (LAPACK) -> rtgevc -> rtgevc_backtransform with the right Schur vectors
    Zq: the columns are LAPACK's eigenvectors of (A, B) up to a complex factor, meet the
    residual bound of (A, B), and equal the oracle's back-transformed vectors."""
    torch = _torch()
    from paper_2003_04776_amd import rtgevc as rt
    _say(f"[qz end to end] m={m} seed={seed}")
    S, T, blk, A, B, Q, Zq = pencils.qz_pencil(m, seed)
    Sd, Td, Vd = rt.colmajor_to_device(S), rt.colmajor_to_device(T), rt.colmajor_to_device(Zq)
    r = rt.tgevc(Sd, Td)
    x = rt.backtransform(Sd, Vd, r.Z, r.scales)
    torch.cuda.synchronize()
    assert int(r.info.item()) == 0 and int(x.info.item()) == 0
    X = x.Z.cpu().numpy()
    ar, ai, be, _ = oracle.eigvals(S, T)
    dist = _match_lapack(A, B, X, blk, ar, ai, be)
    eta = residuals(A, B, X, ar, ai, be, kind=blk)
    _say(f"   distance from LAPACK's eigenvectors {dist:.2e}, max eta {max(eta.values()):.2e}")
    assert dist < 1e-8
    assert max(eta.values()) <= 64 * m * U
    Zo, so, _ = oracle.tgevc(S, T)
    Xo, _ = oracle.backtransform(Zq, Zo, so, blk)
    Zl, _, _ = oracle.tgevc(S, T, precision="ld")
    well = np.max(np.abs(Zo - Zl), axis=0) <= WELL
    assert np.max(np.abs(X[:, well] - Xo[:, well])) <= TOL


@pytest.mark.parametrize("kind,seed,precision", [("general", 110, 0), ("general_stress", 111, 0),
                                                 ("general", 112, 1)])
def test_general_full_size_8192(kind, seed, precision):
    torch = _torch()
    from paper_2003_04776_amd import rtgevc as rt
    m = 8192
    _say(f"[general full] m={m} kind={kind} precision={precision}: generating")
    S, T, blk = pencils.schur_pencil(m, seed, kind, threads=16)
    Sd, Td = rt.colmajor_to_device(S), rt.colmajor_to_device(T)
    res = rt.Solver(m, precision=precision).run(Sd, Td)
    torch.cuda.synchronize()
    assert int(res.info.item()) & ~16 == 0
    Z = res.Z
    assert bool(torch.isfinite(Z).all())
    ar, ai, be, _ = oracle.eigvals(S, T)
    eta = residuals_torch(Sd, Td, Z, ar, ai, be, blk)
    _say(f"   max eta {eta.max():.3e}")
    assert eta.max() <= 64 * m * U
    cols = sorted(set(np.linspace(0, m - 1, 40).astype(int).tolist()))
    sel = np.zeros(m, dtype=np.int32)
    sel[cols] = 1
    Zo, _, _ = oracle.tgevc(S, T, select=sel)
    Zl, _, _ = oracle.tgevc(S, T, select=sel, precision="ld")
    cols = np.nonzero(sel | np.roll(sel & (blk == 1), 1) | np.roll(sel & (blk == 2), -1))[0]
    Zs = Z[:, torch.from_numpy(cols).to(Z.device)].cpu().numpy()
    worst, nill = _worst(Zs, Zo[:, cols], Zl[:, cols])
    _say(f"   sampled {len(cols)} columns: max err {worst:.3e} ill {nill}")
    assert worst <= TOL
