"""Pins for the oracle's left eigenvectors (u^H (beta S - alpha T) = 0): the defining
equation, SciPy's LAPACK left eigenvectors, a closed form of order 2, and the overflow-
stress invariants."""
from __future__ import annotations

import numpy as np
import pytest
import scipy.linalg

import mpmath

import oracle
from helpers import block_kinds_from_S, left_residuals
from paper_2003_04776_amd import pencils

U = 2.0 ** -53


@pytest.mark.parametrize("m,seed,kind", [(1, 1, "normal"), (2, 2, "normal"), (3, 3, "normal"), (40, 4, "normal"),
                                         (97, 5, "normal"), (64, 6, "stress"), (80, 7, "zeroinf")])
def test_left_vectors_solve_the_equation(m, seed, kind):
    S, T, _ = pencils.schur_pencil(m, seed, kind=kind)
    Y, sc, info = oracle.tgevc_left(S, T)
    assert np.isfinite(Y).all() and not sc.any()
    ar, ai, be, _ = oracle.eigvals(S, T)
    eta = left_residuals(S, T, Y, ar, ai, be)
    assert max(eta.values()) <= 64 * max(m, 1) * U, max(eta.values())


@pytest.mark.parametrize("m,seed,kind", [(30, 11, "normal"), (64, 12, "normal"), (120, 13, "general"),
                                         (160, 14, "normal")])
def test_left_matches_lapack(m, seed, kind):
    """Each left eigenvector is parallel (complex cosine 1 to 1e-9) to LAPACK's left
    eigenvector of the same eigenvalue (the right eigenvectors would not be).  (LAPACK's QZ
    is normwise backward stable, so on the overflow-stress pencils, with 1e100
    off-diagonals, its eigenvalues near 1e6 carry no digits; those are pinned against the
    80-digit substitution below.)"""
    S, T, _ = pencils.schur_pencil(m, seed, kind=kind)
    kind = block_kinds_from_S(S)
    Y, _, _ = oracle.tgevc_left(S, T)
    ar, ai, be, _ = oracle.eigvals(S, T)
    w, vl = scipy.linalg.eig(S, T, left=True, right=False)
    c = 0
    while c < m:
        pair = kind[c] == 1
        u = Y[:, c] + (1j * Y[:, c + 1] if pair else 0.0)
        lam = complex(ar[c], ai[c] if pair else 0.0) / be[c]
        j = int(np.argmin(np.abs(w - lam)))
        assert abs(w[j] - lam) <= 1e-9 * max(1.0, abs(lam))
        v = vl[:, j]
        cos = abs(np.vdot(v, u)) / (np.linalg.norm(v) * np.linalg.norm(u))
        assert cos == pytest.approx(1.0, abs=1e-9), (c, cos)
        c += 2 if pair else 1


def test_left_closed_form_order_two():
    """Real upper-triangular pencil of order 2, M = beta S - alpha T: for the second
    eigenvalue (M22 = 0) u = e_2; for the first (M11 = 0) u = (1, -M12 / M22)."""
    S = np.asfortranarray([[2.0, 3.0], [0.0, -1.0]])
    T = np.asfortranarray([[1.0, 0.5], [0.0, 2.0]])
    Y, sc, info = oracle.tgevc_left(S, T)
    assert Y[0, 1] == 0.0 and Y[1, 1] == 1.0
    al, be = 2.0, 1.0                                   # first eigenvalue 2 / 1
    m12, m22 = be * 3.0 - al * 0.5, be * -1.0 - al * 2.0
    ref = np.array([1.0, -m12 / m22])
    ref /= np.abs(ref).max()
    assert np.allclose(Y[:, 0], ref, rtol=4 * U, atol=0)


def test_left_selection_and_unnormalised():
    """Selected columns only (closed under pairs), and the unnormalised representation
    2^scales Y of a stress pencil equals the normalised vectors up to one scale per column."""
    m = 70
    S, T, _ = pencils.schur_pencil(m, 21, kind="stress")
    kind = block_kinds_from_S(S)
    sel = np.zeros(m, dtype=np.int32)
    sel[::4] = 1
    Ys, _, _ = oracle.tgevc_left(S, T, select=sel)
    Yn, _, _ = oracle.tgevc_left(S, T)
    Yu, su, _ = oracle.tgevc_left(S, T, normalize=False)
    for c in range(m):
        p = c - 1 if kind[c] == 2 else c
        chosen = sel[p] or (kind[p] == 1 and sel[p + 1])
        assert Ys[:, c].any() == bool(chosen)
        if chosen:
            assert np.array_equal(Ys[:, c], Yn[:, c])
        cols = [p, p + 1] if kind[p] == 1 else [p]
        t = sum(np.abs(Yu[:, k]) for k in cols).max()
        assert np.allclose(Yu[:, c] / t, Yn[:, c], rtol=0, atol=8 * U)
    assert su.max() > 100


@pytest.mark.parametrize("m,seed,kind", [(1, 31, "normal"), (2, 32, "normal"), (90, 33, "normal"),
                                         (300, 34, "general"), (250, 35, "stress"), (200, 36, "zeroinf")])
def test_left_direct_equals_flipped_pencil(m, seed, kind):
    """The direct forward substitution and the right-eigenvector oracle on the flipped
    transposed pencil (J S^T J, J T^T J) (a second route with other rounding) agree."""
    S, T, _ = pencils.schur_pencil(m, seed, kind=kind)
    Y, _, i1 = oracle.tgevc_left(S, T)
    Yf, _, i2 = oracle.tgevc_left_flip(S, T)
    assert i1 == i2
    assert np.abs(Y - Yf).max() <= 1e-11


def test_left_closed_form_pair():
    """A single complex pair: S = [[a, b], [c, a]], T = t I; the left eigenvector of the
    eigenvalue with positive imaginary part is u = (1, conj(-(beta a - alpha t) / (beta c)))
    before normalisation, the phase fixed by u_0 = 1."""
    a_, b_, c_, t_ = 0.3, 1.5, -0.7, 1.25
    S = np.asfortranarray([[a_, b_], [c_, a_]])
    T = np.asfortranarray([[t_, 0.0], [0.0, t_]])
    Y, _, info = oracle.tgevc_left(S, T)
    assert info == 0
    lam = complex(a_, np.sqrt(-b_ * c_)) / t_
    u = np.array([1.0, np.conj(-(a_ - lam * t_) / c_)])
    u = u / max(abs(u[0].real) + abs(u[0].imag), abs(u[1].real) + abs(u[1].imag))
    got = Y[:, 0] + 1j * Y[:, 1]
    assert np.allclose(got, u, rtol=0, atol=8 * U)
    assert abs(np.conj(got) @ (S - lam * T)).max() <= 8 * U


def _mp_left(S, T, p, kind, dps=80):
    """Independent reference: w = conj(u) with w^T M = 0 for M = S - lambda T (a 1x1 block:
    t_pp S - s_pp T, a multiple that stays defined for an infinite eigenvalue), by forward
    substitution over the blocks after p in 80-digit arithmetic with unbounded exponents and
    no scaling; lambda of a pair from mpmath's eigensolver of T_b^-1 S_b (Im > 0); phase
    w_p = 1; 2x2 blocks by mpmath's LU on the transposed 2x2 system."""
    mpmath.mp.dps = dps
    m = S.shape[0]
    nb = 2 if kind[p] == 1 else 1
    Sm = mpmath.matrix([[mpmath.mpf(float(S[i, j])) for j in range(m)] for i in range(m)])
    Tm = mpmath.matrix([[mpmath.mpf(float(T[i, j])) if i <= j else 0 for j in range(m)] for i in range(m)])
    for i in range(m):
        for j in range(m):
            if i > j + 1 or (i == j + 1 and kind[j] != 1):
                Sm[i, j] = 0
    if nb == 1:
        M = Tm[p, p] * Sm - Sm[p, p] * Tm
    else:
        ev = mpmath.eig(mpmath.inverse(Tm[p:p + 2, p:p + 2]) * Sm[p:p + 2, p:p + 2], left=False, right=False)
        lam = [e for e in ev if mpmath.im(e) > 0][0]
        M = Sm - lam * Tm
    w = [mpmath.mpc(0)] * m
    w[p] = mpmath.mpc(1)
    if nb == 2:
        w[p + 1] = -M[p, p] / M[p + 1, p]
    q = p + nb
    while q < m:
        cols = [q, q + 1] if kind[q] == 1 else [q]
        rhs = [-mpmath.fsum(w[i] * M[i, c] for i in range(q)) for c in cols]
        if len(cols) == 1:
            w[q] = rhs[0] / M[q, q]
        else:
            A = mpmath.matrix([[M[r, c] for r in cols] for c in cols])   # M_qq^T
            sol = mpmath.lu_solve(A, mpmath.matrix(rhs))
            w[q], w[q + 1] = sol[0], sol[1]
        q += len(cols)
    return [mpmath.conj(v) for v in w]


@pytest.mark.parametrize("kind,seed,m", [("normal", 41, 12), ("stress", 42, 12), ("stress", 43, 9),
                                         ("general_stress", 44, 10), ("zeroinf", 45, 11)])
def test_tiny_left_against_high_precision(kind, seed, m):
    S, T, _ = pencils.schur_pencil(m, seed, kind)
    blk = block_kinds_from_S(S)
    Y, _, info = oracle.tgevc_left(S, T)
    assert info == 0
    for p in range(m):
        if blk[p] == 2:
            continue
        u = _mp_left(S, T, p, blk)
        nrm = max(abs(mpmath.re(v)) + abs(mpmath.im(v)) for v in u)
        x = np.array([float(mpmath.re(v) / nrm) for v in u])
        y = np.array([float(mpmath.im(v) / nrm) for v in u])
        assert np.max(np.abs(Y[:, p] - x)) <= 1e-13, (p, Y[:, p], x)
        if blk[p] == 1:
            assert np.max(np.abs(Y[:, p + 1] - y)) <= 1e-13
