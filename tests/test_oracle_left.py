"""Pins for the oracle's left eigenvectors (u^H (beta S - alpha T) = 0): the defining
equation, SciPy's LAPACK left eigenvectors, a closed form of order 2, and the overflow-
stress invariants."""
from __future__ import annotations

import numpy as np
import pytest
import scipy.linalg

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


def test_left_matches_lapack():
    """Each left eigenvector is parallel (complex cosine 1 to 1e-9) to LAPACK's left
    eigenvector of the same eigenvalue (the right eigenvectors would not be)."""
    m = 30
    S, T, _ = pencils.schur_pencil(m, 11)
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
