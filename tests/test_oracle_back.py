"""Pins for the oracle's back-transformation (the eigenvectors of the original pencil
(A, B) = (Q S V^T, Q T V^T) from those of its Schur form): the defining equation of
(A, B), SciPy's LAPACK generalized eigensolver on the dense pencil, and the exact cases
V = I and V a permutation."""
from __future__ import annotations

import numpy as np
import pytest
import scipy.linalg

import oracle
from helpers import block_kinds_from_S, residuals
from paper_2003_04776_amd import pencils

U = 2.0 ** -53


def _orthogonal(m, seed):
    g = np.random.default_rng(seed).standard_normal((m, m))
    q, r = np.linalg.qr(g)
    return np.asfortranarray(q * np.sign(np.diag(r)))


def _dense_pencil(m, seed, kind="normal"):
    S, T, _ = pencils.schur_pencil(m, seed, kind=kind)
    Q, V = _orthogonal(m, seed + 1000), _orthogonal(m, seed + 2000)
    return S, T, Q, V, Q @ S @ V.T, Q @ T @ V.T


@pytest.mark.parametrize("m,seed", [(1, 1), (2, 2), (37, 3), (64, 4), (97, 5)])
def test_back_vectors_solve_the_dense_pencil(m, seed):
    """beta A x - alpha B x = 0 for every x = V z (complex pairs in real form), to
    64 m u relative to (||A|| + ||B||) ||x||."""
    S, T, Q, V, A, B = _dense_pencil(m, seed)
    Z, sc, info = oracle.tgevc(S, T)
    kind = block_kinds_from_S(S)
    ar, ai, be, _ = oracle.eigvals(S, T)
    X, xs = oracle.backtransform(V, Z, sc, kind)
    assert not xs.any()
    eta = residuals(A, B, X, ar, ai, be, kind=kind)
    assert max(eta.values()) <= 64 * m * U, max(eta.values())


def test_back_matches_lapack_eigenvectors():
    """Each back-transformed eigenvector is parallel (complex cosine 1 to 1e-6) to the
    eigenvector SciPy's LAPACK solver returns for the same eigenvalue of (A, B) (a
    transposed or missing V would give cosines near 1/sqrt(m)).  The eigenvalues of the
    dense pencil agree only to its conditioning, so each is matched to the nearest."""
    m = 30
    S, T, Q, V, A, B = _dense_pencil(m, 11)
    Z, sc, info = oracle.tgevc(S, T)
    kind = block_kinds_from_S(S)
    ar, ai, be, _ = oracle.eigvals(S, T)
    X, _ = oracle.backtransform(V, Z, sc, kind)
    w, vr = scipy.linalg.eig(A, B)
    c = 0
    while c < m:
        if kind[c] == 1:
            x, lam = X[:, c] + 1j * X[:, c + 1], (ar[c] + 1j * abs(ai[c])) / be[c]
            step = 2
        else:
            x, lam = X[:, c].astype(complex), ar[c] / be[c]
            step = 1
        j = int(np.argmin(np.abs(w - lam)))
        assert abs(w[j] - lam) <= 1e-5 * max(1.0, abs(lam))
        v = vr[:, j]
        cos = abs(np.vdot(v, x)) / (np.linalg.norm(v) * np.linalg.norm(x))
        assert cos == pytest.approx(1.0, abs=1e-6), (c, cos)
        c += step


def test_back_identity_and_permutation_are_exact():
    """V = I returns the Schur-form eigenvectors: real columns bit for bit, pairs to the
    rounding of re-normalising |x| + |y|; a permutation V returns the same vectors with
    their rows permuted, bit for bit."""
    m = 50
    S, T, _ = pencils.schur_pencil(m, 21)
    Z, sc, info = oracle.tgevc(S, T)
    kind = block_kinds_from_S(S)
    X, xs = oracle.backtransform(np.eye(m, order="F"), Z, sc, kind)
    assert not xs.any()
    real = kind == 0
    assert np.array_equal(X[:, real], Z[:, real])
    assert np.abs(X - Z).max() <= 4 * U
    perm = np.random.default_rng(3).permutation(m)
    P = np.asfortranarray(np.eye(m)[perm])
    Xp, _ = oracle.backtransform(P, Z, sc, kind)
    assert np.array_equal(Xp, X[perm])


def test_back_unnormalised_carries_the_exponents():
    """Unnormalised: 2^xs[c] X[:, c] = V (2^scales[c] Z[:, c]) on an overflow-stress
    pencil whose eigenvectors carry large exponents (compared after one common power of
    two per column, exact scaling)."""
    m = 60
    S, T, Q, V, A, B = _dense_pencil(m, 31, kind="stress")
    Z, sc, info = oracle.tgevc(S, T, normalize=False)
    kind = block_kinds_from_S(S)
    assert sc.max() > 100
    X, xs = oracle.backtransform(V, Z, sc, kind, normalize=False)
    for c in range(m):
        z = Z[:, c]
        if not z.any():
            continue
        ref = V @ np.ldexp(z, sc[c] - xs[c])
        assert np.allclose(X[:, c], ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    Xn, _ = oracle.backtransform(V, Z, sc, kind)
    eta = residuals(A, B, Xn, *oracle.eigvals(S, T)[:3], kind=kind)
    assert max(eta.values()) <= 64 * m * U
