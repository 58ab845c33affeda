"""Pins for the oracle on the general real Schur form (Section 2: S quasi-upper-triangular,
T upper triangular): 2x2 diagonal blocks whose T part has t11 != t22 and t12 != 0, and
whose S part is a general 2x2 matrix, as a QZ reduction produces them (Section 1).  The
pins are independent of the oracle's own formulas: LAPACK's generalized eigenvalues and
eigenvectors (scipy.linalg.eig), 80-digit mpmath substitution whose block eigenvalues come
from mpmath's standard eigensolver of T_b^-1 S_b, the defining equation of the dense
pencil after back-transformation, and double vs extended precision."""
from __future__ import annotations

import mpmath
import numpy as np
import pytest
import scipy.linalg

import oracle
from helpers import residuals
from paper_2003_04776_amd import pencils
from test_oracle import _match_scipy, _mp_eigvec

U = 2.0 ** -53


def test_generator_general_structure():
    S, T, blk = pencils.schur_pencil(600, 50, "general")
    assert np.all(np.tril(T, -1) == 0) and np.all(np.tril(S, -2) == 0)
    pairs = np.flatnonzero(blk == 1)
    t11, t22, t12 = T[pairs, pairs], T[pairs + 1, pairs + 1], T[pairs, pairs + 1]
    assert np.all(t11 != t22)
    assert 0.35 < np.mean(t12 != 0) < 0.65
    assert np.all(S[pairs, pairs] != S[pairs + 1, pairs + 1])
    S2, T2, blk2 = pencils.schur_pencil(600, 50, "general", threads=4)
    assert np.array_equal(S, S2) and np.array_equal(T, T2)


def test_qz_pencil_structure():
    S, T, blk, A, B, Q, Zq = pencils.qz_pencil(80, 51)
    assert np.all(np.tril(T, -1) == 0) and np.all(np.tril(S, -2) == 0)
    assert np.abs(Q @ S @ Zq.T - A).max() < 1e-12 and np.abs(Q @ T @ Zq.T - B).max() < 1e-12
    pairs = np.flatnonzero(blk == 1)
    assert len(pairs) > 5
    assert np.all(T[pairs, pairs] != T[pairs + 1, pairs + 1])


def _lapack_eigvals(S, T):
    w = scipy.linalg.eigvals(S, T)
    return w


@pytest.mark.parametrize("src,m,seed", [("general", 60, 52), ("general", 200, 53), ("qz", 60, 54),
                                        ("qz", 150, 55), ("general_stress", 60, 56)])
def test_eigenvalues_against_lapack(src, m, seed):
    """Every block eigenvalue alpha/beta (with the -s21 t12 term and separate t11, t22
    scalings of a general block) equals one of LAPACK's generalized eigenvalues."""
    if src == "qz":
        S, T, blk = pencils.qz_pencil(m, seed)[:3]
    else:
        S, T, blk = pencils.schur_pencil(m, seed, src)
    ar, ai, be, info = oracle.eigvals(S, T)
    assert info == 0
    lam = (ar + 1j * ai) / be
    if src == "general_stress":
        # LAPACK would see the 1e100 off-diagonals; the block eigenvalues are those of the
        # diagonal blocks alone (Section 2), which LAPACK gets from the block-diagonal part
        Sd, Td = np.zeros_like(S), np.zeros_like(T)
        for p in range(m):
            q = p + 1 if blk[p] == 1 else p
            if blk[p] != 2:
                Sd[p:q + 1, p:q + 1] = S[p:q + 1, p:q + 1]
                Td[p:q + 1, p:q + 1] = T[p:q + 1, p:q + 1]
        w = _lapack_eigvals(Sd, Td)
    else:
        w = _lapack_eigvals(S, T)
    used = set()
    for c in range(m):
        d = np.abs(w - lam[c])
        for k in used:
            d[k] = np.inf
        k = int(np.argmin(d))
        used.add(k)
        assert d[k] <= 1e-12 * max(1.0, abs(lam[c])), (c, lam[c], w[k])
    pairs = np.flatnonzero(blk == 1)
    assert np.all(ai[pairs] > 0) and np.all(ai[pairs + 1] == -ai[pairs])


def test_order_two_general_blocks_high_precision():
    """A single 2x2 block with t11 != t22 and t12 != 0: eigenvalue and eigenvector against
    mpmath's eigensolver of T_b^-1 S_b (80 digits)."""
    rng = np.random.default_rng(57)
    blk = np.array([1, 2], dtype=np.int8)
    for _ in range(60):
        a, b, c, e = rng.standard_normal(), rng.uniform(0.5, 2), -rng.uniform(0.5, 2), rng.uniform(-0.9, 0.9)
        Tb = np.array([[rng.uniform(0.5, 2), rng.standard_normal()], [0.0, rng.uniform(0.5, 2)]])
        S = np.asfortranarray(Tb @ np.array([[a, b], [c, a + e]]))   # complex pair (those of M)
        T = np.asfortranarray(Tb)
        ar, ai, be, info = oracle.eigvals(S, T)
        assert info == 0
        mpmath.mp.dps = 80
        Sb = mpmath.matrix(S.tolist())
        Tb = mpmath.matrix(T.tolist())
        ev = mpmath.eig(mpmath.inverse(Tb) * Sb, left=False, right=False)
        lam = [e for e in ev if mpmath.im(e) > 0][0]
        got = complex(ar[0], ai[0]) / be[0]
        assert abs(got - complex(lam)) <= 1e-14 * abs(complex(lam))
        Z, _, _ = oracle.tgevc(S, T)
        z = _mp_eigvec(S, T, 0, blk)
        nrm = max(abs(mpmath.re(v)) + abs(mpmath.im(v)) for v in z)
        assert np.allclose(Z[:, 0], [float(mpmath.re(v) / nrm) for v in z], atol=1e-14, rtol=0)
        assert np.allclose(Z[:, 1], [float(mpmath.im(v) / nrm) for v in z], atol=1e-14, rtol=0)


@pytest.mark.parametrize("src,seed,m", [("general", 60, 12), ("general", 61, 9), ("general_stress", 62, 12),
                                        ("general_stress", 63, 10), ("qz", 64, 12), ("qz", 65, 8)])
def test_tiny_general_pencils_against_high_precision(src, seed, m):
    """80-digit substitution with unbounded exponent range, for the represented
    (unnormalised) vector 2^k w and the normalised one."""
    if src == "qz":
        S, T, blk = pencils.qz_pencil(m, seed)[:3]
    else:
        S, T, blk = pencils.schur_pencil(m, seed, src)
    Z, sc, info = oracle.tgevc(S, T)
    Zu, scu, _ = oracle.tgevc(S, T, normalize=False)
    assert info == 0 and np.isfinite(Zu).all()
    for p in range(m):
        if blk[p] == 2:
            continue
        z = _mp_eigvec(S, T, p, blk)
        nrm = max(abs(mpmath.re(v)) + abs(mpmath.im(v)) for v in z)
        n = len(z)
        x = np.array([float(mpmath.re(v) / nrm) for v in z])
        y = np.array([float(mpmath.im(v) / nrm) for v in z])
        assert np.max(np.abs(Z[:n, p] - x)) <= 1e-12, (p, Z[:n, p], x)
        if blk[p] == 1:
            assert np.max(np.abs(Z[:n, p + 1] - y)) <= 1e-12
        k = int(scu[p])
        for i in range(n):
            rep = mpmath.ldexp(mpmath.mpf(float(Zu[i, p])), k)
            assert abs(rep - mpmath.re(z[i])) <= mpmath.mpf(1e-12) * nrm
    if src == "general_stress":
        assert scu.max() > 1000


@pytest.mark.parametrize("src,m,seed", [("general", 40, 66), ("general", 64, 67), ("qz", 40, 68), ("qz", 90, 69)])
def test_eigenvectors_against_lapack(src, m, seed):
    if src == "qz":
        S, T, blk = pencils.qz_pencil(m, seed)[:3]
    else:
        S, T, blk = pencils.schur_pencil(m, seed, src)
    Z, sc, info = oracle.tgevc(S, T)
    ar, ai, be, _ = oracle.eigvals(S, T)
    w, V = scipy.linalg.eig(S, T)
    assert _match_scipy(S, T, Z, blk, ar, ai, be, w, V) < 1e-9


@pytest.mark.parametrize("src,m,seed", [("general", 256, 70), ("general", 1000, 71), ("general_stress", 400, 72),
                                        ("qz", 300, 73)])
def test_general_residual_and_extended_precision(src, m, seed):
    if src == "qz":
        S, T, blk = pencils.qz_pencil(m, seed)[:3]
    else:
        S, T, blk = pencils.schur_pencil(m, seed, src)
    Z, sc, info = oracle.tgevc(S, T)
    assert info == 0
    ar, ai, be, _ = oracle.eigvals(S, T)
    eta = residuals(S, T, Z, ar, ai, be)
    assert max(eta.values()) <= 64 * m * U
    Zl, _, _ = oracle.tgevc(S, T, precision="ld")
    d = np.abs(Z - Zl).max(axis=0)
    assert np.mean(d <= 1e-12) > 0.99


def test_qz_end_to_end_against_lapack():
    """(A, B) -> QZ -> Schur-form eigenvectors -> X = Zq z: each column of X is an
    eigenvector of the dense pencil (A, B) (LAPACK's, up to a complex factor) and meets
    the residual bound of (A, B)."""
    m = 70
    S, T, blk, A, B, Q, Zq = pencils.qz_pencil(m, 74)
    Z, sc, info = oracle.tgevc(S, T)
    ar, ai, be, _ = oracle.eigvals(S, T)
    X, xs = oracle.backtransform(Zq, Z, sc, blk)
    w, V = scipy.linalg.eig(A, B)
    assert _match_scipy(A, B, X, blk, ar, ai, be, w, V) < 1e-9
    eta = residuals(A, B, X, ar, ai, be, kind=blk)
    assert max(eta.values()) <= 64 * m * U


@pytest.mark.parametrize("m,seed", [(200, 81), (700, 82)])
def test_unbalanced_pencil_same_eigenvectors(m, seed):
    """The "unbalanced" pencil is (S, 2^-40 T) of the normal pencil (S, T): the eigenvalue
    pairs become (alpha, 2^40 beta) up to the normalisation and the eigenvectors are the same.
    With exact power-of-two scaling every step of the substitution is scaled exactly, so the
    oracle returns the same normalised vectors bit for bit."""
    S, T, _ = pencils.schur_pencil(m, seed)
    Su, Tu, _ = pencils.schur_pencil(m, seed, kind="unbalanced")
    assert np.array_equal(S, Su) and np.array_equal(Tu, T * 2.0 ** -40)
    Z, _, i0 = oracle.tgevc(S, T)
    Zu, _, i1 = oracle.tgevc(Su, Tu)
    assert i0 == i1 == 0
    assert np.array_equal(Z, Zu)
    ar, ai, be, _ = oracle.eigvals(S, T)
    aru, aiu, beu, _ = oracle.eigvals(Su, Tu)
    # lambda_u = 2^40 lambda: alpha_u / beta_u = 2^40 alpha / beta
    fin = be > 0
    np.testing.assert_allclose(aru[fin] / beu[fin], 2.0 ** 40 * ar[fin] / be[fin], rtol=1e-14)
    np.testing.assert_allclose(aiu[fin] / beu[fin], 2.0 ** 40 * ai[fin] / be[fin], rtol=1e-14)
