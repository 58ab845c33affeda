"""Pins for the oracle of complex-arithmetic pencils (the conclusion's extension, Section 7):
complex upper-triangular (S, T), no 2x2 blocks, (beta S - alpha T) z = 0 by complex scalar
robust substitution.  Checked against LAPACK's generalized eigenvectors, an 80-digit mpmath
substitution (also on overflow-stress pencils), a closed form of order 2, the residual and
the double / extended precision agreement."""
from __future__ import annotations

import mpmath
import numpy as np
import pytest
import scipy.linalg

import oracle
from paper_2003_04776_amd import pencils

U = 2.0 ** -53


def _cos(v, z):
    return abs(np.vdot(v, z)) / (np.linalg.norm(v) * np.linalg.norm(z))


@pytest.mark.parametrize("m,seed,kind", [(1, 1, "complex"), (2, 2, "complex"), (30, 3, "complex"),
                                         (64, 4, "complex"), (150, 5, "complex_realeig")])
def test_against_lapack(m, seed, kind):
    S, T = pencils.complex_schur_pencil(m, seed, kind)
    Z, sc, info = oracle.ctgevc(S, T)
    assert info == 0 and not sc.any()
    al, be, _ = oracle.ceigvals(S, T)
    w, V = scipy.linalg.eig(S, T)
    lam = al / be
    for k in range(m):
        j = int(np.argmin(np.abs(w - lam[k])))
        assert abs(w[j] - lam[k]) <= 1e-9 * max(1.0, abs(lam[k]))
        assert _cos(V[:, j], Z[:, k]) == pytest.approx(1.0, abs=1e-10), k
    # the eigenvalues are those of the diagonal: alpha / beta = s_kk / t_kk
    np.testing.assert_allclose(lam, np.diag(S) / np.diag(T), rtol=1e-14)


def test_closed_form_order_two():
    S = np.asfortranarray(np.array([[1.0 + 2.0j, -0.5 + 0.25j], [0.0, -1.5 + 0.5j]]))
    T = np.asfortranarray(np.array([[0.75 - 0.5j, 2.0 + 1.0j], [0.0, 1.25 + 0.0j]]))
    Z, _, info = oracle.ctgevc(S, T)
    assert info == 0
    assert Z[1, 0] == 0 and abs(Z[0, 0]) > 0
    lam = S[1, 1] / T[1, 1]
    z = np.array([-(S[0, 1] - lam * T[0, 1]) / (S[0, 0] - lam * T[0, 0]), 1.0])
    z /= max(abs(v.real) + abs(v.imag) for v in z)
    assert np.allclose(Z[:, 1], z, rtol=0, atol=8 * U)


def _mp_vec(S, T, k, dps=80):
    """80-digit reference with unbounded exponents and no scaling: M = t_kk S - s_kk T (a
    multiple of S - lambda T that stays defined for t_kk = 0), z_k = 1, back-substitution."""
    mpmath.mp.dps = dps
    n = k + 1
    Sm = [[mpmath.mpc(complex(S[i, j])) if i <= j else 0 for j in range(n)] for i in range(n)]
    Tm = [[mpmath.mpc(complex(T[i, j])) if i <= j else 0 for j in range(n)] for i in range(n)]
    M = [[Tm[k][k] * Sm[i][j] - Sm[k][k] * Tm[i][j] for j in range(n)] for i in range(n)]
    z = [mpmath.mpc(0)] * n
    z[k] = mpmath.mpc(1)
    for i in range(k - 1, -1, -1):
        z[i] = -mpmath.fsum(M[i][j] * z[j] for j in range(i + 1, n)) / M[i][i]
    return z


@pytest.mark.parametrize("kind,seed,m", [("complex", 11, 10), ("complex_stress", 12, 10), ("complex_stress", 13, 7),
                                         ("complex_realeig", 14, 9)])
def test_tiny_against_high_precision(kind, seed, m):
    S, T = pencils.complex_schur_pencil(m, seed, kind)
    Z, _, info = oracle.ctgevc(S, T)
    Zu, su, _ = oracle.ctgevc(S, T, normalize=False)
    assert info == 0 and np.isfinite(Zu).all()
    for k in range(m):
        z = _mp_vec(S, T, k)
        nrm = max(abs(mpmath.re(v)) + abs(mpmath.im(v)) for v in z)
        ref = np.array([complex(v / nrm) for v in z])
        assert np.max(np.abs(Z[:k + 1, k] - ref)) <= 1e-13, k
        for i in range(k + 1):   # represented (unnormalised) vector 2^s Z equals the tip-normalised one
            rep = mpmath.ldexp(mpmath.mpf(float(Zu[i, k].real)), int(su[k]))
            assert abs(rep - mpmath.re(z[i])) <= mpmath.mpf(1e-13) * nrm


@pytest.mark.parametrize("m,seed,kind", [(300, 21, "complex"), (300, 22, "complex_stress"), (200, 23, "complex_realeig")])
def test_residual_and_extended_precision(m, seed, kind):
    S, T = pencils.complex_schur_pencil(m, seed, kind)
    Z, _, info = oracle.ctgevc(S, T)
    assert info == 0 and np.isfinite(Z).all()
    al, be, _ = oracle.ceigvals(S, T)
    R = S @ Z * be - T @ Z * al
    nS, nT = np.abs(S).sum(axis=0).max(), np.abs(T).sum(axis=0).max()
    eta = np.abs(R).sum(axis=0) / ((nS + nT) * np.abs(Z).sum(axis=0))
    assert eta.max() <= 64 * m * U
    Zl, _, _ = oracle.ctgevc(S, T, precision="ld")
    assert np.abs(Z - Zl).max() <= 1e-11


def test_selection():
    m = 60
    S, T = pencils.complex_schur_pencil(m, 31)
    sel = np.zeros(m, dtype=np.int32)
    sel[::5] = 1
    Zs, _, _ = oracle.ctgevc(S, T, select=sel)
    Z, _, _ = oracle.ctgevc(S, T)
    for k in range(m):
        if sel[k]:
            assert np.array_equal(Zs[:, k], Z[:, k])
        else:
            assert not Zs[:, k].any()
