"""Pins for the CPU oracle: each test checks the oracle against something other than
itself -- the exact defining bounds of ProtectDivision/ProtectUpdate (Section 4),
closed forms, an independent high-precision solve, SciPy's LAPACK generalized
eigensolver, special cases and invariants."""
from __future__ import annotations

import math
import random
from fractions import Fraction

import mpmath
import numpy as np
import pytest
import scipy.linalg

import oracle
from helpers import block_kinds_from_S, normalized_columns, residuals
from paper_2003_04776_amd import pencils

OMEGA = Fraction(2) ** 1020
U = 2.0 ** -53


# ------------------------------------------------------------------ scalars --

def _rand_pos(rng, lo=-1074, hi=1019):
    e = rng.randint(lo, hi)
    return math.ldexp(rng.uniform(0.5, 1.0), e) or 5e-324


def _pd_cases():
    rng = random.Random(1)
    cases = [(1.0, 1.0), (float(2 ** 1020), 0.5), (float(2 ** 1020), 5e-324),
             (5e-324, 5e-324), (1e300, 1e-300), (float(2 ** 1019), 0.5), (3.0, 2.0 ** -1020),
             (math.nextafter(float(2 ** 1020), 0), 2.0 ** -1), (1.0, math.nextafter(1.0, 0))]
    for _ in range(3000):
        cases.append((_rand_pos(rng), _rand_pos(rng)))
    return cases


def test_protect_division_bound_exact():
    """xi |b| <= |t| Omega with xi = 2^-q, checked in exact rational arithmetic;
    q is the least such exponent (property 1 of Section 4)."""
    for b, t in _pd_cases():
        q = oracle.pd(b, t)
        assert q >= 0
        lhs = Fraction(b) / Fraction(2) ** q
        assert lhs <= Fraction(t) * OMEGA, (b, t, q)
        if q > 0:
            assert Fraction(b) / Fraction(2) ** (q - 1) > Fraction(t) * OMEGA, (b, t, q)


def _pu_cases():
    rng = random.Random(2)
    om = float(2 ** 1020)
    cases = [(0.0, 0.0, 0.0), (om, om, om), (om, 1.0, 0.0), (om, 1.0, om), (1.0, 1.0, om),
             (0.0, om, om), (om, 0.0, om), (om, 5e-324, om), (2.0 ** 510, 2.0 ** 510, 0.0),
             (2.0 ** 510, 2.0 ** 510, om), (math.nextafter(om, 0), 1.0, 0.0),
             (1.5, 2.0 ** 1019, 2.0 ** 1018), (3.0, 2.0 ** 1018, math.nextafter(om, 0))]
    for _ in range(3000):
        cases.append((_rand_pos(rng), _rand_pos(rng), _rand_pos(rng)))
    for _ in range(500):
        et = rng.randint(985, 1019)
        cases.append((_rand_pos(rng, et, et), _rand_pos(rng, 1018 - et, 1022 - et), _rand_pos(rng, 1010, 1019)))
    return cases


def test_protect_update_bound_exact():
    """xi (t x + y) <= Omega exactly (property 2 of Section 4), and q is least up to
    the stated relative margin of 2^-48."""
    for t, x, y in _pu_cases():
        q = oracle.pu(t, x, y)
        assert q >= 0
        s = Fraction(t) * Fraction(x) + Fraction(y)
        assert s / Fraction(2) ** q <= OMEGA, (t, x, y, q)
        if q > 0:
            assert s / Fraction(2) ** (q - 1) > OMEGA * (1 - Fraction(1, 2 ** 48)), (t, x, y, q)


def test_protect_update_zero_third_argument():
    """Algorithm 2 calls ProtectUpdate(||X||, ||B||, 0): the bound is xi ||X|| ||B|| <= Omega."""
    for x, b in [(2.0 ** 1000, 2.0 ** 30), (2.0 ** 1019, 3.0), (1.0, 1.0)]:
        q = oracle.pu(x, b, 0.0)
        assert Fraction(x) * Fraction(b) / Fraction(2) ** q <= OMEGA


def test_complex_division_accuracy():
    """Smith/Baudin-Smith complex division against the exact rational quotient."""
    rng = random.Random(3)
    cases = [(1.0, 1.0, 1.0, 1.0), (1.0, 0.0, 0.0, 1.0), (0.0, 1.0, 1.0, 0.0),
             (2.0 ** 1000, 2.0 ** 1000, 2.0 ** -10, 2.0 ** 1000),
             (2.0 ** -1000, 2.0 ** -1020, 2.0 ** -1020, 2.0 ** -1010),
             (1e300, 1e-300, 1e300, 1e-300), (3.0, -4.0, 1e-300, 2e-300)]
    for _ in range(2000):
        e = [rng.randint(-400, 400) for _ in range(4)]
        cases.append(tuple(math.ldexp(rng.uniform(-1, 1), k) for k in e))
    for a, b, c, d in cases:
        if c == 0 and d == 0:
            continue
        e, f = oracle.cdiv(a, b, c, d)
        A, B, C, D = map(Fraction, (a, b, c, d))
        den = C * C + D * D
        er, fr = (A * C + B * D) / den, (B * C - A * D) / den
        mag = max(abs(er), abs(fr))
        if mag == 0:
            assert e == 0 and f == 0
            continue
        # normal-range results: a few ulps of the larger component
        if float(mag) > 1e-290 and float(mag) < 1e290:
            assert abs(Fraction(e) - er) <= 8 * Fraction(U) * mag, (a, b, c, d, e, f)
            assert abs(Fraction(f) - fr) <= 8 * Fraction(U) * mag, (a, b, c, d, e, f)


# ----------------------------------------------------------- closed forms --

def _pencil(S, T):
    return np.asfortranarray(np.array(S, dtype=float)), np.asfortranarray(np.array(T, dtype=float))


def test_order_one():
    S, T = _pencil([[-3.5]], [[0.25]])
    Z, sc, info = oracle.tgevc(S, T)
    assert info == 0 and Z[0, 0] == 1.0 and sc[0] == 0
    ar, ai, be, _ = oracle.eigvals(S, T)
    assert ar[0] / be[0] == -14.0 and ai[0] == 0


def test_order_one_negative_t():
    """beta >= 0 convention (Section 2): (s, t) with t < 0 becomes (-s, -t)."""
    S, T = _pencil([[2.0]], [[-0.5]])
    ar, ai, be, _ = oracle.eigvals(S, T)
    assert be[0] > 0 and ar[0] / be[0] == -4.0


def test_upper_triangular_two_closed_form():
    """z for lambda_2 = s22/t22 is (-(s12 - lambda t12)/(s11 - lambda t11), 1)."""
    rng = np.random.default_rng(5)
    for _ in range(50):
        s11, s12, s22 = rng.standard_normal(3)
        t11, t22 = rng.uniform(0.5, 2, 2)
        t12 = rng.standard_normal()
        S, T = _pencil([[s11, s12], [0, s22]], [[t11, t12], [0, t22]])
        Z, sc, info = oracle.tgevc(S, T)
        lam = Fraction(s22) / Fraction(t22)
        z0 = -(Fraction(s12) - lam * Fraction(t12)) / (Fraction(s11) - lam * Fraction(t11))
        n = max(abs(z0), Fraction(1))
        exp = [float(z0 / n), float(1 / n)]
        assert np.allclose(Z[:, 1], exp, rtol=4e-15, atol=4e-16), (Z[:, 1], exp)
        assert Z[:, 0].tolist() == [1.0, 0.0]


def test_complex_pair_closed_form():
    """S_b = [[a, b], [c, a]], T_b = t I: lambda = (a + i sqrt(-bc)) / t and
    z = (i sqrt(-bc)/c, 1) (eigenvalue of positive imaginary part)."""
    rng = np.random.default_rng(6)
    for _ in range(50):
        a = rng.standard_normal()
        b = rng.uniform(0.5, 2)
        c = -rng.uniform(0.5, 2)
        t = rng.uniform(0.5, 2)
        S, T = _pencil([[a, b], [c, a]], [[t, 0], [0, t]])
        ar, ai, be, info = oracle.eigvals(S, T)
        assert info == 0
        w = math.sqrt(-b * c)
        assert abs(ar[0] / be[0] - a / t) <= 1e-15 * (abs(a / t) + w / t)
        assert abs(ai[0] / be[0] - w / t) <= 1e-15 * (abs(a / t) + w / t)
        assert ai[1] == -ai[0]
        Z, sc, info = oracle.tgevc(S, T)
        y0 = w / c
        n = max(abs(y0), 1.0)
        # the real part of the tip cancels in exact arithmetic; rounding of alpha leaves O(u)
        assert np.allclose(Z[:, 0], [0.0, 1.0 / n], rtol=0, atol=2e-15)
        assert np.allclose(Z[:, 1], [y0 / n, 0.0], rtol=2e-15, atol=2e-15)


def test_diagonal_pencil_unit_vectors():
    rng = np.random.default_rng(7)
    m = 9
    S = np.asfortranarray(np.diag(rng.standard_normal(m)))
    T = np.asfortranarray(np.diag(rng.uniform(0.5, 2, m)))
    Z, sc, info = oracle.tgevc(S, T)
    assert info == 0
    assert np.array_equal(Z, np.eye(m))


# ------------------------------------------------------ brute force (mpmath) --

def _mp_eigvec(S, T, p, kind, dps=80):
    """Independent reference: the eigenvalue of the diagonal block from mpmath's
    standard eigensolver of T_b^-1 S_b, then row-oriented block back-substitution
    in 80-digit arithmetic with unbounded exponent range and no scaling at all
    (2x2 diagonal blocks solved by mpmath's LU on the 2x2 system).  A 1x1 block uses
    the homogeneous matrix t_pp S - s_pp T, a multiple of S - lambda T that stays
    defined for an infinite eigenvalue (t_pp = 0)."""
    mpmath.mp.dps = dps
    nb = 2 if kind[p] == 1 else 1
    n = p + nb
    Sm = mpmath.matrix([[mpmath.mpf(float(S[i, j])) for j in range(n)] for i in range(n)])
    Tm = mpmath.matrix([[mpmath.mpf(float(T[i, j])) if i <= j else 0 for j in range(n)] for i in range(n)])
    if nb == 1:
        lam = None
    else:
        Sb = Sm[p:p + 2, p:p + 2]
        Tb = Tm[p:p + 2, p:p + 2]
        ev = mpmath.eig(mpmath.inverse(Tb) * Sb, left=False, right=False)
        lam = [e for e in ev if mpmath.im(e) > 0][0]
    M = Tm[p, p] * Sm - Sm[p, p] * Tm if nb == 1 else Sm - lam * Tm
    z = [mpmath.mpc(0)] * n
    if nb == 1:
        z[p] = mpmath.mpc(1)
    else:
        z[p + 1] = mpmath.mpc(1)
        z[p] = -M[p + 1, p + 1] / M[p + 1, p]
    i = p - 1
    while i >= 0:
        i0 = i - 1 if kind[i] == 2 else i
        rows = list(range(i0, i + 1))
        rhs = [-mpmath.fsum(M[r, j] * z[j] for j in range(i + 1, n)) for r in rows]
        if len(rows) == 1:
            z[i0] = rhs[0] / M[i0, i0]
        else:
            A = mpmath.matrix([[M[r, c] for c in rows] for r in rows])
            sol = mpmath.lu_solve(A, mpmath.matrix(rhs))
            z[i0], z[i0 + 1] = sol[0], sol[1]
        i = i0 - 1
    return z


@pytest.mark.parametrize("kind,seed,m", [("normal", 11, 12), ("normal", 12, 9), ("stress", 13, 12),
                                         ("stress", 14, 10), ("normal", 15, 7), ("zeroinf", 16, 12),
                                         ("zeroinf", 17, 9)])
def test_tiny_pencils_against_high_precision(kind, seed, m):
    S, T, blk = pencils.schur_pencil(m, seed, kind)
    Z, sc, info = oracle.tgevc(S, T)
    Zu, scu, _ = oracle.tgevc(S, T, normalize=False)
    assert info == 0
    assert np.isfinite(Zu).all()
    for p in range(m):
        if blk[p] == 2:
            continue
        z = _mp_eigvec(S, T, p, blk)
        nrm = max(abs(mpmath.re(v)) + abs(mpmath.im(v)) for v in z)
        x = np.array([float(mpmath.re(v) / nrm) for v in z])
        y = np.array([float(mpmath.im(v) / nrm) for v in z])
        n = len(z)
        assert np.max(np.abs(Z[:n, p] - x)) <= 1e-13, (p, Z[:n, p], x)
        if blk[p] == 1:
            assert np.max(np.abs(Z[:n, p + 1] - y)) <= 1e-13
        # represented (unnormalised) vector 2^k w equals the exact tip-normalised vector
        k = int(scu[p])
        for i in range(n):
            rep = mpmath.ldexp(mpmath.mpf(float(Zu[i, p])), k)
            assert abs(rep - mpmath.re(z[i])) <= mpmath.mpf(1e-13) * nrm
            if blk[p] == 1:
                rep_i = mpmath.ldexp(mpmath.mpf(float(Zu[i, p + 1])), k)
                assert abs(rep_i - mpmath.im(z[i])) <= mpmath.mpf(1e-13) * nrm


def test_stress_pencil_needs_scaling():
    """The overflow-stress generator makes unscaled substitution overflow: the exact
    eigenvector exceeds the double range, so the oracle's scale exponents are large."""
    S, T, blk = pencils.schur_pencil(12, 13, "stress")
    _, scu, _ = oracle.tgevc(S, T, normalize=False)
    assert scu.max() > 1100


# -------------------------------------------------- library cross-checks --

def _match_scipy(S, T, Z, blk, ar, ai, be, w, V):
    m = S.shape[0]
    lam_o = np.where(be != 0, (ar + 1j * ai) / np.where(be != 0, be, 1), np.inf)
    used = set()
    worst = 0.0
    for p in range(m):
        if blk[p] == 2:
            continue
        lam = lam_o[p]
        if np.isinf(lam):   # an infinite eigenvalue: LAPACK's beta = 0 gives a non-finite w
            j = int(np.flatnonzero(~np.isfinite(w))[0])
        else:
            j = int(np.argmin(np.where(np.isfinite(w), np.abs(w - lam), np.inf)))
        assert j not in used
        used.add(j)
        v = V[:, j]
        z = Z[:, p] + (1j * Z[:, p + 1] if blk[p] == 1 else 0)
        c = np.vdot(v, z) / np.vdot(v, v)
        worst = max(worst, np.linalg.norm(z - c * v) / np.linalg.norm(z))
    return worst


@pytest.mark.parametrize("m,seed,kind", [(20, 21, "normal"), (40, 22, "normal"), (64, 23, "normal"),
                                         (40, 24, "zeroinf"), (64, 25, "zeroinf")])
def test_against_lapack_generalized_eig(m, seed, kind):
    """Eigenvectors parallel to those of LAPACK xGGEV (scipy.linalg.eig(S, T)), also with a
    zero and an infinite eigenvalue."""
    S, T, blk = pencils.schur_pencil(m, seed, kind)
    Z, sc, info = oracle.tgevc(S, T)
    ar, ai, be, _ = oracle.eigvals(S, T)
    w, V = scipy.linalg.eig(S, T)
    assert _match_scipy(S, T, Z, blk, ar, ai, be, w, V) < 1e-9


def test_standard_problem_T_identity():
    """T = I reduces to the standard eigenproblem: compare with scipy.linalg.eig(S)."""
    m = 30
    S, _, blk = pencils.schur_pencil(m, 31)
    T = np.asfortranarray(np.eye(m))
    Z, sc, info = oracle.tgevc(S, T)
    ar, ai, be, _ = oracle.eigvals(S, T)
    w, V = scipy.linalg.eig(S)
    assert _match_scipy(S, T, Z, blk, ar, ai, be, w, V) < 1e-9


def test_all_real_upper_triangular():
    rng = np.random.default_rng(8)
    m = 25
    S = np.asfortranarray(np.triu(rng.standard_normal((m, m))))
    T = np.asfortranarray(np.triu(rng.standard_normal((m, m))) + np.diag(rng.uniform(0.5, 2, m)))
    T[np.diag_indices(m)] = rng.uniform(0.5, 2, m)
    Z, sc, info = oracle.tgevc(S, T)
    blk = np.zeros(m, dtype=np.int8)
    ar, ai, be, _ = oracle.eigvals(S, T)
    assert np.all(ai == 0)
    w, V = scipy.linalg.eig(S, T)
    assert _match_scipy(S, T, Z, blk, ar, ai, be, w, V) < 1e-9


# --------------------------------------------------------------- invariants --

@pytest.mark.parametrize("m,seed,kind", [(256, 0, "normal"), (256, 1, "normal"), (200, 200, "stress"),
                                         (1200, 2, "normal"), (400, 18, "degenerate")])
def test_residual_bound_and_finiteness(m, seed, kind):
    """Normwise residual of S V D - T V B = 0 (Section 2.2) within 64 m u, no
    Inf/NaN, integer scales >= 0, and double vs extended precision agreement.  The
    degenerate pencil repeats zero and infinite eigenvalues, whose singular pivots are
    perturbed (info bit 16) and still meet the residual bound."""
    S, T, blk = pencils.schur_pencil(m, seed, kind)
    Z, sc, info = oracle.tgevc(S, T)
    assert info == (16 if kind == "degenerate" else 0)
    Zu, scu, _ = oracle.tgevc(S, T, normalize=False)
    assert np.isfinite(Z).all() and np.isfinite(Zu).all()
    assert (scu >= 0).all()
    assert np.abs(Zu).max() <= 2.0 ** 1020
    ar, ai, be, _ = oracle.eigvals(S, T)
    eta = residuals(S, T, Z, ar, ai, be)
    assert max(eta.values()) <= 64 * m * U
    Zl, _, _ = oracle.tgevc(S, T, precision="ld")
    assert np.abs(Z - Zl).max() <= 1e-11


def test_normalised_equals_scaled_representation():
    S, T, blk = pencils.schur_pencil(300, 41)
    Z, _, _ = oracle.tgevc(S, T)
    Zu, scu, _ = oracle.tgevc(S, T, normalize=False)
    Zn = normalized_columns(Zu, blk, range(300))
    for c in range(300):
        assert np.array_equal(Zn[c] == 0, Z[:, c] == 0) or np.abs(Zn[c] - Z[:, c]).max() < 1e-15
        assert np.abs(Zn[c] - Z[:, c]).max() <= 2e-16


def test_lemma_rank_two_for_pairs():
    """Lemma of Section 2.1: V = [x y] of a complex eigenvector has rank 2."""
    S, T, blk = pencils.schur_pencil(120, 42)
    Z, _, _ = oracle.tgevc(S, T)
    for p in np.nonzero(blk == 1)[0]:
        sv = np.linalg.svd(Z[:, [p, p + 1]], compute_uv=False)
        assert sv[1] > 1e-8 * sv[0]


def test_select_subset_and_closure():
    """A subset closed under conjugation (Section 5): either flag of a pair selects
    both columns, and the closure is reported with info bit 32."""
    S, T, blk = pencils.schur_pencil(150, 43)
    Zall, _, _ = oracle.tgevc(S, T)
    sel = np.zeros(150, dtype=np.int32)
    pairs = np.nonzero(blk == 1)[0]
    sel[pairs[0] + 1] = 1          # second column only -> closure
    reals = np.nonzero(blk == 0)[0]
    sel[reals[3]] = 1
    sel[pairs[2]] = 1
    sel[pairs[2] + 1] = 1
    Z, sc, info = oracle.tgevc(S, T, select=sel)
    assert info & 32
    on = {pairs[0], pairs[0] + 1, reals[3], pairs[2], pairs[2] + 1}
    for c in range(150):
        if c in on:
            assert np.array_equal(Z[:, c], Zall[:, c])
        else:
            assert not Z[:, c].any()


def test_structure_errors_reported():
    S, T, blk = pencils.schur_pencil(10, 44)
    S2 = S.copy(order="F")
    # two consecutive non-zero sub-diagonal entries
    k = int(np.nonzero(blk == 1)[0][0]) if (blk == 1).any() else 0
    S2[k + 2, k + 1] = 0.5 if k + 2 < 10 else 0.0
    _, info = oracle.blocks(S2)
    assert info & 2
    # a 2x2 block with real eigenvalues (assumption 2 violated)
    S3, T3 = _pencil([[1.0, 2.0], [3.0, 1.0]], [[1.0, 0.0], [0.0, 1.0]])
    _, _, _, info = oracle.eigvals(S3, T3)
    assert info & 4
    # indefinite 1x1 block (alpha = beta = 0)
    S4, T4 = _pencil([[0.0, 1.0], [0.0, 2.0]], [[0.0, 1.0], [0.0, 1.0]])
    Z, _, info = oracle.tgevc(S4, T4)
    assert info & 8
    assert Z[0, 0] == 1.0


def test_generator_structure():
    S, T, blk = pencils.schur_pencil(400, 45, ld=407)
    assert S.strides == (8, 8 * 407)
    assert np.all(np.tril(T, -1) == 0)
    assert np.all(np.tril(S, -2) == 0)
    kind = block_kinds_from_S(S)
    assert np.array_equal(kind, blk)
    frac = 2 * (blk == 1).sum() / 400
    assert 0.35 < frac < 0.65
    for p in np.nonzero(blk == 1)[0]:
        assert S[p, p] == S[p + 1, p + 1] and S[p + 1, p] < 0 < S[p, p + 1]
        assert T[p, p] == T[p + 1, p + 1] and T[p, p + 1] == 0
    # a column regenerates alone and threads do not change the result
    S2, T2, _ = pencils.schur_pencil(400, 45, threads=4)
    assert np.array_equal(S, S2) and np.array_equal(T, T2)


@pytest.mark.parametrize("m,seed,kind", [(300, 3, "normal"), (300, 203, "stress"), (300, 73, "general"),
                                         (300, 74, "general_stress"), (1500, 4, "normal")])
def test_componentwise_backward_error_at_unit_roundoff(m, seed, kind):
    """The oracle is a scalar substitution, backward stable column by column, so its
    componentwise backward error ||(beta S - alpha T) z||_1 / ||beta |S||z| + |alpha||T||z| ||_1
    stays at a few units of roundoff whatever the pencil's scaling (1e100 off-diagonals in
    the stress pencils) and order.  A dropped term, a wrong sign or a transposed operand in the
    substitution moves it to O(1).  (The refinement of the mixed-precision mode flags columns
    by this measure.)"""
    from helpers import backward_errors
    S, T, blk = pencils.schur_pencil(m, seed, kind)
    Z, _, _ = oracle.tgevc(S, T)
    ar, ai, be, _ = oracle.eigvals(S, T)
    om = np.array(list(backward_errors(S, T, Z, ar, ai, be).values()))
    assert om.max() <= 8 * U, om.max()
    # the measure does see a perturbation at the 1e-12 level (relative to each column)
    rng = np.random.default_rng(seed)
    Zp = Z * (1.0 + 1e-12 * rng.standard_normal(Z.shape))
    om_p = np.array(list(backward_errors(S, T, Zp, ar, ai, be).values()))
    assert np.median(om_p) > 1e3 * np.median(om)
