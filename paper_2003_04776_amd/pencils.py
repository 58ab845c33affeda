"""Seeded synthetic real Schur pencils (S, T).

This module only draws random numbers and places them; it contains none of the
eigenvector method's arithmetic.  Both the HIP path and the CPU oracle take their
inputs from here.

The pencils have the structure of a generalized real Schur form (Section 2 of the
paper): S is quasi-upper-triangular with 1x1 and 2x2 diagonal blocks, T is upper
triangular, and each 2x2 block of (S, T) carries a complex-conjugate eigenvalue
pair (assumption 2 of Section 2).

Recipe (per pencil, seed ``seed``):

* block walk: a stream keyed by ``(seed, 0)`` gives one uniform number per visited
  position k; a 2x2 block starts at (k, k+1) when k <= m-2 and the number is below
  1/3, else k is a 1x1 block.  About half of the eigenvalues then lie in pairs.
* column j has its own stream keyed by ``(seed, j + 1)`` so that any column can be
  regenerated alone.  If j is the first column of its diagonal block, the stream
  first draws the block's diagonal values:
    - 1x1: s ~ N(0, 1), t ~ U[0.5, 2];
    - 2x2: S_b = [[a, b], [c, a]] with a ~ N(0, 1), b ~ U[0.5, 2], c = -U[0.5, 2],
      and T_b = t * I with one t ~ U[0.5, 2] (a single t keeps the pair complex).
  Then it draws S[0:b0, j] ~ N(0, 1) and T[0:b0, j] ~ N(0, 1), where b0 is the first
  row of j's diagonal block.
* ``kind="stress"``: every diagonal t is 10**U[-12, -6] and every off-diagonal entry
  of S and T is multiplied by 1e100 (the 2x2 internals a, b, c stay unscaled), so
  unscaled substitution overflows within a few rows.
* ``kind="zeroinf"``: the normal pencil with one zero eigenvalue (s = 0 in the 1x1 block
  one third of the way down the list of 1x1 blocks) and one infinite eigenvalue (t = 0
  in the block two thirds down): distinct eigenvalues, so every eigenvector is defined.
* ``kind="degenerate"``: the normal pencil where, after its regular draws, every 1x1
  block's column draws one more uniform u: u < 0.01 sets s = 0 (zero eigenvalue),
  0.01 <= u < 0.02 sets t = 0 (infinite eigenvalue) -- about 1 percent of each, as in the
  pencils of the paper's experiments (Section 6), so some eigenvalues repeat.
* ``kind="general"``: 2x2 blocks in the general form of a real Schur pencil (Section 2
  only asks for T upper triangular): T_b = [[t11, t12], [0, t22]] with t11, t22 ~ U[0.5, 2]
  drawn separately and t12 ~ N(0, 1) in about half of the blocks (u < 1/2), else 0; and
  S_b = T_b M with M = [[a, b], [c, a + e]], a ~ N(0, 1), b ~ U[0.5, 2], c = -U[0.5, 2],
  e ~ U[-0.9, 0.9].  Then det(S_b - lambda T_b) = det(T_b) det(M - lambda I), and since
  e^2 < 1 <= -4 b c the block's eigenvalues (those of M) are a complex pair.  Draw order
  of the block's column: a, b, c, e, t11, t22, u, t12.  1x1 blocks and off-diagonal entries
  as for "normal".
* ``kind="general_stress"``: "general" with t11, t22 of 10**U[-12, -6], t12 the N(0, 1)
  draw times min(t11, t22), M multiplied by f = 10**U[6, 12] (drawn last), so that the
  eigenvalues spread over the same magnitudes as those of "stress", and every
  off-diagonal entry multiplied by 1e100.

* ``kind="unbalanced"``: the "normal" pencil with T multiplied by 2^-40 (exact): the same
  eigenvectors, eigenvalues 2^40 times larger, and the entries of T far below those of S in
  every row of [S | T].

``qz_pencil`` gives a third source of inputs: the real generalized Schur form
(S, T) = (Q^T A Zq, Q^T B Zq) that LAPACK's QZ algorithm (through SciPy) computes for a
seeded dense pencil (A, B) with N(0, 1) entries -- the pencils the method receives in
practice (Section 1), with 2x2 blocks whose T part has t11 != t22.
"""
from __future__ import annotations

import numpy as np

KINDS = ("normal", "stress", "zeroinf", "degenerate", "general", "general_stress", "unbalanced")


def _stream(seed: int, j: int) -> np.random.Generator:
    return np.random.Generator(np.random.Philox(key=(int(seed) << 64) | (j & 0xFFFFFFFFFFFFFFFF)))


def block_starts(m: int, seed: int) -> np.ndarray:
    """Return int8 array ``kind[k]``: 0 = 1x1 block, 1 = first row of a 2x2 block,
    2 = second row of a 2x2 block."""
    u = _stream(seed, 0).random(max(m, 1))
    kind = np.zeros(m, dtype=np.int8)
    k = 0
    while k < m:
        if k <= m - 2 and u[k] < 1.0 / 3.0:
            kind[k] = 1
            kind[k + 1] = 2
            k += 2
        else:
            k += 1
    return kind


def _tdiag(rng: np.random.Generator, kind: str) -> float:
    if kind in ("stress", "general_stress"):
        return float(10.0 ** rng.uniform(-12.0, -6.0))
    return float(rng.uniform(0.5, 2.0))


def fill_columns(S: np.ndarray, T: np.ndarray, kind_arr: np.ndarray, seed: int,
                 j0: int, j1: int, kind: str = "normal") -> None:
    """Write columns [j0, j1) of S and T (arrays indexed [row, col], any strides)."""
    m = kind_arr.shape[0]
    offscale = 1e100 if kind in ("stress", "general_stress") else 1.0
    general = kind in ("general", "general_stress")
    zero_at = inf_at = -1
    if kind == "zeroinf":
        ones = np.flatnonzero(kind_arr == 0)
        if len(ones) >= 2:
            zero_at, inf_at = int(ones[len(ones) // 3]), int(ones[(2 * len(ones)) // 3])
    for j in range(j0, j1):
        rng = _stream(seed, j + 1)
        b0 = j - 1 if kind_arr[j] == 2 else j
        if kind_arr[j] == 0:
            S[j, j] = rng.standard_normal()
            T[j, j] = _tdiag(rng, kind)
        elif kind_arr[j] == 1 and general:
            a = rng.standard_normal()
            b = rng.uniform(0.5, 2.0)
            c = -rng.uniform(0.5, 2.0)
            e = rng.uniform(-0.9, 0.9)
            t11 = _tdiag(rng, kind)
            t22 = _tdiag(rng, kind)
            t12 = rng.standard_normal() if rng.random() < 0.5 else 0.0
            if kind == "general_stress":
                t12 *= min(t11, t22)
                f = float(10.0 ** rng.uniform(6.0, 12.0))
                a, b, c, e = a * f, b * f, c * f, e * f
            # S_b = T_b M, M = [[a, b], [c, a + e]]
            S[j, j] = t11 * a + t12 * c
            S[j, j + 1] = t11 * b + t12 * (a + e)
            S[j + 1, j] = t22 * c
            S[j + 1, j + 1] = t22 * (a + e)
            T[j, j] = t11
            T[j, j + 1] = t12
            T[j + 1, j + 1] = t22
        elif kind_arr[j] == 1:
            a = rng.standard_normal()
            b = rng.uniform(0.5, 2.0)
            c = -rng.uniform(0.5, 2.0)
            t = _tdiag(rng, kind)
            S[j, j] = a
            S[j, j + 1] = b
            S[j + 1, j] = c
            S[j + 1, j + 1] = a
            T[j, j] = t
            T[j + 1, j + 1] = t
            T[j, j + 1] = 0.0
        if b0 > 0:
            cs, ct = S[:b0, j], T[:b0, j]
            if cs.flags.c_contiguous and ct.flags.c_contiguous:
                rng.standard_normal(out=cs)     # fills in place without holding the GIL
                rng.standard_normal(out=ct)
            else:
                cs[...] = rng.standard_normal(b0)
                ct[...] = rng.standard_normal(b0)
            if offscale != 1.0:
                cs *= offscale
                ct *= offscale
        if kind_arr[j] == 0:
            if j == zero_at:
                S[j, j] = 0.0
            elif j == inf_at:
                T[j, j] = 0.0
            elif kind == "degenerate":
                u = rng.random()
                if u < 0.01:
                    S[j, j] = 0.0
                elif u < 0.02:
                    T[j, j] = 0.0
        if kind == "unbalanced":
            T[: j + 1, j] *= 2.0 ** -40
    del m


def schur_pencil(m: int, seed: int, kind: str = "normal", ld: int | None = None,
                 threads: int = 1):
    """Return (S, T, blockkind) with S, T column-major float64 of shape (m, m).

    If ``ld`` > m the arrays are views of column-major (ld, m) buffers, so the
    leading dimension seen through ``S.strides`` is ``ld``.  ``threads`` > 1 fills
    the columns from that many threads (same values: every column has its own
    stream, and the in-place normal fills run without the interpreter lock).
    """
    if kind not in KINDS:
        raise ValueError(f"kind must be one of {KINDS}")
    ld = max(m, 1) if ld is None else int(ld)
    if ld < max(m, 1):
        raise ValueError("ld must be >= m")
    Sb = np.zeros((ld, m), dtype=np.float64, order="F")
    Tb = np.zeros((ld, m), dtype=np.float64, order="F")
    S, T = Sb[:m], Tb[:m]
    kind_arr = block_starts(m, seed)
    if threads <= 1 or m < 2048:
        fill_columns(S, T, kind_arr, seed, 0, m, kind)
    else:
        from concurrent.futures import ThreadPoolExecutor
        chunk = 256
        ranges = [(j, min(j + chunk, m)) for j in range(0, m, chunk)]
        with ThreadPoolExecutor(max_workers=int(threads)) as ex:
            list(ex.map(lambda r: fill_columns(S, T, kind_arr, seed, r[0], r[1], kind), ranges))
    return S, T, kind_arr


def qz_pencil(m: int, seed: int):
    """Real generalized Schur form of a seeded dense pencil.

    A and B have N(0, 1) entries from the stream keyed by ``(seed, 0)`` (A first, column
    by column); ``scipy.linalg.qz(A, B, output="real")`` gives A = Q S Zq^T and
    B = Q T Zq^T with Q, Zq orthogonal.  Entries below S's first sub-diagonal and below
    T's diagonal are set to exact zeros (LAPACK leaves them at zero or rounding level).
    Returns (S, T, blockkind, A, B, Q, Zq), all column-major float64."""
    import scipy.linalg
    rng = _stream(seed, 0)
    A = np.asfortranarray(rng.standard_normal((m, m)).T)
    B = np.asfortranarray(rng.standard_normal((m, m)).T)
    if m == 0:
        e = np.zeros((0, 0), order="F")
        return e, e.copy(), np.zeros(0, np.int8), A, B, e.copy(), e.copy()
    S, T, Q, Zq = scipy.linalg.qz(A, B, output="real")
    S = np.asfortranarray(np.triu(S, -1))
    T = np.asfortranarray(np.triu(T))
    kind = np.zeros(m, dtype=np.int8)
    k = 0
    while k < m:
        if k + 1 < m and S[k + 1, k] != 0.0:
            kind[k], kind[k + 1] = 1, 2
            k += 2
        else:
            if k + 1 < m:
                S[k + 1, k] = 0.0
            k += 1
    return S, T, kind, A, B, np.asfortranarray(Q), np.asfortranarray(Zq)


def batch_sizes(count: int = 512, lo: int = 64, hi: int = 2048, seed: int = 3999) -> np.ndarray:
    """Sizes m_i ~ U{lo..hi} of a batch of independent pencils."""
    rng = _stream(seed, 0)
    return rng.integers(lo, hi + 1, size=count)


COMPLEX_KINDS = ("complex", "complex_stress", "complex_realeig")


def complex_schur_pencil(m: int, seed: int, kind: str = "complex", ld: int | None = None,
                         threads: int = 1):
    """Return (S, T): complex upper-triangular pencils (a complex generalized Schur form, the
    pencils of the conclusion's complex-arithmetic extension: no 2x2 blocks), complex128,
    column-major (Fortran order), shape (m, m); with ``ld`` > m they are views of (ld, m)
    buffers.

    Recipe: column j has its own Philox stream keyed by (seed, j + 1), drawing in order
    s_jj = N(0,1) + i N(0,1); |t_jj| ~ U[0.5, 2] and its phase ~ U[0, 2 pi); then the real and
    imaginary parts of S[0:j, j] (N(0,1) each), then those of T[0:j, j].  Kinds:
    * "complex_stress": |t_jj| = 10**U[-12, -6] and every off-diagonal entry times 1e100 (the
      overflow-stress recipe of the real pencils);
    * "complex_realeig": every third column (j % 3 == 1) keeps only the real parts of s_jj and
      of t_jj = |t_jj| (phase 0), so that its eigenvalue s_jj / t_jj is exactly real (and
      distinct almost surely).
    Entries below the diagonal are zero.  ``threads`` > 1 fills the columns from that many
    threads (same values: every column has its own stream)."""
    if kind not in COMPLEX_KINDS:
        raise ValueError(f"kind must be one of {COMPLEX_KINDS}")
    ld = max(m, 1) if ld is None else int(ld)
    if ld < max(m, 1):
        raise ValueError("ld must be >= m")
    Sb = np.zeros((ld, m), dtype=np.complex128, order="F")
    Tb = np.zeros((ld, m), dtype=np.complex128, order="F")
    S, T = Sb[:m], Tb[:m]
    stress = kind == "complex_stress"
    if threads > 1 and m >= 2048:
        from concurrent.futures import ThreadPoolExecutor
        chunk = 256
        with ThreadPoolExecutor(max_workers=int(threads)) as ex:
            list(ex.map(lambda j0: _fill_complex(S, T, seed, kind, j0, min(j0 + chunk, m)), range(0, m, chunk)))
    else:
        _fill_complex(S, T, seed, kind, 0, m)
    return S, T


def _fill_complex(S, T, seed: int, kind: str, j0: int, j1: int) -> None:
    stress = kind == "complex_stress"
    for j in range(j0, j1):
        rng = _stream(seed, j + 1)
        s = complex(rng.standard_normal(), rng.standard_normal())
        mag = 10.0 ** rng.uniform(-12.0, -6.0) if stress else rng.uniform(0.5, 2.0)
        ph = rng.uniform(0.0, 2.0 * np.pi)
        t = mag * complex(np.cos(ph), np.sin(ph))
        if kind == "complex_realeig" and j % 3 == 1:
            s, t = complex(s.real, 0.0), complex(mag, 0.0)
        S[j, j] = s
        T[j, j] = t
        if j > 0:
            sr, si = rng.standard_normal(j), rng.standard_normal(j)
            tr, ti = rng.standard_normal(j), rng.standard_normal(j)
            scale = 1e100 if stress else 1.0
            S[:j, j] = (sr + 1j * si) * scale
            T[:j, j] = (tr + 1j * ti) * scale
