"""CPU oracle for robust generalized eigenvectors of a real Schur pencil.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU-baseline leg
of the benchmark may import this package; the product library never does.

The arithmetic is plain C (``oracle_impl.h``), built here with gcc into
``liboracle_tgevc.so`` and called through ctypes.  It computes each eigenvector on
its own by scalar robust back-substitution (Sections 2 and 4 of the paper), in
double precision and, as an independent conditioning check, in x86 extended
precision.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SO = os.path.join(_HERE, "liboracle_tgevc.so")
_SRC = [os.path.join(_HERE, "tgevc_oracle.c"), os.path.join(_HERE, "oracle_impl.h")]

_lib = None


def build() -> str:
    """Compile the oracle with gcc (no fast-math, no contraction)."""
    cmd = ["gcc", "-O3", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
           "-o", _SO + ".tmp", _SRC[0], "-lm"]
    subprocess.run(cmd, check=True, cwd=_HERE)
    os.replace(_SO + ".tmp", _SO)
    return _SO


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_SO):
            build()
        L = ctypes.CDLL(_SO)
        i64, i32p, dp = ctypes.c_int64, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)
        for suf in ("_d", "_ld"):
            for name in ("oracle_tgevc", "oracle_tgevc_left", "oracle_ctgevc"):
                f = getattr(L, name + suf)
                f.restype = ctypes.c_int
                f.argtypes = [i64, dp, i64, dp, i64, i32p, dp, i64, i32p, ctypes.c_int, ctypes.c_int]
            for name in ("oracle_eigvals", "oracle_ceigvals"):
                f = getattr(L, name + suf)
                f.restype = ctypes.c_int
                f.argtypes = [i64, dp, i64, dp, i64, dp, dp, dp]
            f = getattr(L, "oracle_blocks" + suf)
            f.restype = ctypes.c_int
            f.argtypes = [i64, dp, i64, ctypes.POINTER(ctypes.c_int8)]
        L.oracle_pd_d.restype = ctypes.c_int
        L.oracle_pd_d.argtypes = [ctypes.c_double, ctypes.c_double]
        L.oracle_pu_d.restype = ctypes.c_int
        L.oracle_pu_d.argtypes = [ctypes.c_double] * 3
        L.oracle_pd_ld_dbl.restype = ctypes.c_int
        L.oracle_pd_ld_dbl.argtypes = [ctypes.c_double, ctypes.c_double]
        L.oracle_pu_ld_dbl.restype = ctypes.c_int
        L.oracle_pu_ld_dbl.argtypes = [ctypes.c_double] * 3
        L.oracle_cdiv_d.restype = None
        L.oracle_cdiv_d.argtypes = [ctypes.c_double] * 4 + [dp, dp]
        L.oracle_omega_exp_d.restype = ctypes.c_int
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _ld_of(A: np.ndarray) -> int:
    if A.dtype != np.float64 or A.ndim != 2 or A.strides[0] != 8:
        raise ValueError("expected a column-major float64 matrix")
    return A.strides[1] // 8 if A.shape[1] > 1 else max(A.shape[0], 1)


OMEGA_EXP = 1020


def pd(b: float, t: float, precision: str = "double") -> int:
    """ProtectDivision exponent q (xi = 2^-q)."""
    f = lib().oracle_pd_d if precision == "double" else lib().oracle_pd_ld_dbl
    return int(f(float(b), float(t)))


def pu(t: float, x: float, y: float, precision: str = "double") -> int:
    """ProtectUpdate exponent q (xi = 2^-q) with bound xi (t x + y) <= Omega."""
    f = lib().oracle_pu_d if precision == "double" else lib().oracle_pu_ld_dbl
    return int(f(float(t), float(x), float(y)))


def cdiv(a: float, b: float, c: float, d: float):
    e, f = ctypes.c_double(), ctypes.c_double()
    lib().oracle_cdiv_d(a, b, c, d, ctypes.byref(e), ctypes.byref(f))
    return e.value, f.value


def blocks(S: np.ndarray):
    m = S.shape[0]
    blk = np.zeros(max(m, 1), dtype=np.int8)
    info = lib().oracle_blocks_d(m, _dp(S), _ld_of(S), blk.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)))
    return blk[:m], int(info)


def eigvals(S: np.ndarray, T: np.ndarray, precision: str = "double"):
    """Normalised (alpha_re, alpha_im, beta) and info bits."""
    m = S.shape[0]
    ar, ai, be = (np.zeros(max(m, 1)) for _ in range(3))
    f = lib().oracle_eigvals_d if precision == "double" else lib().oracle_eigvals_ld
    info = f(m, _dp(S), _ld_of(S), _dp(T), _ld_of(T), _dp(ar), _dp(ai), _dp(be))
    return ar[:m], ai[:m], be[:m], int(info)


def _call_tgevc(name, S, T, select, normalize, precision, threads):
    m = S.shape[0]
    if threads is None:
        threads = os.cpu_count() or 1
    Z = np.zeros((m, m), dtype=np.float64, order="F")
    scales = np.zeros(max(m, 1), dtype=np.int32)
    sel = None
    if select is not None:
        sel = np.ascontiguousarray(np.asarray(select, dtype=np.int32))
        if sel.shape != (m,):
            raise ValueError("select must have length m")
    f = getattr(lib(), name + ("_d" if precision == "double" else "_ld"))
    i32p = ctypes.POINTER(ctypes.c_int32)
    info = f(m, _dp(S), _ld_of(S), _dp(T), _ld_of(T),
             sel.ctypes.data_as(i32p) if sel is not None else None,
             _dp(Z), max(m, 1), scales.ctypes.data_as(i32p), int(bool(normalize)), int(threads))
    return Z, scales[:m], int(info)


def tgevc(S: np.ndarray, T: np.ndarray, select=None, normalize: bool = True,
          precision: str = "double", threads: int | None = None):
    """All (or the selected) right eigenvectors.  Returns (Z, scales, info)."""
    return _call_tgevc("oracle_tgevc", S, T, select, normalize, precision, threads)


def backtransform(V: np.ndarray, Z: np.ndarray, scales, blk, normalize: bool = True):
    """Eigenvectors of the original pencil from those of its Schur form.

    With the real Schur decomposition S = U^T A V, T = U^T B V of Section 1 (U, V
    orthogonal), S z = lambda T z gives A (V z) = U S z = lambda U T z = lambda B (V z):
    the eigenvector of (A, B) is x = V z.  (Section 1 writes U z; the defining equation
    holds for V z, and the pins below check that one.)  Column c of the
    result represents 2^xs[c] X[:, c] = V (2^scales[c] Z[:, c]); a complex pair
    (blk[p] == 1) is z = Z[:, p] + i Z[:, p+1] and shares one exponent.  Each column (or
    pair) is brought to a maximum magnitude in [1/2, 1) by a power of two before the
    product, so nothing overflows.  normalize: max_i |x_i| (real) or max_i |x_i| + |y_i|
    (pair) equal to one and xs = 0, as for the eigenvectors of the Schur form.
    Returns (X, xs)."""
    m = Z.shape[0]
    X = np.zeros((m, m), dtype=np.float64, order="F")
    xs = np.zeros(m, dtype=np.int32)
    c = 0
    while c < m:
        cols = [c, c + 1] if (blk[c] == 1 and c + 1 < m) else [c]
        zmax = max(float(np.max(np.abs(Z[:, k]))) for k in cols)
        if zmax > 0.0:
            e = int(np.frexp(zmax)[1])
            for k in cols:
                X[:, k] = V @ np.ldexp(Z[:, k], -e)
            if normalize:
                t = np.abs(X[:, cols[0]]) + (np.abs(X[:, cols[1]]) if len(cols) == 2 else 0.0)
                tmax = float(np.max(t))
                if tmax > 0.0:
                    for k in cols:
                        X[:, k] = X[:, k] / tmax
            else:
                for k in cols:
                    xs[k] = int(scales[cols[0]]) + e
        c += len(cols)
    return X, xs


def tgevc_left(S: np.ndarray, T: np.ndarray, select=None, normalize: bool = True,
               precision: str = "double", threads: int | None = None):
    """Left eigenvectors u of the Schur pencil: u^H (beta S - alpha T) = 0.

    Computed directly (oracle_impl.h, oracle_tgevc_left): with w = conj(u), w^T C = 0 for
    C = beta S - alpha T is a forward substitution from the eigenvalue's own block down,
    each block row's update protected with its 1-norm (the conclusion, Section 7, names
    left eigenvectors as the same computation with the 1-norm).  Phase: u_p = 1 at the
    first row of the eigenvalue's block.  For a complex pair (p, p+1), column p holds Re u
    and column p+1 Im u of the left eigenvector for alpha_im[p] > 0.  Returns
    (Y, scales, info) like tgevc."""
    return _call_tgevc("oracle_tgevc_left", S, T, select, normalize, precision, threads)


def tgevc_left_flip(S: np.ndarray, T: np.ndarray, select=None, normalize: bool = True,
                    precision: str = "double", threads: int | None = None):
    """The left eigenvectors by a second route, for cross-checking tgevc_left: with J the
    exchange matrix, (S', T') = (J S^T J, J T^T J) is again a real Schur pencil, and
    u^H (beta S - alpha T) = 0 holds iff (beta S' - alpha T') (J conj(u)) = 0, so u is J times
    the conjugate of a right eigenvector of (S', T') (the right oracle).  Same layout."""
    m = S.shape[0]
    Sf = np.array(S.T[::-1, ::-1], order="F")   # (copies with positive strides)
    Tf = np.array(T.T[::-1, ::-1], order="F")
    sel = None if select is None else np.ascontiguousarray(np.asarray(select, dtype=np.int32)[::-1])
    Zf, scf, info = tgevc(Sf, Tf, select=sel, normalize=normalize, precision=precision, threads=threads)
    Y = np.array(Zf[::-1, ::-1], order="F")
    scales = np.ascontiguousarray(scf[::-1])
    kind, _ = blocks(S)
    for p in np.flatnonzero(kind == 1):
        re, im = Y[:, p + 1].copy(), Y[:, p].copy()
        Y[:, p], Y[:, p + 1] = re, -im
    return Y, scales, info


def _cld_of(A: np.ndarray) -> int:
    if A.dtype != np.complex128 or A.ndim != 2 or A.strides[0] != 16:
        raise ValueError("expected a column-major complex128 matrix")
    return A.strides[1] // 16 if A.shape[1] > 1 else max(A.shape[0], 1)


def _cdp(A):
    return A.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def ctgevc(S: np.ndarray, T: np.ndarray, select=None, normalize: bool = True,
           precision: str = "double", threads: int | None = None):
    """Right eigenvectors of a complex upper-triangular pencil (S, T) (oracle_ctgevc in
    oracle_impl.h: complex scalar robust back-substitution, z_k = 1 at the eigenvalue's own
    row).  Returns (Z complex128 column-major, scales, info)."""
    m = S.shape[0]
    if threads is None:
        threads = os.cpu_count() or 1
    Z = np.zeros((m, m), dtype=np.complex128, order="F")
    scales = np.zeros(max(m, 1), dtype=np.int32)
    sel = None
    if select is not None:
        sel = np.ascontiguousarray(np.asarray(select, dtype=np.int32))
        if sel.shape != (m,):
            raise ValueError("select must have length m")
    f = getattr(lib(), "oracle_ctgevc" + ("_d" if precision == "double" else "_ld"))
    i32p = ctypes.POINTER(ctypes.c_int32)
    info = f(m, _cdp(S), _cld_of(S), _cdp(T), _cld_of(T),
             sel.ctypes.data_as(i32p) if sel is not None else None,
             _cdp(Z), max(m, 1), scales.ctypes.data_as(i32p), int(bool(normalize)), int(threads))
    return Z, scales[:m], int(info)


def ceigvals(S: np.ndarray, T: np.ndarray, precision: str = "double"):
    """Normalised (alpha, beta) of the complex pencil: alpha complex, beta real >= 0."""
    m = S.shape[0]
    ar, ai, be = (np.zeros(max(m, 1)) for _ in range(3))
    f = getattr(lib(), "oracle_ceigvals" + ("_d" if precision == "double" else "_ld"))
    info = f(m, _cdp(S), _cld_of(S), _cdp(T), _cld_of(T), _dp(ar), _dp(ai), _dp(be))
    return (ar + 1j * ai)[:m], be[:m], int(info)
