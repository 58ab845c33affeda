"""Shared test helpers: residuals and normalised comparisons (no method arithmetic
beyond checking the defining equation S V D - T V B = 0)."""
from __future__ import annotations

import numpy as np


def block_kinds_from_S(S: np.ndarray) -> np.ndarray:
    m = S.shape[0]
    kind = np.zeros(m, dtype=np.int8)
    k = 0
    while k < m:
        if k + 1 < m and S[k + 1, k] != 0.0:
            kind[k], kind[k + 1] = 1, 2
            k += 2
        else:
            k += 1
    return kind


def residuals(S, T, Z, ar, ai, be, cols=None, kind=None):
    """eta_c = ||S Z_c D - T Z_c B||_1 / ((||S||_1 + ||T||_1) ||Z_c||_1) for each
    selected column c, with (alpha, beta) rescaled so max(beta, |a|+|b|) = 1
    (equation of Section 2.2, large-matrix form, column by column).  kind: the block
    structure (taken from S's sub-diagonal unless given, e.g. for a dense pencil
    equivalent to a Schur pencil)."""
    m = S.shape[0]
    if kind is None:
        kind = block_kinds_from_S(S)
    nS = np.abs(S).sum(axis=0).max() if m else 0.0
    nT = np.abs(T).sum(axis=0).max() if m else 0.0
    if cols is None:
        cols = range(m)
    out = {}
    for c in cols:
        p = c - 1 if kind[c] == 2 else c
        a, b, bt = float(ar[p]), float(ai[p]), float(be[p])
        s = max(bt, abs(a) + abs(b))
        if s > 0:
            a, b, bt = a / s, b / s, bt / s
        if kind[p] == 0:
            z = Z[:, p]
            r = bt * (S @ z) - a * (T @ z)
            zn = np.abs(z).sum()
        else:
            x, y = Z[:, p], Z[:, p + 1]
            # S [x y] beta I - T [x y] [[a, b], [-b, a]]
            Sx, Sy, Tx, Ty = S @ x, S @ y, T @ x, T @ y
            rx = bt * Sx - (a * Tx - b * Ty)
            ry = bt * Sy - (b * Tx + a * Ty)
            r = rx if c == p else ry
            zn = np.abs(Z[:, c]).sum()
        den = (nS + nT) * zn
        out[c] = float(np.abs(r).sum() / den) if den > 0 else 0.0
    return out


def normalized_columns(Z, kind, cols):
    """Each eigenvector divided by max_i(|x_i| + |y_i|) (pairs) or max_i |x_i|."""
    Zn = {}
    for c in cols:
        p = c - 1 if kind[c] == 2 else c
        if kind[p] == 1:
            n = (np.abs(Z[:, p]) + np.abs(Z[:, p + 1])).max()
        else:
            n = np.abs(Z[:, p]).max()
        Zn[c] = Z[:, c] / n if n > 0 else Z[:, c].copy()
    return Zn


def residuals_torch(S, T, Z, ar, ai, be, kind):
    """Same residual as ``residuals`` for every column at once, in FP64 on the
    device holding the tensors (S, T, Z column-major torch tensors; ar, ai, be, kind
    numpy arrays).  Returns a numpy array of eta_c."""
    import torch
    dev = Z.device
    m = Z.shape[0]
    kind = np.asarray(kind)
    p = np.where(kind == 2, np.arange(m) - 1, np.arange(m))
    a, b, bt = ar[p].astype(float), np.abs(ai[p]).astype(float), be[p].astype(float)
    s = np.maximum(bt, np.abs(a) + b)
    s[s == 0] = 1.0
    a, b, bt = a / s, b / s, bt / s
    SZ = S @ Z
    TZ = T @ Z
    A = torch.from_numpy(a).to(dev)
    Bv = torch.from_numpy(b).to(dev)
    BT = torch.from_numpy(bt).to(dev)
    # (T Z B)_c: real: a T z_c; pair (p, p+1): col p: a T x - b T y; col p+1: b T x + a T y
    TZB = TZ * A
    k1 = torch.from_numpy(np.nonzero(kind == 1)[0]).to(dev)
    if k1.numel():
        TZB[:, k1] = A[k1] * TZ[:, k1] - Bv[k1] * TZ[:, k1 + 1]
        TZB[:, k1 + 1] = Bv[k1] * TZ[:, k1] + A[k1] * TZ[:, k1 + 1]
    R = SZ * BT - TZB
    nS = S.abs().sum(dim=0).max()
    nT = T.abs().sum(dim=0).max()
    den = (nS + nT) * Z.abs().sum(dim=0)
    eta = R.abs().sum(dim=0) / torch.where(den > 0, den, torch.ones_like(den))
    return eta.cpu().numpy()


def left_residuals(S, T, Y, ar, ai, be):
    """eta_c = ||u^H (beta S - alpha T)||_1 / ((||S||_1 + ||T||_1) ||u||_1), complex pairs
    (p, p+1) as u = Y_p + i Y_{p+1} with alpha = ar_p + i ai_p, (alpha, beta) scaled so that
    max(beta, |Re alpha| + |Im alpha|) = 1."""
    m = S.shape[0]
    kind = block_kinds_from_S(S)
    nS = np.abs(S).sum(axis=0).max() if m else 0.0
    nT = np.abs(T).sum(axis=0).max() if m else 0.0
    out = {}
    c = 0
    while c < m:
        pair = kind[c] == 1
        a = complex(ar[c], ai[c] if pair else 0.0)
        b = float(be[c])
        s = max(b, abs(a.real) + abs(a.imag))
        a, b = a / s, b / s
        u = Y[:, c] + (1j * Y[:, c + 1] if pair else 0.0)
        r = np.conj(u) @ (b * S - a * T)
        den = (nS + nT) * np.abs(u).sum()
        out[c] = float(np.abs(r).sum() / den) if den > 0 else 0.0
        c += 2 if pair else 1
    return out


def backward_errors(S, T, Z, ar, ai, be, kind=None):
    """Componentwise backward error of every eigenvector column (pairs once, at their first
    column): omega_c = ||r||_1 / || beta |S| |z| + |alpha|_1 |T| |z| ||_1 with
    r = (beta S - alpha T) z (Section 2), complex magnitudes |Re| + |Im|.  A backward-stable
    substitution gives omega_c of the order of the unit roundoff whatever the scaling of the
    pencil.  Works on numpy arrays or, for large orders, torch tensors on one device (S, T,
    Z column-major; ar, ai, be, kind numpy).  Returns {c: omega_c}."""
    m = S.shape[0]
    if kind is None:
        kind = block_kinds_from_S(np.asarray(S) if not hasattr(S, "cpu") else S.cpu().numpy())
    kind = np.asarray(kind)
    torch_mode = hasattr(Z, "device") and not isinstance(Z, np.ndarray)
    if torch_mode:
        SZ, TZ = (S @ Z).cpu().numpy(), (T @ Z).cpu().numpy()
        aZ = Z.abs()
        aSZ, aTZ = (S.abs() @ aZ).cpu().numpy(), (T.abs() @ aZ).cpu().numpy()
    else:
        SZ, TZ = S @ Z, T @ Z
        aZ = np.abs(Z)
        aSZ, aTZ = np.abs(S) @ aZ, np.abs(T) @ aZ
    out = {}
    c = 0
    while c < m:
        a, bt = float(ar[c]), float(be[c])
        if kind[c] == 1:
            b = float(ai[c])
            rx = bt * SZ[:, c] - a * TZ[:, c] + b * TZ[:, c + 1]
            ry = bt * SZ[:, c + 1] - b * TZ[:, c] - a * TZ[:, c + 1]
            num = np.abs(rx).sum() + np.abs(ry).sum()
            den = (bt * (aSZ[:, c] + aSZ[:, c + 1]).sum()
                   + (abs(a) + abs(b)) * (aTZ[:, c] + aTZ[:, c + 1]).sum())
            out[c] = float(num / den) if den > 0 else 0.0
            c += 2
        else:
            r = bt * SZ[:, c] - a * TZ[:, c]
            den = bt * aSZ[:, c].sum() + abs(a) * aTZ[:, c].sum()
            out[c] = float(np.abs(r).sum() / den) if den > 0 else 0.0
            c += 1
    return out


def backward_errors_torch(S, T, Z, ar, ai, be, kind):
    """backward_errors for every eigenvalue at once on the GPU (S, T, Z column-major torch
    FP64 tensors on one device; ar, ai, be, kind numpy).  Returns a numpy array of omega."""
    import torch
    dev = Z.device
    kind = np.asarray(kind)
    first = np.nonzero(kind != 2)[0]
    pair = kind[first] == 1
    a = torch.from_numpy(np.asarray(ar, dtype=float)[first]).to(dev)
    b = torch.from_numpy(np.where(pair, np.asarray(ai, dtype=float)[first], 0.0)).to(dev)
    bt = torch.from_numpy(np.asarray(be, dtype=float)[first]).to(dev)
    fi = torch.from_numpy(first).to(dev)
    nx = torch.from_numpy(np.where(pair, first + 1, first)).to(dev)
    pm = torch.from_numpy(pair).to(dev)
    SZ, TZ = S @ Z, T @ Z
    rx = bt * SZ[:, fi] - a * TZ[:, fi] + b * TZ[:, nx]
    ry = torch.where(pm, bt * SZ[:, nx] - b * TZ[:, fi] - a * TZ[:, nx], torch.zeros_like(rx))
    num = rx.abs().sum(dim=0) + ry.abs().sum(dim=0)
    del SZ, TZ, rx, ry
    aZ = Z.abs()
    az = aZ[:, fi] + torch.where(pm, aZ[:, nx], torch.zeros_like(aZ[:, fi]))
    del aZ
    den = bt * (S.abs() @ az).sum(dim=0) + (a.abs() + b.abs()) * (T.abs() @ az).sum(dim=0)
    return (num / torch.where(den > 0, den, torch.ones_like(den))).cpu().numpy()
