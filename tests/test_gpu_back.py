"""Parity of the HIP back-transformation (rtgevc_backtransform, through the C ABI) with the
oracle's X = V Z, element by element on seeded inputs, plus the eigen-equation of the
original pencil (A, B) = (Q S V^T, Q T V^T) and the edge cases.

Bar: with the same Z given to both sides the results differ only by the order of the
sums of the contraction: normalised columns within 1e-12 (m u |V| |z| is below 1e-12
for these sizes).  End to end (the GPU's own Z), within 1e-10 as the eigenvectors of the
Schur form; the residual of (A, B) within 64 m u."""
from __future__ import annotations

import sys

import numpy as np
import pytest

import oracle
from helpers import block_kinds_from_S, residuals
from paper_2003_04776_amd import pencils

pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def _torch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _orthogonal(m, seed):
    g = np.random.default_rng(seed).standard_normal((m, m))
    q, r = np.linalg.qr(g)
    return np.asfortranarray(q * np.sign(np.diag(r)))


def _dense(m, seed):
    """A dense V (the back-transformation does not need it orthogonal)."""
    return np.asfortranarray(np.random.default_rng(seed).standard_normal((m, m)) / np.sqrt(max(m, 1)))


def gpu_back(S, V, Z, scales=None, mb=0, normalize=True, inplace=False):
    torch = _torch()
    from paper_2003_04776_amd import rtgevc as rt
    m = S.shape[0]
    Sd, Vd, Zd = rt.colmajor_to_device(S), rt.colmajor_to_device(V), rt.colmajor_to_device(Z)
    sd = torch.as_tensor(np.asarray(scales, dtype=np.int32), device="cuda") if scales is not None else None
    bt = rt.BackTransformer(m, mb=mb, normalize=normalize)
    res = bt.run(Sd, Vd, Zd, sd, X=Zd if inplace else None)
    torch.cuda.synchronize()
    return res.Z.cpu().numpy(), res.scales.cpu().numpy(), int(res.info.item())


@pytest.mark.parametrize("m,mb,seed", [(1, 64, 1), (2, 64, 2), (3, 128, 3), (64, 64, 4), (65, 64, 5),
                                       (129, 128, 6), (300, 64, 7), (383, 128, 8), (521, 128, 9)])
def test_back_parity_same_z(m, mb, seed):
    S, T, _ = pencils.schur_pencil(m, seed)
    Z, sc, info = oracle.tgevc(S, T)
    kind = block_kinds_from_S(S)
    V = _orthogonal(m, seed + 7)
    _say(f"back parity m={m} mb={mb} seed={seed}")
    Xg, xsg, ig = gpu_back(S, V, Z, sc, mb=mb)
    Xo, xso = oracle.backtransform(V, Z, sc, kind)[:2]
    assert ig == 0 and not xsg.any()
    assert np.abs(Xg - Xo).max() <= 1e-12, np.abs(Xg - Xo).max()


@pytest.mark.parametrize("m,mb,seed", [(200, 64, 21), (450, 128, 22)])
def test_back_end_to_end_solves_dense_pencil(m, mb, seed):
    """GPU Z, then GPU X: within 1e-10 of the oracle's X, and beta A x - alpha B x small."""
    torch = _torch()
    from paper_2003_04776_amd import rtgevc as rt
    S, T, _ = pencils.schur_pencil(m, seed)
    kind = block_kinds_from_S(S)
    Q, V = _orthogonal(m, seed + 1), _orthogonal(m, seed + 2)
    _say(f"back end to end m={m} mb={mb}")
    r = rt.tgevc(rt.colmajor_to_device(S), rt.colmajor_to_device(T), mb=mb)
    bt = rt.BackTransformer(m, mb=mb)
    res = bt.run(rt.colmajor_to_device(S), rt.colmajor_to_device(V), r.Z, r.scales)
    torch.cuda.synchronize()
    Xg = res.Z.cpu().numpy()
    Zo, so, _ = oracle.tgevc(S, T)
    Xo, _ = oracle.backtransform(V, Zo, so, kind)
    assert np.abs(Xg - Xo).max() <= 1e-10
    A, B = Q @ S @ V.T, Q @ T @ V.T
    ar, ai, be, _ = oracle.eigvals(S, T)
    eta = residuals(A, B, Xg, ar, ai, be, kind=kind)
    assert max(eta.values()) <= 64 * m * U


@pytest.mark.parametrize("mb", [64, 128])
def test_back_unnormalised_stress_exponents(mb):
    """Overflow-stress eigenvectors with large exponents, not normalised: the represented
    vectors 2^xs X agree with the oracle's (compared per column after one common power of
    two); a huge |V| makes the library scale Z_c down, still without overflow."""
    m = 300
    S, T, _ = pencils.schur_pencil(m, 31, kind="stress")
    kind = block_kinds_from_S(S)
    Z, sc, _ = oracle.tgevc(S, T, normalize=False)
    for vscale in (1.0, 2.0 ** 900):
        V = _dense(m, 32) * vscale
        _say(f"back stress mb={mb} vscale=2^{int(np.log2(vscale))}")
        Xg, xsg, ig = gpu_back(S, V, Z, sc, mb=mb, normalize=False)
        Xo, xso = oracle.backtransform(V / vscale, Z, sc, kind, normalize=False)
        assert ig == 0 and np.isfinite(Xg).all()
        if vscale > 1.0:
            assert (xsg > sc).any()      # some columns were scaled down
        e = int(np.log2(vscale))
        for c in range(m):
            if not Xo[:, c].any():
                continue
            g = np.ldexp(Xg[:, c], int(xsg[c]) - e - int(xso[c]))   # 2^xsg Xg = 2^e 2^xso Xo
            assert np.allclose(g, Xo[:, c], rtol=0, atol=1e-12 * np.abs(Xo[:, c]).max()), c


def test_back_in_place_equals_out_of_place():
    m = 333
    S, T, _ = pencils.schur_pencil(m, 41)
    Z, sc, _ = oracle.tgevc(S, T)
    V = _dense(m, 42)
    _say("back in place")
    X1, xs1, _ = gpu_back(S, V, Z, sc, mb=64)
    X2, xs2, _ = gpu_back(S, V, Z, sc, mb=64, inplace=True)
    assert np.array_equal(X1, X2) and np.array_equal(xs1, xs2)


def test_back_unselected_and_nonfinite():
    """Zero (unselected) columns stay zero with exponent 0; a NaN in V sets info bit 1."""
    m = 150
    S, T, _ = pencils.schur_pencil(m, 51)
    sel = np.zeros(m, dtype=np.int32)
    sel[::3] = 1
    Z, sc, _ = oracle.tgevc(S, T, select=sel)
    V = _dense(m, 52)
    _say("back unselected")
    Xg, xsg, ig = gpu_back(S, V, Z, sc)
    zero = ~Z.any(axis=0)
    assert zero.any() and not Xg[:, zero].any() and not xsg.any() and ig == 0
    Xo, _ = oracle.backtransform(V, Z, sc, block_kinds_from_S(S))
    assert np.abs(Xg - Xo).max() <= 1e-12
    V[7, 11] = np.nan
    _, _, ig = gpu_back(S, V, Z, sc)
    assert ig & 1


def test_back_full_size_8192_sampled():
    """m = 8192 in the launch configuration of the tile-128 path: the oracle's
    eigenvectors of sampled columns (the rest zero) go to both sides; the GPU's X on those
    columns against the oracle's X = V z."""
    m = 8192
    S, T, _ = pencils.schur_pencil(m, 61, threads=16)
    kind = block_kinds_from_S(S)
    sel = np.zeros(m, dtype=np.int32)
    sel[list(range(0, m, 257)) + [m - 2, m - 1]] = 1
    _say("back full size 8192: oracle sample")
    Z, sc, _ = oracle.tgevc(S, T, select=sel)
    cols = np.flatnonzero(Z.any(axis=0))
    V = _dense(m, 62)
    _say(f"back full size 8192: {len(cols)} columns")
    Xg, xsg, ig = gpu_back(S, V, Z, sc, mb=128)
    Xo, _ = oracle.backtransform(V, Z, sc, kind)
    assert ig == 0 and len(cols) > 30
    assert np.abs(Xg[:, cols] - Xo[:, cols]).max() <= 1e-12
    assert not Xg[:, ~Z.any(axis=0)].any()


def test_back_graph_capture_replays():
    """The back-transformation is a fixed sequence of kernel launches (no allocation, no
    memset, no synchronisation): captured once, every replay, with eager work and
    synchronisation in between, reproduces the eager result bit for bit."""
    torch = _torch()
    from paper_2003_04776_amd import rtgevc as rt
    m = 700
    S, T, _ = pencils.schur_pencil(m, 81)
    Z, sc, _ = oracle.tgevc(S, T)
    Sd, Vd, Zd = rt.colmajor_to_device(S), rt.colmajor_to_device(_dense(m, 82)), rt.colmajor_to_device(Z)
    sd = torch.as_tensor(sc, device="cuda")
    bt = rt.BackTransformer(m, mb=64)
    X = rt.colmajor_empty(m)
    xs = torch.empty(m, dtype=torch.int32, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    _say("back graph: eager")
    bt.run(Sd, Vd, Zd, sd, X=X, xscales=xs, info=info)
    torch.cuda.synchronize()
    ref = X.clone()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            bt.run(Sd, Vd, Zd, sd, X=X, xscales=xs, info=info, stream=s)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    for rep in range(3):
        X.fill_(float("nan"))
        xs.fill_(7)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(X, ref) and not bool(xs.any()) and int(info.item()) == 0, rep
        _say(f"   replay {rep}: identical")


def test_back_padded_leading_dimensions():
    """S, V, Z and X with leading dimensions larger than m give the same result."""
    torch = _torch()
    from paper_2003_04776_amd import rtgevc as rt
    m = 260
    S, T, _ = pencils.schur_pencil(m, 91)
    Z, sc, _ = oracle.tgevc(S, T)
    V = _dense(m, 92)
    _say("back padded leading dimensions")
    X1, xs1, _ = gpu_back(S, V, Z, sc, mb=128)
    Sd = rt.colmajor_to_device(S, ld=m + 3)
    Vd = rt.colmajor_to_device(V, ld=m + 5)
    Zd = rt.colmajor_to_device(Z, ld=m + 7)
    X = rt.colmajor_empty(m, ld=m + 9)
    res = rt.BackTransformer(m, mb=128).run(Sd, Vd, Zd, torch.as_tensor(sc, device="cuda"), X=X)
    torch.cuda.synchronize()
    assert np.array_equal(res.Z.cpu().numpy(), X1) and np.array_equal(res.scales.cpu().numpy(), xs1)


def test_back_null_scales_and_info():
    """scales = NULL means all exponents zero and info = NULL uses the workspace's own
    word: the same result as with both given (normalised Z has zero exponents)."""
    torch = _torch()
    import ctypes
    from paper_2003_04776_amd import rtgevc as rt
    m = 150
    S, T, _ = pencils.schur_pencil(m, 95)
    Z, sc, _ = oracle.tgevc(S, T)
    V = _dense(m, 96)
    _say("back null scales and info")
    X1, xs1, _ = gpu_back(S, V, Z, sc, mb=64)
    Sd, Vd, Zd = rt.colmajor_to_device(S), rt.colmajor_to_device(V), rt.colmajor_to_device(Z)
    X = rt.colmajor_empty(m)
    xs = torch.empty(m, dtype=torch.int32, device="cuda")
    bt = rt.BackTransformer(m, mb=64)
    rc = rt.load().rtgevc_backtransform(m, Sd.data_ptr(), m, Vd.data_ptr(), m, Zd.data_ptr(), m, None,
                                        X.data_ptr(), m, xs.data_ptr(), None, bt.work.data_ptr(), bt.nbytes,
                                        ctypes.byref(bt.opts), rt._stream_ptr(None))
    assert rc == 0
    torch.cuda.synchronize()
    assert np.array_equal(X.cpu().numpy(), X1) and np.array_equal(xs.cpu().numpy(), xs1)
