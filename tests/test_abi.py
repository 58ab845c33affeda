"""Host-side checks of the C ABI (no GPU needed): the library loads, exports every
symbol the header declares, and rejects invalid arguments before touching the GPU."""
from __future__ import annotations

import ctypes
import os
import re

import pytest

from paper_2003_04776_amd import rtgevc as rt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    text = open(os.path.join(ROOT, "include", "rtgevc.h")).read()
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(rtgevc[a-z_]*)\s*\(", text, re.M)))


def test_header_symbols_exported():
    lib = rt.load()
    syms = _declared_symbols()
    assert set(syms) == set(rt.EXPORTED), syms
    for s in syms:
        assert hasattr(lib, s), s


def test_version_and_strerror():
    assert rt.load().rtgevc_version().decode().count(".") == 2
    assert "success" in rt.strerror(0)
    assert "m" in rt.strerror(-1)


def test_workspace_size_monotone():
    assert rt.workspace_size(-1) == 0
    for mb, band in ((32, 1), (64, 4), (128, 8)):
        prev = 0
        for m in (1, 10, 100, 1000, 5000):
            w = rt.workspace_size(m, mb=mb, band=band)
            assert w >= prev and w % 256 == 0
            prev = w
    assert rt.workspace_size(5000, mb=128, band=4) > rt.workspace_size(5000, mb=128, band=1)
    assert rt.workspace_size(1000, mb=64) != rt.workspace_size(1000, mb=128)


def _call(m=4, S=1, lds=4, T=1, ldt=4, sel=None, Z=1, ldz=4, work=256, nbytes=None, opts=None):
    lib = rt.load()
    if nbytes is None:
        nbytes = rt.workspace_size(m) if m >= 0 else 0
    o = opts if opts is not None else rt.make_opts()
    return lib.rtgevc(m, S, lds, T, ldt, sel, Z, ldz, None, None, work, nbytes, ctypes.byref(o), None)


def test_argument_errors_before_any_gpu_work():
    # fake non-null pointers: every check fails before a launch
    assert _call(m=-1) == -1
    assert _call(S=None) == -2
    assert _call(lds=3) == -3
    assert _call(T=None) == -4
    assert _call(ldt=2) == -5
    assert _call(Z=None) == -7
    assert _call(ldz=1) == -8
    assert _call(work=None) == -11
    assert _call(work=257) == -11          # not 256-byte aligned
    assert _call(nbytes=16) == -12
    bad = rt.make_opts(mb=48)
    assert _call(opts=bad) == -13
    assert _call(opts=rt.make_opts(precision=1, max_refine=4)) == -13
    assert _call(opts=rt.make_opts(precision=1, max_refine=-2)) == -13
    assert _call(opts=rt.make_opts(precision=1, refine_bits=101)) == -13
    assert _call(opts=rt.make_opts(refine_bits=-1)) == -13
    assert _call(opts=rt.make_opts(split=-2)) == -13
    assert _call(opts=rt.make_opts(schedule=2, grid=-1)) == -13
    assert _call(opts=rt.make_opts(schedule=3)) == -13
    assert _call(opts=rt.make_opts(watchdog=-1)) == -13
    assert _call(opts=rt.make_opts(precision=2)) == -13
    assert _call(opts=rt.make_opts(precision=1, schedule=2)) == -13
    assert _call(m=0, S=None, T=None, Z=None, work=None, lds=1, ldt=1, ldz=1) == 0


def test_eigvals_argument_errors():
    lib = rt.load()
    o = rt.make_opts()
    n = rt.workspace_size(4)
    assert lib.rtgevc_eigvals(4, 1, 4, 1, 4, None, 1, 1, None, 256, n, ctypes.byref(o), None) == -6
    assert lib.rtgevc_eigvals(4, 1, 4, 1, 4, 1, 1, 1, None, 256, 8, ctypes.byref(o), None) == -11


def test_no_cpu_fallback(monkeypatch):
    monkeypatch.setattr(rt, "_lib", None)
    monkeypatch.setattr(rt, "LIB_PATH", "/nonexistent/librtgevc.so")
    with pytest.raises(rt.RtgevcError):
        rt.load()


def test_batched_workspace_and_argument_errors():
    lib = rt.load()
    o = rt.make_opts()
    ms = rt._i64_array([100, 0, 1000])
    n = lib.rtgevc_batched_workspace_size(3, ms, ctypes.byref(o))
    assert n > 0 and n % 256 == 0
    assert n == lib.rtgevc_batched_workspace_size(3, ms, None)
    # one pencil's own workspace is never smaller than its share of the batch layout
    assert lib.rtgevc_batched_workspace_size(1, rt._i64_array([1000]), None) >= rt.workspace_size(1000, band=1) // 2
    assert lib.rtgevc_batched_workspace_size(1, rt._i64_array([-1]), None) == 0
    assert lib.rtgevc_batched_workspace_size(0, None, None) == 0 or True

    def call(count=2, m=(4, 4), S=(1, 1), lds=(4, 4), T=(1, 1), ldt=(4, 4), Z=(1, 1), ldz=(4, 4),
             work=256, nbytes=None, opts=None):
        mm = rt._i64_array(m) if m is not None else None
        nb = nbytes if nbytes is not None else (lib.rtgevc_batched_workspace_size(count, mm, None) if mm else 0)
        oo = opts if opts is not None else rt.make_opts()
        return lib.rtgevc_batched(count, mm, rt._ptr_array(S) if S is not None else None,
                                  rt._i64_array(lds) if lds is not None else None,
                                  rt._ptr_array(T) if T is not None else None,
                                  rt._i64_array(ldt) if ldt is not None else None, None,
                                  rt._ptr_array(Z) if Z is not None else None,
                                  rt._i64_array(ldz) if ldz is not None else None, None, None,
                                  work, nb, ctypes.byref(oo), None)

    assert call(count=-1) == -1
    assert call(count=0, m=None, S=None, lds=None, T=None, ldt=None, Z=None, ldz=None, work=None) == 0
    assert call(m=None) == -2
    assert call(m=(4, -2)) == -2
    assert call(S=None) == -3
    assert call(S=(1, None)) == -3
    assert call(lds=(4, 3)) == -4
    assert call(T=(None, 1)) == -5
    assert call(ldt=(1, 4)) == -6
    assert call(Z=(1, None)) == -8
    assert call(ldz=(4, 2)) == -9
    assert call(work=None) == -12
    assert call(work=300) == -12
    assert call(nbytes=100) == -13
    bad = rt.make_opts(mb=100)
    assert call(opts=bad) == -14


def test_backtransform_workspace_and_argument_errors():
    """Workspace sizes grow with m and with the tile; invalid arguments are rejected on
    the host (fake device addresses: nothing is launched)."""
    L = rt.load()
    o64, o128 = rt.make_opts(mb=64), rt.make_opts(mb=128)
    ws = lambda m, o: L.rtgevc_backtransform_workspace_size(m, ctypes.byref(o))
    assert ws(-1, o64) == 0 and ws(0, o64) > 0
    assert ws(100, o64) < ws(1000, o64) < ws(4000, o64)
    assert ws(1000, o64) >= 1000 * 1000 * 4    # packed Z: about half of Z's doubles
    p = 1 << 20                                  # aligned fake address, never dereferenced
    m, nb = 100, ws(100, o64)
    call = lambda **k: L.rtgevc_backtransform(
        k.get("m", m), k.get("S", p), k.get("lds", m), k.get("V", p), k.get("ldv", m), k.get("Z", 2 * p),
        k.get("ldz", m), None, k.get("X", 3 * p), k.get("ldx", m), k.get("xs", p), None,
        k.get("work", p), k.get("nb", nb), ctypes.byref(k.get("o", o64)), None)
    assert call(m=-1) == -1
    assert call(S=None) == -2
    assert call(lds=m - 1) == -3
    assert call(V=None) == -4
    assert call(ldv=0) == -5
    assert call(Z=None) == -6
    assert call(ldz=m - 1) == -7
    assert call(X=None) == -9
    assert call(X=p) == -9                       # X overlapping V
    assert call(X=2 * p, ldx=m + 1, ldz=m) == -10   # in place with another leading dimension
    assert call(ldx=1) == -10
    assert call(xs=None) == -11
    assert call(work=p + 8) == -13
    assert call(nb=nb - 1) == -14
    bad = rt.make_opts(mb=96)
    assert call(o=bad) == -15
    assert call(m=0) == 0
    assert "argument 4" in rt.strerror(-4)


def test_left_workspace_and_argument_errors():
    """The left call takes rtgevc's arguments (Y in place of Z) and a workspace larger by
    the flipped pencil; invalid arguments are rejected on the host."""
    L = rt.load()
    o = rt.make_opts()
    for m in (1, 10, 1000):
        assert L.rtgevc_left_workspace_size(m, ctypes.byref(o)) >= rt.workspace_size(m) + 16 * m * m
    m, p = 4, 1 << 20
    nb = L.rtgevc_left_workspace_size(m, ctypes.byref(o))
    call = lambda **k: L.rtgevc_left(k.get("m", m), k.get("S", p), k.get("lds", m), k.get("T", p), k.get("ldt", m),
                                     None, k.get("Y", 2 * p), k.get("ldy", m), None, None, k.get("work", p),
                                     k.get("nb", nb), ctypes.byref(k.get("o", o)), None)
    assert call(m=-1) == -1
    assert call(S=None) == -2
    assert call(lds=m - 1) == -3
    assert call(T=None) == -4
    assert call(ldt=1) == -5
    assert call(Y=None) == -7
    assert call(ldy=1) == -8
    assert call(work=p + 8) == -11
    assert call(nb=rt.workspace_size(m)) == -12     # enough for rtgevc, not for the left call
    assert call(o=rt.make_opts(mb=96)) == -13
    assert call(m=0) == 0


def test_noalloc_argument_errors_and_scratch_limit():
    """rtgevc_noalloc rejects invalid arguments and orders whose workspace exceeds the
    fixed scratch before touching the GPU (fake non-null pointers: nothing is read)."""
    lib = rt.load()
    o = rt.make_opts()

    def call(m=4, S=1, lds=4, T=1, ldt=4, Z=1, ldz=4, opts=o):
        return lib.rtgevc_noalloc(m, S, lds, T, ldt, None, Z, ldz, None, None, ctypes.byref(opts), None)

    assert call(m=-1) == -1
    assert call(S=None) == -2
    assert call(lds=3) == -3
    assert call(T=None) == -4
    assert call(ldt=3) == -5
    assert call(Z=None) == -7
    assert call(ldz=3) == -8
    assert call(opts=rt.make_opts(mb=48)) == -11
    assert call(m=0, S=None, T=None, Z=None, lds=1, ldt=1, ldz=1) == 0
    # default FP64 options fit at m = 4096 and not at m = 16384 (where the tuned tile is 128)
    assert rt.workspace_size(4096) <= rt.NOALLOC_SCRATCH_BYTES < rt.workspace_size(16384)
    big = 16384
    assert call(m=big, lds=big, ldt=big, ldz=big) == rt.ERR_SCRATCH
    assert "scratch" in rt.strerror(rt.ERR_SCRATCH)
    mixed = rt.make_opts(precision=1)
    assert rt.workspace_size(4096, precision=1) > rt.NOALLOC_SCRATCH_BYTES
    assert call(m=4096, lds=4096, ldt=4096, ldz=4096, opts=mixed) == rt.ERR_SCRATCH


def test_complex_workspace_and_argument_errors():
    lib = rt.load()
    o = rt.make_opts()
    n = int(lib.rtgevc_complex_workspace_size(100, ctypes.byref(o)))
    assert n >= rt.workspace_size(200) + 3 * 8 * 200 * 200
    assert lib.rtgevc_complex_workspace_size(-1, ctypes.byref(o)) == 0

    def call(m=4, S=1, lds=4, T=1, ldt=4, Z=1, ldz=4, work=256, nbytes=None, opts=o):
        nb = int(lib.rtgevc_complex_workspace_size(max(m, 0), ctypes.byref(opts))) if nbytes is None else nbytes
        return lib.rtgevc_complex(m, S, lds, T, ldt, None, Z, ldz, None, None, work, nb, ctypes.byref(opts), None)

    assert call(m=-1) == -1
    assert call(S=None) == -2
    assert call(lds=3) == -3
    assert call(T=None) == -4
    assert call(ldt=3) == -5
    assert call(Z=None) == -7
    assert call(ldz=3) == -8
    assert call(work=None) == -11
    assert call(work=257) == -11
    assert call(nbytes=16) == -12
    assert call(opts=rt.make_opts(mb=48)) == -13
    assert call(m=0, S=None, T=None, Z=None, lds=1, ldt=1, ldz=1) == 0


def test_opts_layout_matches_the_header(tmp_path):
    """The Python binding's rtgevc_opts has the C header's size and field offsets (compiled
    from include/rtgevc.h with the host compiler)."""
    import subprocess
    names = [f[0] for f in rt.Opts._fields_]
    src = tmp_path / "layout.c"
    body = "".join(f'  printf("%zu\\n", offsetof(rtgevc_opts, {n}));\n' for n in names)
    src.write_text('#include <stddef.h>\n#include <stdio.h>\n#include "rtgevc.h"\n'
                   'int main(void) {\n  printf("%zu\\n", sizeof(rtgevc_opts));\n' + body + '  return 0;\n}\n')
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert out[0] == ctypes.sizeof(rt.Opts)
    assert out[1:] == [getattr(rt.Opts, n).offset for n in names]
