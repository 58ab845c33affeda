"""Python binding of librtgevc.so: argument marshalling only.

Every step of the computation runs in the library's HIP kernels; torch supplies
device memory and the stream.  If the library is missing, every call raises: there
is no CPU fallback.

Matrices are column-major float64 device tensors: a tensor ``A`` with
``A.stride(0) == 1`` and ``A.stride(1) == ld >= m`` (for instance ``B.t()`` of a
contiguous row-major ``B``, or ``colmajor_to_device(numpy_array)``).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librtgevc.so")

INFO_NONFINITE = 1
INFO_BAD_STRUCTURE = 2
INFO_REAL_PAIR = 4
INFO_INDEFINITE = 8
INFO_PERTURBED = 16
INFO_SELECT_CLOSED = 32
INFO_REFINE = 64
INFO_WATCHDOG = 128
INFO_PRESCALED = 256


class RtgevcError(RuntimeError):
    pass


class Opts(ctypes.Structure):
    _fields_ = [("mb", ctypes.c_int32), ("normalize", ctypes.c_int32), ("band", ctypes.c_int32),
                ("schedule", ctypes.c_int32), ("watchdog", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("max_refine", ctypes.c_int32), ("refine_bits", ctypes.c_int32), ("split", ctypes.c_int32),
                ("grid", ctypes.c_int32)]


_lib = None


def load():
    """Load the built library (raises if it is missing: no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RtgevcError(f"{LIB_PATH} is not built; run paper_2003_04776_amd.build.build()")
    L = ctypes.CDLL(LIB_PATH)
    i64, vp, sz = ctypes.c_int64, ctypes.c_void_p, ctypes.c_size_t
    op = ctypes.POINTER(Opts)
    L.rtgevc_workspace_size.restype = sz
    L.rtgevc_workspace_size.argtypes = [i64, op]
    L.rtgevc.restype = ctypes.c_int
    L.rtgevc.argtypes = [i64, vp, i64, vp, i64, vp, vp, i64, vp, vp, vp, sz, op, vp]
    L.rtgevc_complex_workspace_size.restype = sz
    L.rtgevc_complex_workspace_size.argtypes = [i64, op]
    L.rtgevc_complex.restype = ctypes.c_int
    L.rtgevc_complex.argtypes = [i64, vp, i64, vp, i64, vp, vp, i64, vp, vp, vp, sz, op, vp]
    L.rtgevc_noalloc.restype = ctypes.c_int
    L.rtgevc_noalloc.argtypes = [i64, vp, i64, vp, i64, vp, vp, i64, vp, vp, op, vp]
    L.rtgevc_eigvals.restype = ctypes.c_int
    L.rtgevc_eigvals.argtypes = [i64, vp, i64, vp, i64, vp, vp, vp, vp, vp, sz, op, vp]
    L.rtgevc_timed.restype = ctypes.c_int
    L.rtgevc_timed.argtypes = [i64, vp, i64, vp, i64, vp, vp, i64, vp, vp, vp, sz, op, vp,
                               ctypes.POINTER(ctypes.c_double), ctypes.c_int]
    L.rtgevc_batched_workspace_size.restype = sz
    L.rtgevc_batched_workspace_size.argtypes = [ctypes.c_int32, vp, op]
    L.rtgevc_batched.restype = ctypes.c_int
    L.rtgevc_batched.argtypes = [ctypes.c_int32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, op, vp]
    L.rtgevc_left_workspace_size.restype = sz
    L.rtgevc_left_workspace_size.argtypes = [i64, op]
    L.rtgevc_left.restype = ctypes.c_int
    L.rtgevc_left.argtypes = [i64, vp, i64, vp, i64, vp, vp, i64, vp, vp, vp, sz, op, vp]
    L.rtgevc_backtransform_workspace_size.restype = sz
    L.rtgevc_backtransform_workspace_size.argtypes = [i64, op]
    L.rtgevc_backtransform.restype = ctypes.c_int
    L.rtgevc_backtransform.argtypes = [i64, vp, i64, vp, i64, vp, i64, vp, vp, i64, vp, vp, vp, sz, op, vp]
    L.rtgevc_resolve_opts.restype = ctypes.c_int
    L.rtgevc_resolve_opts.argtypes = [i64, ctypes.c_int32, op, op]
    L.rtgevc_strerror.restype = ctypes.c_char_p
    L.rtgevc_strerror.argtypes = [ctypes.c_int]
    L.rtgevc_version.restype = ctypes.c_char_p
    L.rtgevc_version.argtypes = []
    _lib = L
    return L


EXPORTED = ("rtgevc_workspace_size", "rtgevc", "rtgevc_eigvals", "rtgevc_timed",
            "rtgevc_batched_workspace_size", "rtgevc_batched", "rtgevc_left_workspace_size", "rtgevc_left",
            "rtgevc_backtransform_workspace_size",
            "rtgevc_backtransform", "rtgevc_resolve_opts", "rtgevc_strerror", "rtgevc_version",
            "rtgevc_noalloc", "rtgevc_complex_workspace_size", "rtgevc_complex")
NOALLOC_SCRATCH_BYTES = 64 << 20   # RTGEVC_NOALLOC_SCRATCH_BYTES
ERR_SCRATCH = -2000                # RTGEVC_ERR_SCRATCH
TIMED_NSTATS = 17


SCHEDULE_BANDS = 1     # band wavefront with look-ahead (default)
SCHEDULE_WALKER = 2    # persistent walker with device-side dependency counters


PRECISION_FP64 = 0
PRECISION_MIXED = 1    # tile-update contraction on the int8 matrix cores from split operands


def make_opts(mb: int = 0, normalize: bool = True, band: int = 0, schedule: int = 0, watchdog: int = 0,
              precision: int = 0, max_refine: int = 0, refine_bits: int = 0, split: int = 0, grid: int = 0) -> Opts:
    o = Opts()
    o.grid = int(grid)
    o.split = int(split)
    o.max_refine = int(max_refine)
    o.refine_bits = int(refine_bits)
    o.precision = int(precision)
    o.mb = int(mb)
    o.normalize = 1 if normalize else 0
    o.band = int(band)
    o.schedule = int(schedule)
    o.watchdog = int(watchdog)
    return o


def workspace_size(m: int, mb: int = 0, normalize: bool = True, band: int = 0, schedule: int = 0,
                   precision: int = 0, max_refine: int = 0, refine_bits: int = 0) -> int:
    o = make_opts(mb, normalize, band, schedule, 0, precision, max_refine, refine_bits)
    return int(load().rtgevc_workspace_size(int(m), ctypes.byref(o)))


def resolve_opts(m: int, batched: bool = False, mb: int = 0, band: int = 0, normalize: bool = True,
                 schedule: int = 0, precision: int = 0, with_schedule: bool = False, split: int = 0,
                 with_split: bool = False):
    """(mb, band) — and the schedule with with_schedule, then the tiles per launch of a
    band's update of the rows above it (-1: one launch) with with_split — the library would
    use for order m with these options."""
    o, out = make_opts(mb, normalize, band, schedule, 0, precision, split=split), Opts()
    _check(load().rtgevc_resolve_opts(int(m), 1 if batched else 0, ctypes.byref(o), ctypes.byref(out)),
           "rtgevc_resolve_opts")
    res = (int(out.mb), int(out.band)) + ((int(out.schedule),) if with_schedule else ())
    return res + ((int(out.split),) if with_split else ())


def strerror(code: int) -> str:
    return load().rtgevc_strerror(int(code)).decode()


def _check(rc: int, what: str):
    if rc != 0:
        raise RtgevcError(f"{what} failed ({rc}): {strerror(rc)}")


def _ld(A, m: int) -> int:
    import torch
    if A.dtype != torch.float64 or A.dim() != 2 or A.device.type != "cuda":
        raise ValueError("expected a float64 CUDA matrix")
    if tuple(A.shape) != (m, m):
        raise ValueError(f"expected shape ({m}, {m}), got {tuple(A.shape)}")
    if m > 1 and A.stride(0) != 1:
        raise ValueError("expected a column-major matrix (stride(0) == 1)")
    return max(A.stride(1), m, 1) if m > 1 else max(m, 1)


def colmajor_to_device(A: np.ndarray, device="cuda", ld: int | None = None):
    """Copy a column-major numpy matrix to a column-major device tensor (ld >= m)."""
    import torch
    m, n = A.shape
    ld = m if ld is None else ld
    buf = torch.zeros((n, ld), dtype=torch.float64, device=device)
    buf[:, :m] = torch.from_numpy(np.ascontiguousarray(A.T))
    return buf.t()[:m]


def colmajor_empty(m: int, device="cuda", ld: int | None = None):
    import torch
    ld = m if ld is None else ld
    return torch.empty((m, max(ld, 1)), dtype=torch.float64, device=device).t()[:m]


def _stream_ptr(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


@dataclass
class Result:
    Z: object
    scales: object
    info: object


class Solver:
    """Holds a workspace for repeated calls of one order m (the workspace is the only
    allocation, made once by torch; the library itself allocates nothing)."""

    def __init__(self, m: int, mb: int = 0, normalize: bool = True, band: int = 0, device="cuda",
                 schedule: int = 0, watchdog: int = 0, precision: int = 0, left: bool = False,
                 max_refine: int = 0, refine_bits: int = 0, split: int = 0, grid: int = 0):
        import torch
        self.m = int(m)
        self.left = bool(left)
        self.opts = make_opts(mb, normalize, band, schedule, watchdog, precision, max_refine, refine_bits, split, grid)
        size = load().rtgevc_left_workspace_size if self.left else load().rtgevc_workspace_size
        self.nbytes = int(size(self.m, ctypes.byref(self.opts)))
        self.work = torch.empty(max(self.nbytes, 256), dtype=torch.uint8, device=device)
        self.device = device

    def run(self, S, T, select=None, Z=None, scales=None, info=None, stream=None) -> Result:
        import torch
        m = self.m
        lds, ldt = _ld(S, m), _ld(T, m)
        if Z is None:
            Z = colmajor_empty(m, self.device)
        ldz = _ld(Z, m)
        if scales is None:
            scales = torch.empty(max(m, 1), dtype=torch.int32, device=self.device)
        if info is None:
            info = torch.zeros(1, dtype=torch.int32, device=self.device)
        sel = None
        if select is not None:
            sel = torch.as_tensor(select, dtype=torch.int32, device=self.device).contiguous()
            if sel.shape != (m,):
                raise ValueError("select must have length m")
        fn = load().rtgevc_left if self.left else load().rtgevc
        rc = fn(m, S.data_ptr(), lds, T.data_ptr(), ldt,
                sel.data_ptr() if sel is not None else None,
                Z.data_ptr(), ldz, scales.data_ptr(), info.data_ptr(),
                self.work.data_ptr(), self.nbytes, ctypes.byref(self.opts),
                _stream_ptr(stream))
        _check(rc, "rtgevc_left" if self.left else "rtgevc")
        return Result(Z, scales[:m], info)

    def run_timed(self, S, T, Z, scales, info, stream=None):
        """rtgevc_timed: same work, HIP events around every launch; returns the stats
        dict (synchronises the stream).  Right eigenvectors only."""
        if self.left:
            raise RtgevcError("run_timed times the right-eigenvector call; time rtgevc_left with events")
        m = self.m
        lds, ldt, ldz = _ld(S, m), _ld(T, m), _ld(Z, m)
        st = (ctypes.c_double * TIMED_NSTATS)()
        rc = load().rtgevc_timed(m, S.data_ptr(), lds, T.data_ptr(), ldt, None, Z.data_ptr(), ldz,
                                 scales.data_ptr(), info.data_ptr(), self.work.data_ptr(), self.nbytes,
                                 ctypes.byref(self.opts), _stream_ptr(stream), st, TIMED_NSTATS)
        _check(rc, "rtgevc_timed")
        keys = ("total_ms", "pre_ms", "solve_ms", "update_ms", "consolidate_ms", "n_pre", "n_solve",
                "n_update", "n_consolidate", "update_flops", "M", "mb", "refine_ms", "sweeps",
                "side_update_ms", "side_update_flops", "n_side_update")
        return dict(zip(keys, list(st)))

    def eigvals(self, S, T, stream=None):
        import torch
        m = self.m
        lds, ldt = _ld(S, m), _ld(T, m)
        out = [torch.empty(max(m, 1), dtype=torch.float64, device=self.device) for _ in range(3)]
        info = torch.zeros(1, dtype=torch.int32, device=self.device)
        rc = load().rtgevc_eigvals(m, S.data_ptr(), lds, T.data_ptr(), ldt, out[0].data_ptr(),
                                   out[1].data_ptr(), out[2].data_ptr(), info.data_ptr(),
                                   self.work.data_ptr(), self.nbytes, ctypes.byref(self.opts),
                                   _stream_ptr(stream))
        _check(rc, "rtgevc_eigvals")
        return out[0][:m], out[1][:m], out[2][:m], info


def tgevc_left(S, T, select=None, normalize: bool = True, mb: int = 0, band: int = 0, stream=None,
               schedule: int = 0, precision: int = 0, max_refine: int = 0, refine_bits: int = 0) -> Result:
    """All (or the selected) left eigenvectors u of the Schur pencil, u^H (beta S - alpha T) = 0
    (Result.Z holds them)."""
    return Solver(S.shape[0], mb=mb, normalize=normalize, band=band, device=S.device,
                  schedule=schedule, precision=precision, left=True, max_refine=max_refine,
                  refine_bits=refine_bits).run(S, T, select, stream=stream)


def tgevc(S, T, select=None, normalize: bool = True, mb: int = 0, band: int = 0, stream=None,
          schedule: int = 0, precision: int = 0, max_refine: int = 0, refine_bits: int = 0) -> Result:
    """All (or the selected) right eigenvectors of the Schur pencil (S, T)."""
    return Solver(S.shape[0], mb=mb, normalize=normalize, band=band, device=S.device,
                  schedule=schedule, precision=precision, max_refine=max_refine,
                  refine_bits=refine_bits).run(S, T, select, stream=stream)


def tgevc_noalloc(S, T, select=None, normalize: bool = True, mb: int = 0, band: int = 0, stream=None,
                  schedule: int = 0, precision: int = 0, Z=None, scales=None, info=None,
                  max_refine: int = 0, refine_bits: int = 0) -> Result:
    """rtgevc_noalloc: the same eigenvectors as tgevc, computed in the library's fixed device
    scratch (no workspace; torch allocates only the outputs that are not passed in)."""
    import torch
    m = int(S.shape[0])
    dev = S.device
    lds, ldt = _ld(S, m), _ld(T, m)
    if Z is None:
        Z = colmajor_empty(m, dev)
    ldz = _ld(Z, m)
    if scales is None:
        scales = torch.empty(max(m, 1), dtype=torch.int32, device=dev)
    if info is None:
        info = torch.zeros(1, dtype=torch.int32, device=dev)
    sel = None
    if select is not None:
        sel = torch.as_tensor(select, dtype=torch.int32, device=dev).contiguous()
        if sel.shape != (m,):
            raise ValueError("select must have length m")
    o = make_opts(mb, normalize, band, schedule, 0, precision, max_refine, refine_bits)
    rc = load().rtgevc_noalloc(m, S.data_ptr(), lds, T.data_ptr(), ldt,
                               sel.data_ptr() if sel is not None else None,
                               Z.data_ptr(), ldz, scales.data_ptr(), info.data_ptr(),
                               ctypes.byref(o), _stream_ptr(stream))
    _check(rc, "rtgevc_noalloc")
    return Result(Z, scales[:m], info)


def _cld(A, m: int) -> int:
    import torch
    if A.dtype != torch.complex128 or A.dim() != 2 or A.device.type != "cuda":
        raise ValueError("expected a complex128 CUDA matrix")
    if tuple(A.shape) != (m, m):
        raise ValueError(f"expected shape ({m}, {m}), got {tuple(A.shape)}")
    if m > 1 and A.stride(0) != 1:
        raise ValueError("expected a column-major matrix (stride(0) == 1)")
    return max(A.stride(1), m, 1) if m > 1 else max(m, 1)


def ccolmajor_to_device(A: np.ndarray, device="cuda", ld: int | None = None):
    """Copy a column-major complex numpy matrix to a column-major complex128 device tensor."""
    import torch
    m, n = A.shape
    ld = m if ld is None else ld
    buf = torch.zeros((n, ld), dtype=torch.complex128, device=device)
    buf[:, :m] = torch.from_numpy(np.ascontiguousarray(A.T))
    return buf.t()[:m]


class ComplexSolver:
    """Eigenvectors of complex upper-triangular pencils of order m (rtgevc_complex), holding
    the workspace (one torch allocation, made once)."""

    def __init__(self, m: int, mb: int = 0, normalize: bool = True, band: int = 0, device="cuda",
                 schedule: int = 0, precision: int = 0, max_refine: int = 0, refine_bits: int = 0):
        import torch
        self.m = int(m)
        self.opts = make_opts(mb, normalize, band, schedule, 0, precision, max_refine, refine_bits)
        self.nbytes = int(load().rtgevc_complex_workspace_size(self.m, ctypes.byref(self.opts)))
        self.work = torch.empty(max(self.nbytes, 256), dtype=torch.uint8, device=device)
        self.device = device

    def run(self, S, T, select=None, Z=None, scales=None, info=None, stream=None) -> Result:
        import torch
        m = self.m
        lds, ldt = _cld(S, m), _cld(T, m)
        if Z is None:
            Z = torch.empty((m, max(m, 1)), dtype=torch.complex128, device=self.device).t()[:m]
        ldz = _cld(Z, m)
        if scales is None:
            scales = torch.empty(max(m, 1), dtype=torch.int32, device=self.device)
        if info is None:
            info = torch.zeros(1, dtype=torch.int32, device=self.device)
        sel = None
        if select is not None:
            sel = torch.as_tensor(select, dtype=torch.int32, device=self.device).contiguous()
            if sel.shape != (m,):
                raise ValueError("select must have length m")
        rc = load().rtgevc_complex(m, S.data_ptr(), lds, T.data_ptr(), ldt,
                                   sel.data_ptr() if sel is not None else None,
                                   Z.data_ptr(), ldz, scales.data_ptr(), info.data_ptr(),
                                   self.work.data_ptr(), self.nbytes, ctypes.byref(self.opts),
                                   _stream_ptr(stream))
        _check(rc, "rtgevc_complex")
        return Result(Z, scales[:m], info)


def tgevc_complex(S, T, select=None, normalize: bool = True, mb: int = 0, band: int = 0, stream=None,
                  schedule: int = 0, precision: int = 0) -> Result:
    """All (or the selected) right eigenvectors of a complex upper-triangular pencil (S, T)."""
    return ComplexSolver(S.shape[0], mb=mb, normalize=normalize, band=band, device=S.device,
                         schedule=schedule, precision=precision).run(S, T, select, stream=stream)


def _i64_array(vals):
    return (ctypes.c_int64 * len(vals))(*[int(v) for v in vals])


def _ptr_array(vals):
    return (ctypes.c_void_p * len(vals))(*[v if v is None else int(v) for v in vals])


class BatchSolver:
    """Holds the workspace of a batch of pencils with orders ``ms`` (one torch allocation,
    made once); ``run`` enqueues rtgevc_batched on the current stream and can be captured
    in a CUDA/HIP graph (it only launches kernels)."""

    def __init__(self, ms, mb: int = 0, normalize: bool = True, device="cuda", band: int = 0, split: int = 0):
        import torch
        self.ms = [int(v) for v in ms]
        self.count = len(self.ms)
        self.opts = make_opts(mb, normalize, band, split=split)
        self._m = _i64_array(self.ms)
        self.nbytes = int(load().rtgevc_batched_workspace_size(self.count, self._m, ctypes.byref(self.opts)))
        self.work = torch.empty(max(self.nbytes, 256), dtype=torch.uint8, device=device)
        self.device = device

    def outputs(self):
        """Fresh Z matrices, scales vectors and the info vector for this batch."""
        import torch
        Z = [colmajor_empty(m, self.device) for m in self.ms]
        sc = [torch.empty(max(m, 1), dtype=torch.int32, device=self.device) for m in self.ms]
        info = torch.zeros(max(self.count, 1), dtype=torch.int32, device=self.device)
        return Z, sc, info

    def run(self, S, T, Z, scales, info, select=None, stream=None):
        n = self.count
        if not (len(S) == len(T) == len(Z) == len(scales) == n):
            raise ValueError("one S, T, Z and scales per pencil")
        lds = [_ld(S[i], m) for i, m in enumerate(self.ms)]
        ldt = [_ld(T[i], m) for i, m in enumerate(self.ms)]
        ldz = [_ld(Z[i], m) for i, m in enumerate(self.ms)]
        sel = None
        if select is not None:
            sel = _ptr_array([None if x is None else x.data_ptr() for x in select])
        self._keep = (S, T, Z, scales, select)   # the device buffers outlive a captured graph's replays
        rc = load().rtgevc_batched(
            n, self._m, _ptr_array([x.data_ptr() for x in S]), _i64_array(lds),
            _ptr_array([x.data_ptr() for x in T]), _i64_array(ldt), sel,
            _ptr_array([x.data_ptr() for x in Z]), _i64_array(ldz),
            _ptr_array([x.data_ptr() for x in scales]), info.data_ptr(),
            self.work.data_ptr(), self.nbytes, ctypes.byref(self.opts), _stream_ptr(stream))
        _check(rc, "rtgevc_batched")
        return Z, [sc[:m] for sc, m in zip(scales, self.ms)], info


def tgevc_batched(S, T, select=None, normalize: bool = True, mb: int = 0, stream=None, band: int = 0,
                  split: int = 0):
    """Right eigenvectors of every pencil (S[i], T[i]) in one batched call."""
    bs = BatchSolver([x.shape[0] for x in S], mb=mb, normalize=normalize, device=S[0].device, band=band,
                     split=split)
    Z, sc, info = bs.outputs()
    return bs.run(S, T, Z, sc, info, select=select, stream=stream)


class BackTransformer:
    """Back-transformation X = V Z (rtgevc_backtransform) for one order m, holding its
    workspace (allocated once by torch)."""

    def __init__(self, m: int, mb: int = 0, normalize: bool = True, device="cuda"):
        import torch
        self.m = int(m)
        self.opts = make_opts(mb, normalize)
        self.nbytes = int(load().rtgevc_backtransform_workspace_size(self.m, ctypes.byref(self.opts)))
        self.work = torch.empty(max(self.nbytes, 256), dtype=torch.uint8, device=device)
        self.device = device

    def run(self, S, V, Z, scales=None, X=None, xscales=None, info=None, stream=None) -> Result:
        """Returns Result(X, xscales, info); X may be Z (in place)."""
        import torch
        m = self.m
        if X is None:
            X = colmajor_empty(m, self.device)
        if xscales is None:
            xscales = torch.empty(max(m, 1), dtype=torch.int32, device=self.device)
        if info is None:
            info = torch.zeros(1, dtype=torch.int32, device=self.device)
        rc = load().rtgevc_backtransform(m, S.data_ptr(), _ld(S, m), V.data_ptr(), _ld(V, m),
                                         Z.data_ptr(), _ld(Z, m),
                                         scales.data_ptr() if scales is not None else None,
                                         X.data_ptr(), _ld(X, m), xscales.data_ptr(), info.data_ptr(),
                                         self.work.data_ptr(), self.nbytes, ctypes.byref(self.opts),
                                         _stream_ptr(stream))
        _check(rc, "rtgevc_backtransform")
        return Result(X, xscales[:m], info)


def backtransform(S, V, Z, scales=None, X=None, normalize: bool = True, mb: int = 0, stream=None) -> Result:
    """Eigenvectors X = V Z of the original pencil (A, B) = (Q S V^T, Q T V^T) from the
    Schur-form eigenvectors (Z, scales) returned by tgevc."""
    return BackTransformer(S.shape[0], mb=mb, normalize=normalize, device=S.device).run(
        S, V, Z, scales, X=X, stream=stream)
