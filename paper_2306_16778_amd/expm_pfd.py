"""Python binding of libexpm_pfd (include/expm_pfd.h): argument marshalling only.

Every function here has the name of the C entry point it calls.  Device arrays
are torch tensors on the GPU (PyTorch supplies device memory and streams); all
arithmetic runs in the library's HIP kernels.  The binding never falls back to a
CPU computation: if the library is missing it raises.

Layout: the C ABI takes column-major complex128 matrices.  A torch tensor X of
shape (rows, cols) is passed as-is when it is already column-major
(X.stride() == (1, ld)), otherwise as a column-major copy.  Results come back as
column-major tensors of the logical shape (rows, cols).
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libexpm_pfd.so")

EXPM_PFD_FP64 = 0
EXPM_PFD_MIXED = 1
# largest order and degree the library accepts (EXPM_PFD_MAX_N, EXPM_PFD_MAX_DEGREE)
MAX_N = 8192
MAX_DEGREE = 64

# every symbol declared in include/expm_pfd.h
EXPORTED = (
    "expm_pfd_constants",
    "expm_pfd_plan",
    "expm_pfd_workspace_bytes",
    "expm_pfd_apply",
    "expm_pfd_destroy",
    "expm_pfd_plan_check",
    "expm_pfd_apply_noalloc",
    "expm_pfd_apply_batched",
    "expm_pfd_batch_plan",
    "expm_pfd_batch_apply",
    "expm_pfd_batch_check",
    "expm_pfd_batch_info",
    "expm_pfd_batch_destroy",
    "expm_pfd_tridiag_plan",
    "expm_pfd_tridiag_factor",
    "expm_pfd_tridiag_apply",
    "expm_pfd_tridiag_diagonals",
    "expm_pfd_tridiag_destroy",
    "expm_pfd_band_plan",
    "expm_pfd_band_apply",
    "expm_pfd_band_destroy",
    "expm_pfd_choose_degree",
    "expm_pfd_strerror",
    "expm_pfd_trace",
    "expm_pfd_trace_summary",
    "expm_pfd_queue_create",
    "expm_pfd_register_matrix",
    "expm_pfd_unregister_matrix",
    "expm_pfd_submit",
    "expm_pfd_poll",
    "expm_pfd_wait",
    "expm_pfd_queue_drain",
    "expm_pfd_queue_stats_get",
    "expm_pfd_queue_destroy",
)

# kernel classes of the tracer (EXPM_PFD_K_*)
KERNEL_CLASSES = ("form", "panel", "lu_gemm", "lu_trsm", "moves", "solve_trsm", "solve_gemm", "accum",
                  "ir_gemm", "elementwise", "lu_trail")


class ExpmPfdError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {expm_pfd_strerror(code)} (code {code})")
        self.code = code


class _QueueStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("tridiag_requests", ctypes.c_int64), ("reductions", ctypes.c_int64),
                ("completed", ctypes.c_int64), ("failed", ctypes.c_int64),
                ("fallbacks", ctypes.c_int64), ("groups", ctypes.c_int64),
                ("p50_ms", ctypes.c_double), ("p99_ms", ctypes.c_double), ("mean_ms", ctypes.c_double),
                ("max_ms", ctypes.c_double), ("solves_per_s", ctypes.c_double),
                ("mean_group_size", ctypes.c_double), ("padded_up", ctypes.c_int64), ("peak_bytes", ctypes.c_size_t),
                ("registered", ctypes.c_int64), ("registered_bytes", ctypes.c_size_t)]


class _Opts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("ir_max_iter", ctypes.c_int), ("ir_extended", ctypes.c_int),
                ("real_data", ctypes.c_int), ("graph", ctypes.c_int), ("autotune", ctypes.c_int),
                ("lu_tile", ctypes.c_int), ("uplo", ctypes.c_int), ("shift", ctypes.c_double),
                ("ir_tol", ctypes.c_double), ("shift_scale_t", ctypes.c_int), ("tridiag_reuse", ctypes.c_int)]

# tile shapes of the LU trailing update, in the order of expm_pfd_opts.lu_tile - 1
LU_TILES = ("64x64", "128x64", "64x128")


_lib = None


def load_library() -> ctypes.CDLL:
    """Load libexpm_pfd.so from the package directory (built by build())."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"libexpm_pfd.so is not built ({LIB_PATH}); run python -m paper_2306_16778_amd.build")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, c_int, c_double = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    lib.expm_pfd_constants.argtypes = [c_int, vp, vp]
    lib.expm_pfd_plan.argtypes = [ctypes.POINTER(vp), i64, c_int, c_double, i64, ctypes.POINTER(_Opts)]
    lib.expm_pfd_workspace_bytes.argtypes = [i64, c_int, i64, ctypes.POINTER(_Opts), ctypes.POINTER(ctypes.c_size_t)]
    lib.expm_pfd_apply.argtypes = [vp, vp, i64, vp, i64, i64, vp, i64, vp]
    lib.expm_pfd_destroy.argtypes = [vp]
    lib.expm_pfd_plan_check.argtypes = [vp]
    lib.expm_pfd_apply_noalloc.argtypes = [i64, c_int, c_double, vp, i64, vp, i64, i64, vp, i64,
                                           ctypes.POINTER(_Opts), vp, vp]
    lib.expm_pfd_apply_batched.argtypes = [c_int, vp, vp, c_int, vp, vp, vp, vp, vp, vp, vp,
                                           ctypes.POINTER(_Opts), vp, vp]
    lib.expm_pfd_batch_plan.argtypes = [ctypes.POINTER(vp), c_int, vp, vp, c_int, ctypes.POINTER(_Opts)]
    lib.expm_pfd_batch_apply.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.expm_pfd_batch_check.argtypes = [vp]
    lib.expm_pfd_batch_info.argtypes = [vp, ctypes.POINTER(c_int), ctypes.POINTER(c_int), ctypes.POINTER(c_int)]
    lib.expm_pfd_batch_destroy.argtypes = [vp]
    lib.expm_pfd_tridiag_plan.argtypes = [ctypes.POINTER(vp), i64, c_int, i64, ctypes.POINTER(_Opts)]
    lib.expm_pfd_tridiag_factor.argtypes = [vp, vp, i64, vp]
    lib.expm_pfd_tridiag_apply.argtypes = [vp, c_double, vp, i64, i64, vp, i64, vp]
    lib.expm_pfd_tridiag_diagonals.argtypes = [vp, vp, vp]
    lib.expm_pfd_tridiag_destroy.argtypes = [vp]
    lib.expm_pfd_band_plan.argtypes = [ctypes.POINTER(vp), i64, i64, c_int, i64, ctypes.POINTER(_Opts)]
    lib.expm_pfd_band_apply.argtypes = [vp, c_double, vp, i64, vp, i64, i64, vp, i64, vp]
    lib.expm_pfd_band_destroy.argtypes = [vp]
    lib.expm_pfd_choose_degree.argtypes = [c_double, c_int, ctypes.POINTER(c_int), ctypes.POINTER(c_double)]
    lib.expm_pfd_trace.argtypes = [c_int]
    lib.expm_pfd_trace_summary.argtypes = [c_int, ctypes.POINTER(c_double), ctypes.POINTER(i64),
                                           ctypes.POINTER(c_double), ctypes.POINTER(c_double)]
    lib.expm_pfd_queue_create.argtypes = [ctypes.POINTER(vp), ctypes.c_size_t, c_int, ctypes.POINTER(_Opts), c_int,
                                          c_int]
    lib.expm_pfd_register_matrix.argtypes = [vp, vp, i64, i64, vp, ctypes.POINTER(i64)]
    lib.expm_pfd_unregister_matrix.argtypes = [vp, i64]
    lib.expm_pfd_submit.argtypes = [vp, i64, vp, i64, i64, c_double, vp, i64, i64, vp, i64, vp,
                                    ctypes.POINTER(ctypes.c_uint64)]
    lib.expm_pfd_poll.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(c_int), ctypes.POINTER(c_int)]
    lib.expm_pfd_wait.argtypes = [vp, ctypes.c_uint64, ctypes.POINTER(c_int)]
    lib.expm_pfd_queue_drain.argtypes = [vp]
    lib.expm_pfd_queue_stats_get.argtypes = [vp, ctypes.POINTER(_QueueStats)]
    lib.expm_pfd_queue_destroy.argtypes = [vp]
    lib.expm_pfd_strerror.argtypes = [c_int]
    lib.expm_pfd_strerror.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name != "expm_pfd_strerror":
            getattr(lib, name).restype = c_int
    _lib = lib
    return lib


def _check(code: int, where: str):
    if code != 0:
        raise ExpmPfdError(code, where)


def _opts(precision, ir_max_iter, ir_extended=0, shift=0.0, real_data=False, graph=False, autotune=False,
          lu_tile=None, uplo="L", ir_tol=0.0, shift_scale_t=False) -> _Opts:
    p = {"fp64": EXPM_PFD_FP64, "mixed": EXPM_PFD_MIXED}.get(precision, precision)
    o = _Opts()
    o.precision = int(p)
    o.ir_max_iter = int(ir_max_iter)
    o.ir_extended = int(ir_extended)
    o.shift = float(shift)
    o.ir_tol = float(ir_tol)
    o.shift_scale_t = 1 if shift_scale_t else 0
    o.real_data = 1 if real_data else 0
    o.graph = 1 if graph else 0
    o.autotune = 1 if autotune else 0
    o.lu_tile = 0 if lu_tile is None else (LU_TILES.index(lu_tile) + 1 if isinstance(lu_tile, str) else int(lu_tile))
    o.uplo = {"L": 0, "U": 1}.get(uplo, uplo)
    return o


def expm_pfd_strerror(code: int) -> str:
    return load_library().expm_pfd_strerror(int(code)).decode()


def expm_pfd_constants(degree: int):
    """(theta, a): complex128 arrays of length degree/2 (host only)."""
    lib = load_library()
    th = np.zeros(2 * max(degree // 2, 1), dtype=np.float64)
    a = np.zeros_like(th)
    _check(lib.expm_pfd_constants(int(degree), th.ctypes.data, a.ctypes.data), "expm_pfd_constants")
    return th.view(np.complex128).copy(), a.view(np.complex128).copy()


def expm_pfd_workspace_bytes(n: int, degree: int, m_max: int = 0, precision="fp64", ir_max_iter: int = 0) -> int:
    lib = load_library()
    out = ctypes.c_size_t(0)
    o = _opts(precision, ir_max_iter)
    _check(lib.expm_pfd_workspace_bytes(int(n), int(degree), int(m_max), ctypes.byref(o), ctypes.byref(out)),
           "expm_pfd_workspace_bytes")
    return int(out.value)


class Plan:
    """Owns an expm_pfd_plan_t."""

    def __init__(self, handle, n, degree, t, m_max, precision):
        self.handle = handle
        self.n, self.degree, self.t, self.m_max, self.precision = n, degree, t, m_max, precision

    def __del__(self):
        try:
            if self.handle:
                expm_pfd_destroy(self)
        except Exception:
            pass


def expm_pfd_plan(n: int, degree: int, t: float, m_max: int = 0, precision="fp64", ir_max_iter: int = 0,
                  ir_extended: int = 0, shift: float = 0.0, real_data: bool = False, graph: bool = False,
                  autotune: bool = False, lu_tile=None, uplo="L", ir_tol: float = 0.0,
                  shift_scale_t: bool = False) -> Plan:
    """lu_tile: None (built-in or autotuned), a name from LU_TILES, or the C option value (1..3).
    uplo: "L" (lower triangle of A read) or "U"."""
    lib = load_library()
    h = ctypes.c_void_p()
    o = _opts(precision, ir_max_iter, ir_extended, shift, real_data, graph, autotune, lu_tile, uplo, ir_tol,
              shift_scale_t)
    _check(lib.expm_pfd_plan(ctypes.byref(h), int(n), int(degree), float(t), int(m_max), ctypes.byref(o)),
           "expm_pfd_plan")
    return Plan(h.value, n, degree, t, m_max, precision)


def expm_pfd_destroy(plan: Plan):
    if plan.handle:
        _check(load_library().expm_pfd_destroy(plan.handle), "expm_pfd_destroy")
        plan.handle = None


def expm_pfd_plan_check(plan: Plan) -> int:
    """Raise ExpmPfdError if a triangular sweep of this plan lost its dependency order;
    otherwise 0, or 1 if the last apply's refinement missed its tolerance (mixed plans
    with the convergence test)."""
    rc = load_library().expm_pfd_plan_check(plan.handle)
    if rc < 0:
        _check(rc, "expm_pfd_plan_check")
    return rc


def _colmajor(x, torch):
    """Column-major complex128 device tensor with the same logical shape; returns (tensor, ld)."""
    if x.dtype != torch.complex128:
        raise TypeError("complex128 expected")
    if not x.is_cuda:
        raise TypeError("device tensor expected")
    r, c = x.shape
    if x.stride(0) == 1 and x.stride(1) >= max(r, 1):
        return x, x.stride(1)
    y = x.t().contiguous().t()
    return y, max(r, 1)


def _stream_ptr(stream, torch):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def expm_pfd_apply(plan: Plan, A, V=None, X=None, stream=None):
    """X = R_d(tA)V (V None: V = I).  Returns X (column-major complex128 tensor)."""
    import torch

    lib = load_library()
    Ac, lda = _colmajor(A, torch)
    n = Ac.shape[0]
    if V is None:
        Vp, ldv, m = None, n, n
    else:
        Vc, ldv = _colmajor(V, torch)
        Vp, m = Vc.data_ptr(), Vc.shape[1]
    if X is None:
        X = torch.empty((m, n), dtype=torch.complex128, device=Ac.device).t()
    if not (X.stride(0) == 1 and X.stride(1) >= n and tuple(X.shape) == (n, m)):
        raise ValueError("X must be a column-major (n, m) complex128 tensor")
    _check(lib.expm_pfd_apply(plan.handle, Ac.data_ptr(), lda, Vp, ldv, m, X.data_ptr(), X.stride(1),
                              _stream_ptr(stream, torch)), "expm_pfd_apply")
    # keep staged copies alive until the stream has consumed them
    X._expm_keepalive = (Ac, V if V is None else Vc)
    return X


# size of the library's fixed device scratch array (EXPM_PFD_NOALLOC_BYTES)
NOALLOC_BYTES = 128 << 20


def expm_pfd_apply_noalloc(n: int, degree: int, t: float, A, V=None, X=None, precision="fp64",
                           ir_max_iter: int = 0, ir_extended: int = 0, shift: float = 0.0, real_data: bool = False,
                           lu_tile=None, uplo="L", info=None, stream=None, ir_tol: float = 0.0,
                           shift_scale_t: bool = False):
    """X = R_d(tA)V without any device allocation by the library (its fixed scratch
    array holds the workspace).  X, when given, must be a column-major (n, m)
    complex128 tensor; info an optional int32 device tensor of one element."""
    import torch

    lib = load_library()
    Ac, lda = _colmajor(A, torch)
    if Ac.shape[0] != n:
        raise ValueError("A must be n x n")
    if V is None:
        Vp, ldv, m, Vc = None, n, n, None
    else:
        Vc, ldv = _colmajor(V, torch)
        Vp, m = Vc.data_ptr(), Vc.shape[1]
    if X is None:
        X = torch.empty((m, n), dtype=torch.complex128, device=Ac.device).t()
    if not (X.stride(0) == 1 and X.stride(1) >= n and tuple(X.shape) == (n, m)):
        raise ValueError("X must be a column-major (n, m) complex128 tensor")
    if info is not None and (info.dtype != torch.int32 or not info.is_cuda or info.numel() != 1):
        raise ValueError("info must be a one-element int32 device tensor")
    o = _opts(precision, ir_max_iter, ir_extended, shift, real_data, lu_tile=lu_tile, uplo=uplo, ir_tol=ir_tol,
              shift_scale_t=shift_scale_t)
    _check(lib.expm_pfd_apply_noalloc(int(n), int(degree), float(t), Ac.data_ptr(), lda, Vp, ldv, m, X.data_ptr(),
                                      X.stride(1), ctypes.byref(o), None if info is None else info.data_ptr(),
                                      _stream_ptr(stream, torch)), "expm_pfd_apply_noalloc")
    X._expm_keepalive = (Ac, Vc)
    return X


def expm_pfd_apply_batched(As: Sequence, Vs: Sequence, ts: Sequence[float], degree: int, precision="fp64",
                           ir_max_iter: int = 0, stream=None, info=None, uplo="L", shift: float = 0.0,
                           real_data: bool = False, ir_extended: int = 0, ir_tol: float = 0.0,
                           shift_scale_t: bool = False):
    """X_i = R_d(t_i A_i) V_i for every i (V_i None: V_i = I).  Returns the list of X_i.

    info: optional host int32 numpy array of len(As), filled with each problem's status."""
    import torch

    lib = load_library()
    count = len(As)
    Ac, Vc, Xs = [], [], []
    n = np.zeros(count, np.int64)
    lda = np.zeros(count, np.int64)
    ldv = np.zeros(count, np.int64)
    m = np.zeros(count, np.int64)
    ldx = np.zeros(count, np.int64)
    t = np.asarray(ts, dtype=np.float64)
    pa = (ctypes.c_void_p * count)()
    pv = (ctypes.c_void_p * count)()
    px = (ctypes.c_void_p * count)()
    for i in range(count):
        a, la = _colmajor(As[i], torch)
        Ac.append(a)
        n[i], lda[i], pa[i] = a.shape[0], la, a.data_ptr()
        if Vs[i] is None:
            Vc.append(None)
            m[i], ldv[i], pv[i] = n[i], n[i], None
        else:
            v, lv = _colmajor(Vs[i], torch)
            Vc.append(v)
            m[i], ldv[i], pv[i] = v.shape[1], lv, v.data_ptr()
        x = torch.empty((int(m[i]), int(n[i])), dtype=torch.complex128, device=a.device).t()
        Xs.append(x)
        ldx[i], px[i] = n[i], x.data_ptr()
    o = _opts(precision, ir_max_iter, ir_extended, shift, real_data, uplo=uplo, ir_tol=ir_tol,
              shift_scale_t=shift_scale_t)
    if info is not None and (info.dtype != np.int32 or info.size != count or not info.flags.c_contiguous):
        raise ValueError("info must be a contiguous int32 array with one entry per problem")
    _check(lib.expm_pfd_apply_batched(count, n.ctypes.data, t.ctypes.data, int(degree), pa, lda.ctypes.data, pv,
                                      ldv.ctypes.data, m.ctypes.data, px, ldx.ctypes.data, ctypes.byref(o),
                                      _stream_ptr(stream, torch), None if info is None else info.ctypes.data),
           "expm_pfd_apply_batched")
    return Xs


class BatchPlan:
    """Owns an expm_pfd_batch_t and the host arrays of its problem shapes."""

    def __init__(self, handle, n, m):
        self.handle = handle
        self.n, self.m = n, m
        self._keep = None

    def __del__(self):
        try:
            if self.handle:
                expm_pfd_batch_destroy(self)
        except Exception:
            pass


def expm_pfd_batch_plan(n: Sequence[int], m: Sequence[int], degree: int, precision="fp64", ir_max_iter: int = 0,
                        graph: bool = False, autotune: bool = False, lu_tile=None,
                        real_data: bool = False, uplo="L", shift: float = 0.0, ir_extended: int = 0,
                        ir_tol: float = 0.0, shift_scale_t: bool = False) -> BatchPlan:
    """Batch plan for problems of orders n[i] with m[i] right-hand-side columns (0: V_i = I)."""
    lib = load_library()
    nn = np.ascontiguousarray(n, dtype=np.int64)
    mm = np.ascontiguousarray(m, dtype=np.int64)
    if nn.shape != mm.shape:
        raise ValueError("n and m must have the same length")
    h = ctypes.c_void_p()
    o = _opts(precision, ir_max_iter, ir_extended, shift, real_data, graph, autotune, lu_tile, uplo, ir_tol,
              shift_scale_t)
    _check(lib.expm_pfd_batch_plan(ctypes.byref(h), len(nn), nn.ctypes.data, mm.ctypes.data, int(degree),
                                   ctypes.byref(o)), "expm_pfd_batch_plan")
    return BatchPlan(h.value, nn, mm)


def expm_pfd_batch_apply(b: BatchPlan, As: Sequence, Vs: Sequence, ts: Sequence[float], Xs=None, stream=None,
                         info=None):
    """X_i = R_d(t_i A_i) V_i on the plan's problems (V_i None where m[i] = 0).  Returns the list of X_i.

    info: optional int32 device tensor with one entry per problem, written with each status.
    The inputs (and any column-major copies made here) are kept alive on the plan
    until its next apply, so the asynchronous launches can read them."""
    import torch

    lib = load_library()
    count = len(b.n)
    if len(As) != count or len(Vs) != count or len(ts) != count:
        raise ValueError("one A, V and t per problem of the plan")
    Ac, Vc, out = [], [], []
    lda = np.zeros(count, np.int64)
    ldv = np.zeros(count, np.int64)
    ldx = np.zeros(count, np.int64)
    t = np.asarray(ts, dtype=np.float64)
    pa = (ctypes.c_void_p * count)()
    pv = (ctypes.c_void_p * count)()
    px = (ctypes.c_void_p * count)()
    for i in range(count):
        a, la = _colmajor(As[i], torch)
        if a.shape[0] != b.n[i]:
            raise ValueError(f"A[{i}] has order {a.shape[0]}, the plan {b.n[i]}")
        Ac.append(a)
        lda[i], pa[i] = la, a.data_ptr()
        cols = int(b.m[i]) if b.m[i] else int(b.n[i])
        if Vs[i] is None:
            Vc.append(None)
            ldv[i], pv[i] = b.n[i], None
        else:
            v, lv = _colmajor(Vs[i], torch)
            Vc.append(v)
            ldv[i], pv[i] = lv, v.data_ptr()
        x = Xs[i] if Xs is not None else torch.empty((cols, int(b.n[i])), dtype=torch.complex128,
                                                      device=a.device).t()
        if not (x.stride(0) == 1 and tuple(x.shape) == (int(b.n[i]), cols)):
            raise ValueError("X must be column-major (n, m) complex128")
        out.append(x)
        ldx[i], px[i] = x.stride(1), x.data_ptr()
    if info is not None and (info.dtype != torch.int32 or not info.is_cuda or info.numel() != count
                             or not info.is_contiguous()):
        raise ValueError("info must be a contiguous int32 device tensor with one entry per problem")
    _check(lib.expm_pfd_batch_apply(b.handle, t.ctypes.data, pa, lda.ctypes.data, pv, ldv.ctypes.data, px,
                                    ldx.ctypes.data, None if info is None else info.data_ptr(),
                                    _stream_ptr(stream, torch)), "expm_pfd_batch_apply")
    b._keep = (Ac, Vc, out, info)
    return out


def expm_pfd_batch_check(b: BatchPlan):
    _check(load_library().expm_pfd_batch_check(b.handle), "expm_pfd_batch_check")


def expm_pfd_batch_info(b: BatchPlan) -> dict:
    g, s, t = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    _check(load_library().expm_pfd_batch_info(b.handle, ctypes.byref(g), ctypes.byref(s), ctypes.byref(t)),
           "expm_pfd_batch_info")
    return {"groups": g.value, "schedule": s.value, "lu_tile_max": LU_TILES[t.value]}


def expm_pfd_batch_destroy(b: BatchPlan):
    if b.handle:
        _check(load_library().expm_pfd_batch_destroy(b.handle), "expm_pfd_batch_destroy")
        b.handle = None
        b._keep = None


class TridiagPlan:
    """Owns an expm_pfd_tri_t (the tridiagonal route: one reduction of A, many t)."""

    def __init__(self, handle, n, degree, m_max):
        self.handle = handle
        self.n, self.degree, self.m_max = n, degree, m_max
        self._keep = None

    def __del__(self):
        try:
            if self.handle:
                expm_pfd_tridiag_destroy(self)
        except Exception:
            pass


def expm_pfd_tridiag_plan(n: int, degree: int, m_max: int = 16, uplo="L", shift: float = 0.0,
                          shift_scale_t: bool = False) -> TridiagPlan:
    lib = load_library()
    h = ctypes.c_void_p()
    o = _opts("fp64", 0, shift=shift, uplo=uplo, shift_scale_t=shift_scale_t)
    _check(lib.expm_pfd_tridiag_plan(ctypes.byref(h), int(n), int(degree), int(m_max), ctypes.byref(o)),
           "expm_pfd_tridiag_plan")
    return TridiagPlan(h.value, n, degree, m_max)


def expm_pfd_tridiag_factor(tri: TridiagPlan, A, stream=None):
    """A = Q T Q^H on the device (asynchronous on `stream`, default the current one)."""
    import torch

    Ac, lda = _colmajor(A, torch)
    if Ac.shape[0] != tri.n:
        raise ValueError("A must be n x n")
    _check(load_library().expm_pfd_tridiag_factor(tri.handle, Ac.data_ptr(), lda, _stream_ptr(stream, torch)),
           "expm_pfd_tridiag_factor")
    tri._keep = Ac


def expm_pfd_tridiag_apply(tri: TridiagPlan, t: float, V, X=None, stream=None):
    """X = R_d(tA)V from the plan's reduction of A.  V: (n, m) complex128 device tensor."""
    import torch

    Vc, ldv = _colmajor(V, torch)
    n, m = Vc.shape
    if X is None:
        X = torch.empty((m, n), dtype=torch.complex128, device=Vc.device).t()
    if not (X.stride(0) == 1 and X.stride(1) >= n and tuple(X.shape) == (n, m)):
        raise ValueError("X must be a column-major (n, m) complex128 tensor")
    _check(load_library().expm_pfd_tridiag_apply(tri.handle, float(t), Vc.data_ptr(), ldv, m, X.data_ptr(),
                                                 X.stride(1), _stream_ptr(stream, torch)), "expm_pfd_tridiag_apply")
    X._expm_keepalive = Vc
    return X


def expm_pfd_tridiag_diagonals(tri: TridiagPlan):
    """(d, e): diagonal and subdiagonal of T (host float64 arrays)."""
    d = np.zeros(tri.n)
    e = np.zeros(max(tri.n - 1, 1))
    _check(load_library().expm_pfd_tridiag_diagonals(tri.handle, d.ctypes.data, e.ctypes.data),
           "expm_pfd_tridiag_diagonals")
    return d, e[: tri.n - 1]


def expm_pfd_tridiag_destroy(tri: TridiagPlan):
    if tri.handle:
        _check(load_library().expm_pfd_tridiag_destroy(tri.handle), "expm_pfd_tridiag_destroy")
        tri.handle = None
        tri._keep = None


class BandPlan:
    """Owns an expm_pfd_band_t (the banded route)."""

    def __init__(self, handle, n, kd, degree, m_max):
        self.handle = handle
        self.n, self.kd, self.degree, self.m_max = n, kd, degree, m_max

    def __del__(self):
        try:
            if self.handle:
                expm_pfd_band_destroy(self)
        except Exception:
            pass


def expm_pfd_band_plan(n: int, kd: int, degree: int, m_max: int = 16, uplo="L", real_data: bool = False,
                       shift: float = 0.0, shift_scale_t: bool = False) -> BandPlan:
    lib = load_library()
    h = ctypes.c_void_p()
    o = _opts("fp64", 0, shift=shift, real_data=real_data, uplo=uplo, shift_scale_t=shift_scale_t)
    _check(lib.expm_pfd_band_plan(ctypes.byref(h), int(n), int(kd), int(degree), int(m_max), ctypes.byref(o)),
           "expm_pfd_band_plan")
    return BandPlan(h.value, n, kd, degree, m_max)


def expm_pfd_band_apply(plan: BandPlan, t: float, AB, V, X=None, stream=None):
    """X = R_d(tA)V for A in band storage.  AB: (ldab >= kd + 1, n) complex128 device
    tensor in LAPACK band layout (column j of AB holds column j's band); V: (n, m)."""
    import torch

    ABc, ldab = _colmajor(AB, torch)
    Vc, ldv = _colmajor(V, torch)
    n, m = Vc.shape
    if ABc.shape[1] != plan.n or n != plan.n:
        raise ValueError("AB must have n columns and V n rows")
    if X is None:
        X = torch.empty((m, n), dtype=torch.complex128, device=Vc.device).t()
    if not (X.stride(0) == 1 and X.stride(1) >= n and tuple(X.shape) == (n, m)):
        raise ValueError("X must be a column-major (n, m) complex128 tensor")
    _check(load_library().expm_pfd_band_apply(plan.handle, float(t), ABc.data_ptr(), ldab, Vc.data_ptr(), ldv, m,
                                              X.data_ptr(), X.stride(1), _stream_ptr(stream, torch)),
           "expm_pfd_band_apply")
    X._expm_keepalive = (ABc, Vc)
    return X


def expm_pfd_band_destroy(plan: BandPlan):
    if plan.handle:
        _check(load_library().expm_pfd_band_destroy(plan.handle), "expm_pfd_band_destroy")
        plan.handle = None


def expm_pfd_choose_degree(tol: float, digits: int = 16):
    """(degree, bound, guaranteed): the degree adapted to `digits` significant digits
    for the uniform tolerance `tol` (host only)."""
    d = ctypes.c_int()
    b = ctypes.c_double()
    rc = load_library().expm_pfd_choose_degree(float(tol), int(digits), ctypes.byref(d), ctypes.byref(b))
    if rc < 0:
        _check(rc, "expm_pfd_choose_degree")
    return d.value, b.value, rc == 0


def expm_pfd_trace(classes=()):
    """Time later launches of the given kernel classes (names or indices); () stops. Clears records."""
    mask = 0
    for c in classes:
        mask |= 1 << (KERNEL_CLASSES.index(c) if isinstance(c, str) else int(c))
    _check(load_library().expm_pfd_trace(mask), "expm_pfd_trace")


def expm_pfd_trace_summary(kernel_class):
    """dict(ms, launches, flops, bytes) for a kernel class (name or EXPM_PFD_K_* index)."""
    cls = KERNEL_CLASSES.index(kernel_class) if isinstance(kernel_class, str) else int(kernel_class)
    ms, fl, by = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    k = ctypes.c_int64()
    _check(load_library().expm_pfd_trace_summary(cls, ctypes.byref(ms), ctypes.byref(k), ctypes.byref(fl),
                                                 ctypes.byref(by)), "expm_pfd_trace_summary")
    return {"ms": ms.value, "launches": k.value, "flops": fl.value, "bytes": by.value}


# ---- queued serving ---------------------------------------------------------------

class Queue:
    """Owns an expm_pfd_queue_t and keeps each request's device tensors alive until it completes."""

    def __init__(self, handle):
        self.handle = handle
        self._live = {}
        self._sources = []  # registered matrices' sources until their copies are done

    def __del__(self):
        try:
            if self.handle:
                expm_pfd_queue_destroy(self)
        except Exception:
            pass


def expm_pfd_queue_create(hbm_budget: int, degree: int, precision="fp64", ir_max_iter: int = 0, max_group: int = 64,
                          streams: int = 3, shift: float = 0.0, real_data: bool = False,
                          ir_extended: int = 0, uplo="L", ir_tol: float = 0.0, shift_scale_t: bool = False,
                          tridiag_reuse: int = 0) -> Queue:
    lib = load_library()
    h = ctypes.c_void_p()
    o = _opts(precision, ir_max_iter, ir_extended, shift, real_data, uplo=uplo, ir_tol=ir_tol,
              shift_scale_t=shift_scale_t)
    o.tridiag_reuse = int(tridiag_reuse)
    _check(lib.expm_pfd_queue_create(ctypes.byref(h), int(hbm_budget), int(degree), ctypes.byref(o), int(max_group),
                                     int(streams)), "expm_pfd_queue_create")
    return Queue(h.value)


def expm_pfd_register_matrix(q: Queue, A, stream=None) -> int:
    """Register A with the queue (copied on `stream`, default the current one, after the
    work already enqueued there); returns the matrix id."""
    import torch

    Ac, lda = _colmajor(A, torch)
    mid = ctypes.c_int64()
    _check(load_library().expm_pfd_register_matrix(q.handle, Ac.data_ptr(), Ac.shape[0], lda,
                                                   _stream_ptr(stream, torch), ctypes.byref(mid)),
           "expm_pfd_register_matrix")
    # the copy is stream-ordered: keep the source alive until the stream has passed it
    q._sources.append((Ac, torch.cuda.Event()))
    q._sources[-1][1].record(stream if stream is not None else torch.cuda.current_stream())
    q._sources = [(a, e) for a, e in q._sources if not e.query()]
    return int(mid.value)


def expm_pfd_unregister_matrix(q: Queue, mat_id: int):
    _check(load_library().expm_pfd_unregister_matrix(q.handle, int(mat_id)), "expm_pfd_unregister_matrix")


def expm_pfd_submit(q: Queue, mat, t: float, V, X=None, stream=None):
    """Enqueue X = R_d(t A) V; returns (ticket, X).

    mat: a registered matrix id, or an (n, n) complex128 device tensor read in place (kept alive
    here until the ticket completes).  V: (n, m) complex128 device tensor, m <= 16.  The request is
    ordered after the work already enqueued on `stream` (default: the current stream)."""
    import torch

    Vc, ldv = _colmajor(V, torch)
    n, m = Vc.shape
    if X is None:
        X = torch.empty((m, n), dtype=torch.complex128, device=Vc.device).t()
    tk = ctypes.c_uint64()
    if isinstance(mat, int):
        Ac, ap, lda = None, None, n
        mid = int(mat)
    else:
        Ac, lda = _colmajor(mat, torch)
        if Ac.shape != (n, n):
            raise ValueError("A must be n x n with n the rows of V")
        ap, mid = Ac.data_ptr(), -1
    _check(load_library().expm_pfd_submit(q.handle, mid, ap, n, lda, float(t), Vc.data_ptr(), m, ldv, X.data_ptr(),
                                          X.stride(1), _stream_ptr(stream, torch), ctypes.byref(tk)),
           "expm_pfd_submit")
    q._live[tk.value] = (Vc, X, Ac)
    return tk.value, X


def expm_pfd_poll(q: Queue, ticket: int):
    """(done, info): done is True once the ticket's result is in X; info its status then
    (0, 1: solved again on the FP64 path after the refinement missed its tolerance, 2: non-finite)."""
    d, info = ctypes.c_int(), ctypes.c_int()
    _check(load_library().expm_pfd_poll(q.handle, ctypes.c_uint64(ticket), ctypes.byref(d), ctypes.byref(info)),
           "expm_pfd_poll")
    if d.value:
        q._live.pop(ticket, None)
    return bool(d.value), int(info.value)


def expm_pfd_wait(q: Queue, ticket: int) -> int:
    """Block until the ticket completes; returns its status (as expm_pfd_poll's info)."""
    info = ctypes.c_int()
    _check(load_library().expm_pfd_wait(q.handle, ctypes.c_uint64(ticket), ctypes.byref(info)), "expm_pfd_wait")
    q._live.pop(ticket, None)
    return int(info.value)


def expm_pfd_queue_drain(q: Queue):
    _check(load_library().expm_pfd_queue_drain(q.handle), "expm_pfd_queue_drain")
    q._live.clear()


def expm_pfd_queue_stats_get(q: Queue) -> dict:
    st = _QueueStats()
    _check(load_library().expm_pfd_queue_stats_get(q.handle, ctypes.byref(st)), "expm_pfd_queue_stats_get")
    return {k: getattr(st, k) for k, _ in _QueueStats._fields_}


def expm_pfd_queue_destroy(q: Queue):
    if q.handle:
        _check(load_library().expm_pfd_queue_destroy(q.handle), "expm_pfd_queue_destroy")
        q.handle = None
        q._live.clear()
        q._sources = []
