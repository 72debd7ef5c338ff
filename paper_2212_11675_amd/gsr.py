"""ctypes binding of ``libgsr.so`` (C ABI declared in include/gsr.h).

Argument marshalling only: every step of the hot path runs in the library's HIP kernels.
Functions carry the C names; array arguments are torch CUDA tensors (the binding passes
their device pointers and the current HIP stream).  Raises ``GsrError`` on any non-OK
status and ``ImportError`` if the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgsr.so")
ABI_VERSION = 4  # GSR_ABI_VERSION of include/gsr.h

GSR_F64 = 0
GSR_F32V = 1

_STATUS = {0: "GSR_OK", -1: "GSR_E_INVAL", -2: "GSR_E_LAYOUT", -3: "GSR_E_NOMEM",
           -4: "GSR_E_HIP", -5: "GSR_E_BREAKDOWN", -6: "GSR_E_UNSUPPORTED",
           -7: "GSR_E_NODEVICE"}

#: every entry point include/gsr.h declares
EXPORTS = (
    "gsr_abi_version", "gsr_status_string", "gsr_last_error", "gsr_lsqr_setup", "gsr_destroy",
    "gsr_get_size", "gsr_aprod1", "gsr_aprod2", "gsr_aprod1_f32v", "gsr_aprod2_f32v",
    "gsr_precond", "gsr_residual", "gsr_lsqr_solve", "gsr_lsqr_solve_var",
    "gsr_lsqr_solve_async", "gsr_lsqr_solve_adjoint", "gsr_grad_vals", "gsr_set_constraints",
    "gsr_update_values", "gsr_aprod2_noalloc",
    "gsr_batch_setup", "gsr_batch_destroy", "gsr_batch_col_offsets", "gsr_batch_aprod1",
    "gsr_batch_aprod2", "gsr_batch_solve",
)


class GsrError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        self.status = status
        super().__init__(f"{where}: {_STATUS.get(status, status)}: {message}")


class Dims(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_stars", ctypes.c_int64),
                ("n_dfa", ctypes.c_int32), ("n_instr", ctypes.c_int32),
                ("n_glob", ctypes.c_int32)]


class SetupOpts(ctypes.Structure):
    _fields_ = [("build_f32", ctypes.c_int32), ("validate", ctypes.c_int32),
                ("allow_empty_cols", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("itnlim", ctypes.c_int32), ("fixed_iters", ctypes.c_int32),
                ("atol", ctypes.c_double), ("btol", ctypes.c_double),
                ("precision", ctypes.c_int32), ("max_refine", ctypes.c_int32),
                ("refine_tol", ctypes.c_double), ("check_every", ctypes.c_int32),
                ("profile", ctypes.c_int32), ("conlim", ctypes.c_double),
                ("refine_itnlim", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("refine_first_tol", ctypes.c_double)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("itn", ctypes.c_int32), ("istop", ctypes.c_int32),
                ("n_refine", ctypes.c_int32), ("nonfinite", ctypes.c_int32),
                ("rnorm", ctypes.c_double), ("arnorm", ctypes.c_double),
                ("anorm", ctypes.c_double), ("znorm", ctypes.c_double),
                ("bnorm", ctypes.c_double), ("ms_pass1", ctypes.c_double),
                ("ms_pass2", ctypes.c_double), ("n_pass", ctypes.c_int32),
                ("fused", ctypes.c_int32), ("acond", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load() -> ctypes.CDLL:
    """The loaded library; raises ImportError if it was never built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    st = ctypes.c_int
    sig = {
        "gsr_abi_version": (i32, []),
        "gsr_status_string": (ctypes.c_char_p, [st]),
        "gsr_last_error": (ctypes.c_char_p, []),
        "gsr_lsqr_setup": (st, [ctypes.POINTER(Dims), vp, vp, vp, vp, ctypes.POINTER(SetupOpts),
                                vp, ctypes.POINTER(vp)]),
        "gsr_destroy": (st, [vp]),
        "gsr_get_size": (st, [vp, ctypes.POINTER(i64), ctypes.POINTER(i64)]),
        "gsr_aprod1": (st, [vp, vp, vp, vp]),
        "gsr_aprod2": (st, [vp, vp, vp, vp]),
        "gsr_aprod1_f32v": (st, [vp, vp, vp, vp]),
        "gsr_aprod2_f32v": (st, [vp, vp, vp, vp]),
        "gsr_precond": (st, [vp, i32, vp, vp]),
        "gsr_residual": (st, [vp, vp, vp, vp, vp]),
        "gsr_lsqr_solve": (st, [vp, vp, vp, ctypes.POINTER(SolveOpts),
                                ctypes.POINTER(SolveInfo), vp]),
        "gsr_lsqr_solve_var": (st, [vp, vp, vp, vp, ctypes.POINTER(SolveOpts),
                                    ctypes.POINTER(SolveInfo), vp]),
        "gsr_lsqr_solve_async": (st, [vp, vp, vp, ctypes.POINTER(SolveOpts), vp, vp]),
        "gsr_lsqr_solve_adjoint": (st, [vp, vp, vp, vp, ctypes.POINTER(SolveOpts),
                                        ctypes.POINTER(SolveInfo), vp]),
        "gsr_grad_vals": (st, [vp, vp, vp, vp, vp, vp, vp]),
        "gsr_set_constraints": (st, [vp, i64, vp, vp, vp, vp]),
        "gsr_update_values": (st, [vp, vp, vp]),
        "gsr_aprod2_noalloc": (st, [ctypes.POINTER(Dims), vp, vp, vp, vp, vp, vp, vp]),
        "gsr_batch_setup": (st, [i32, ctypes.POINTER(Dims), ctypes.POINTER(i64), vp, vp, vp, vp,
                                 i32, ctypes.POINTER(SetupOpts), vp, ctypes.POINTER(vp)]),
        "gsr_batch_destroy": (st, [vp]),
        "gsr_batch_col_offsets": (st, [vp, ctypes.POINTER(i64)]),
        "gsr_batch_aprod1": (st, [vp, vp, vp, vp]),
        "gsr_batch_aprod2": (st, [vp, vp, vp, vp]),
        "gsr_batch_solve": (st, [vp, vp, vp, ctypes.POINTER(SolveOpts),
                                 ctypes.POINTER(SolveInfo), vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if lib.gsr_abi_version() != ABI_VERSION:
        raise ImportError(f"{LIB_PATH} has ABI version {lib.gsr_abi_version()}, this binding "
                          f"expects {ABI_VERSION}: rebuild it")
    _lib = lib
    return lib


def _check(status: int, where: str):
    if status != 0:
        msg = load().gsr_last_error().decode(errors="replace")
        raise GsrError(status, where, msg)


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(t: torch.Tensor, dtype: torch.dtype, numel: int | None, name: str) -> ctypes.c_void_p:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name}: a CUDA (HIP) tensor is required")
    if t.dtype != dtype:
        raise TypeError(f"{name}: dtype {t.dtype}, expected {dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: tensor must be contiguous")
    if numel is not None and t.numel() != numel:
        raise ValueError(f"{name}: {t.numel()} elements, expected {numel}")
    return ctypes.c_void_p(t.data_ptr())


def make_dims(n_rows, n_stars, n_dfa, n_instr, n_glob=1) -> Dims:
    return Dims(int(n_rows), int(n_stars), int(n_dfa), int(n_instr), int(n_glob))


def solve_opts(itnlim=100, fixed_iters=True, atol=1e-14, btol=1e-14, precision=GSR_F64,
               max_refine=4, refine_tol=1e-10, check_every=16, profile=False,
               conlim=0.0, refine_itnlim=0, refine_first_tol=0.0) -> SolveOpts:
    return SolveOpts(int(itnlim), int(bool(fixed_iters)), float(atol), float(btol),
                     int(precision), int(max_refine), float(refine_tol), int(check_every),
                     int(bool(profile)), float(conlim), int(refine_itnlim), 0,
                     float(refine_first_tol))


class Handle:
    """An opened system; keeps the caller's tensors alive while the library references them."""

    def __init__(self, ptr: ctypes.c_void_p, dims: Dims, keep: tuple):
        self.ptr = ptr
        self.dims = dims
        self._keep = keep
        self._con = None
        self.n_obs = int(dims.n_rows)
        self._sizes()

    def _sizes(self):
        n_rows, n_cols = ctypes.c_int64(), ctypes.c_int64()
        _check(load().gsr_get_size(self.ptr, ctypes.byref(n_rows), ctypes.byref(n_cols)),
               "gsr_get_size")
        self.m, self.n = n_rows.value, n_cols.value

    def close(self):
        if self.ptr:
            _check(load().gsr_destroy(self.ptr), "gsr_destroy")
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gsr_lsqr_setup(dims: Dims, vals, star, att, instr, *, build_f32=False, validate=True,
                   allow_empty_cols=False, stream=None) -> Handle:
    m = dims.n_rows
    args = (_dev(vals, torch.float64, 24 * m, "vals"), _dev(star, torch.int32, m, "star"),
            _dev(att, torch.int32, m, "att"), _dev(instr, torch.int32, 6 * m, "instr"))
    opts = SetupOpts(int(build_f32), int(validate), int(allow_empty_cols), 0)
    out = ctypes.c_void_p()
    _check(load().gsr_lsqr_setup(ctypes.byref(dims), *args, ctypes.byref(opts), _stream(stream),
                                 ctypes.byref(out)), "gsr_lsqr_setup")
    return Handle(out, dims, (vals, star, att, instr))


def gsr_destroy(h: Handle):
    h.close()


def gsr_aprod1(h: Handle, x, y, stream=None):
    """y += A x"""
    _check(load().gsr_aprod1(h.ptr, _dev(x, torch.float64, h.n, "x"),
                             _dev(y, torch.float64, h.m, "y"), _stream(stream)), "gsr_aprod1")


def gsr_aprod2(h: Handle, y, x, stream=None):
    """x += A^T y"""
    _check(load().gsr_aprod2(h.ptr, _dev(y, torch.float64, h.m, "y"),
                             _dev(x, torch.float64, h.n, "x"), _stream(stream)), "gsr_aprod2")


def gsr_aprod1_f32v(h: Handle, x, y, stream=None):
    _check(load().gsr_aprod1_f32v(h.ptr, _dev(x, torch.float64, h.n, "x"),
                                  _dev(y, torch.float64, h.m, "y"), _stream(stream)),
           "gsr_aprod1_f32v")


def gsr_aprod2_f32v(h: Handle, y, x, stream=None):
    _check(load().gsr_aprod2_f32v(h.ptr, _dev(y, torch.float64, h.m, "y"),
                                  _dev(x, torch.float64, h.n, "x"), _stream(stream)),
           "gsr_aprod2_f32v")


def gsr_precond(h: Handle, p, precision=GSR_F64, stream=None):
    _check(load().gsr_precond(h.ptr, int(precision), _dev(p, torch.float64, h.n, "p"),
                              _stream(stream)), "gsr_precond")


def gsr_residual(h: Handle, b, x, r, stream=None):
    _check(load().gsr_residual(h.ptr, _dev(b, torch.float64, h.m, "b"),
                               _dev(x, torch.float64, h.n, "x"), _dev(r, torch.float64, h.m, "r"),
                               _stream(stream)), "gsr_residual")


def gsr_lsqr_solve(h: Handle, b, x, opts: SolveOpts | None = None, stream=None) -> dict:
    info = SolveInfo()
    _check(load().gsr_lsqr_solve(h.ptr, _dev(b, torch.float64, h.m, "b"),
                                 _dev(x, torch.float64, h.n, "x"),
                                 ctypes.byref(opts) if opts is not None else None,
                                 ctypes.byref(info), _stream(stream)), "gsr_lsqr_solve")
    return info.as_dict()


def gsr_lsqr_solve_var(h: Handle, b, x, var, opts: SolveOpts | None = None,
                       stream=None) -> dict:
    """PC-LSQR plus the variance estimate var ~ diag((A^T A)^-1) (binary64)."""
    info = SolveInfo()
    _check(load().gsr_lsqr_solve_var(h.ptr, _dev(b, torch.float64, h.m, "b"),
                                     _dev(x, torch.float64, h.n, "x"),
                                     _dev(var, torch.float64, h.n, "var"),
                                     ctypes.byref(opts) if opts is not None else None,
                                     ctypes.byref(info), _stream(stream)), "gsr_lsqr_solve_var")
    return info.as_dict()


def solve_info_buffer(device="cuda") -> torch.Tensor:
    """Device memory for one gsr_solve_info (the output of gsr_lsqr_solve_async)."""
    return torch.zeros(ctypes.sizeof(SolveInfo), dtype=torch.uint8, device=device)


def read_solve_info(buf: torch.Tensor) -> dict:
    """Copy a device gsr_solve_info to the host.  The copy is ordered on torch's current
    stream: if the solve ran on another stream, synchronize that stream first."""
    host_bytes = buf.cpu().numpy().tobytes()
    return SolveInfo.from_buffer_copy(host_bytes).as_dict()


def gsr_lsqr_solve_async(h: Handle, b, x, info_dev, opts: SolveOpts | None = None,
                         stream=None) -> None:
    """Stream-ordered PC-LSQR (binary64, or the precision form with its correction loop
    tested on the device): no synchronization, capturable into a graph; the solve
    information lands in info_dev (see solve_info_buffer / read_solve_info)."""
    _check(load().gsr_lsqr_solve_async(h.ptr, _dev(b, torch.float64, h.m, "b"),
                                       _dev(x, torch.float64, h.n, "x"),
                                       ctypes.byref(opts) if opts is not None else None,
                                       _dev(info_dev, torch.uint8, ctypes.sizeof(SolveInfo),
                                            "info_dev"),
                                       _stream(stream)), "gsr_lsqr_solve_async")


def gsr_lsqr_solve_adjoint(h: Handle, g, mu, lam, opts: SolveOpts | None = None,
                           stream=None) -> tuple[dict, dict]:
    info = (SolveInfo * 2)()
    _check(load().gsr_lsqr_solve_adjoint(h.ptr, _dev(g, torch.float64, h.n, "g"),
                                         _dev(mu, torch.float64, h.m, "mu"),
                                         _dev(lam, torch.float64, h.n, "lam"),
                                         ctypes.byref(opts) if opts is not None else None,
                                         info, _stream(stream)), "gsr_lsqr_solve_adjoint")
    return info[0].as_dict(), info[1].as_dict()


def gsr_grad_vals(h: Handle, r, mu, x, lam, dvals, stream=None):
    _check(load().gsr_grad_vals(h.ptr, _dev(r, torch.float64, h.m, "r"),
                                _dev(mu, torch.float64, h.m, "mu"),
                                _dev(x, torch.float64, h.n, "x"),
                                _dev(lam, torch.float64, h.n, "lam"),
                                _dev(dvals, torch.float64, 24 * h.n_obs, "dvals"),
                                _stream(stream)), "gsr_grad_vals")


def gsr_update_values(h: Handle, vals, stream=None):
    """New coefficient values (same index map): the handle's copies and preconditioner are
    rebuilt in place; the handle references `vals` from now on."""
    _check(load().gsr_update_values(h.ptr, _dev(vals, torch.float64, 24 * h.n_obs, "vals"),
                                    _stream(stream)), "gsr_update_values")
    h._keep = (vals,) + tuple(h._keep[1:])


def gsr_aprod2_noalloc(dims: Dims, vals, star, att, instr, y, x, stream=None):
    """x += A^T y on the caller's arrays, no handle and no allocation (the library's fixed
    device scratch holds the block partial sums; calls overlapping on one GPU race)."""
    m = dims.n_rows
    n = 5 * dims.n_stars + 3 * dims.n_dfa + dims.n_instr + dims.n_glob
    _check(load().gsr_aprod2_noalloc(ctypes.byref(dims), _dev(vals, torch.float64, 24 * m, "vals"),
                                     _dev(star, torch.int32, m, "star"),
                                     _dev(att, torch.int32, m, "att"),
                                     _dev(instr, torch.int32, 6 * m, "instr"),
                                     _dev(y, torch.float64, m, "y"),
                                     _dev(x, torch.float64, n, "x"), _stream(stream)),
           "gsr_aprod2_noalloc")


def gsr_set_constraints(h: Handle, ptr=None, col=None, val=None, stream=None):
    """Constraint rows C (compressed rows: ptr [n_con+1] int64, col [nnz] int64 absolute
    columns, val [nnz] float64, CUDA tensors) below the observation rows; None removes them.
    Row-space vectors of the handle then have h.m = n_rows + n_con entries."""
    if ptr is None:
        _check(load().gsr_set_constraints(h.ptr, 0, None, None, None, _stream(stream)),
               "gsr_set_constraints")
        h._con = None
    else:
        n_con = ptr.numel() - 1
        if n_con < 0:
            raise ValueError("ptr: at least one entry (n_con + 1) is required")
        nnz = col.numel()
        args = (_dev(ptr, torch.int64, n_con + 1, "ptr"), _dev(col, torch.int64, nnz, "col"),
                _dev(val, torch.float64, nnz, "val"))
        h._con = None  # after an error the handle has no constraint rows
        try:
            _check(load().gsr_set_constraints(h.ptr, n_con, *args, _stream(stream)),
                   "gsr_set_constraints")
            h._con = (ptr, col, val)
        finally:
            h._sizes()
        return
    h._sizes()


# ---- batching -----------------------------------------------------------------------------

class Batch:
    def __init__(self, ptr, n_sys, k, row_offset, keep):
        self.ptr = ptr
        self.n_sys = n_sys
        self.k = k
        self.row_offset = list(row_offset)
        self._keep = keep
        co = (ctypes.c_int64 * (n_sys + 1))()
        _check(load().gsr_batch_col_offsets(ptr, co), "gsr_batch_col_offsets")
        self.col_offset = list(co)
        self.m = self.row_offset[-1]
        self.n = self.col_offset[-1]

    def close(self):
        if self.ptr:
            _check(load().gsr_batch_destroy(self.ptr), "gsr_batch_destroy")
            self.ptr = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def gsr_batch_setup(dims_list, row_offset, vals, star, att, instr, k, *, validate=True,
                    allow_empty_cols=False, stream=None) -> Batch:
    n_sys = len(dims_list)
    darr = (Dims * n_sys)(*dims_list)
    ro = (ctypes.c_int64 * (n_sys + 1))(*[int(v) for v in row_offset])
    m = int(row_offset[-1])
    args = (_dev(vals, torch.float64, 24 * m, "vals"), _dev(star, torch.int32, m, "star"),
            _dev(att, torch.int32, m, "att"), _dev(instr, torch.int32, 6 * m, "instr"))
    opts = SetupOpts(0, int(validate), int(allow_empty_cols), 0)
    out = ctypes.c_void_p()
    _check(load().gsr_batch_setup(n_sys, darr, ro, *args, int(k), ctypes.byref(opts),
                                  _stream(stream), ctypes.byref(out)), "gsr_batch_setup")
    return Batch(out, n_sys, int(k), row_offset, (vals, star, att, instr))


def gsr_batch_destroy(b: Batch):
    b.close()


def gsr_batch_aprod1(b: Batch, X, Y, stream=None):
    _check(load().gsr_batch_aprod1(b.ptr, _dev(X, torch.float64, b.n * b.k, "X"),
                                   _dev(Y, torch.float64, b.m * b.k, "Y"), _stream(stream)),
           "gsr_batch_aprod1")


def gsr_batch_aprod2(b: Batch, Y, X, stream=None):
    _check(load().gsr_batch_aprod2(b.ptr, _dev(Y, torch.float64, b.m * b.k, "Y"),
                                   _dev(X, torch.float64, b.n * b.k, "X"), _stream(stream)),
           "gsr_batch_aprod2")


def gsr_batch_solve(b: Batch, B, X, opts: SolveOpts | None = None, stream=None) -> list[dict]:
    """Per-pair solve information (entry s*k + j).  On a breakdown (GSR_E_BREAKDOWN) the
    raised GsrError carries the same list as `.info`."""
    info = (SolveInfo * (b.n_sys * b.k))()
    st = load().gsr_batch_solve(b.ptr, _dev(B, torch.float64, b.m * b.k, "B"),
                                _dev(X, torch.float64, b.n * b.k, "X"),
                                ctypes.byref(opts) if opts is not None else None, info,
                                _stream(stream))
    out = [i.as_dict() for i in info]
    try:
        _check(st, "gsr_batch_solve")
    except GsrError as e:
        e.info = out
        raise
    return out
