"""ORACLE -- test infrastructure, not part of the product.

Thin ctypes binding of ``oracle.c``: a plain single-threaded CPU implementation
(IEEE double) of the Gaia AVU-GSR PC-LSQR hot path -- aprod 1 / aprod 2
(Algorithms 1 and 2 of arXiv 2212.11675), the column-norm preconditioner
(Section 2), PC-LSQR with its variance estimate (Section 3 flowchart; Paige & Saunders
1982), the mixed-precision residual correction and the adjoint gradient.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the GPU library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
# a different build of the same source (e.g. a deliberately broken copy used to check that
# the pins catch mistakes) can be swapped in for a test run
_LIB = os.environ.get("GSR_ORACLE_LIB", _LIB)


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with gcc: -O2, no OpenMP, no fast-math, no FMA contraction."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-shared", "-fPIC", "-std=c11",
                               "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Dims(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_stars", ctypes.c_int64),
                ("n_dfa", ctypes.c_int32), ("n_instr", ctypes.c_int32),
                ("n_glob", ctypes.c_int32)]


class Con(ctypes.Structure):
    """Constraint rows (compressed row form, absolute columns, binary64 values)."""
    _fields_ = [("n_con", ctypes.c_int64), ("ptr", ctypes.c_void_p), ("col", ctypes.c_void_p),
                ("val", ctypes.c_void_p)]


class Info(ctypes.Structure):
    _fields_ = [("itn", ctypes.c_int32), ("istop", ctypes.c_int32),
                ("rnorm", ctypes.c_double), ("arnorm", ctypes.c_double),
                ("anorm", ctypes.c_double), ("znorm", ctypes.c_double),
                ("bnorm", ctypes.c_double), ("acond", ctypes.c_double)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        vp, i32, f64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
        pd = ctypes.POINTER(Dims)
        pc = ctypes.c_void_p  # or_con * (NULL: no constraint rows)
        lib.or_n_cols.restype = ctypes.c_int64
        lib.or_n_cols.argtypes = [pd]
        for name in ("or_aprod1", "or_aprod2"):
            f = getattr(lib, name)
            f.restype = None
            f.argtypes = [pd, vp, vp, vp, vp, pc, vp, vp]
        lib.or_colnorm.restype = None
        lib.or_colnorm.argtypes = [pd, vp, vp, vp, vp, pc, vp]
        lib.or_pclsqr.restype = ctypes.c_int
        lib.or_pclsqr.argtypes = [pd, vp, vp, vp, vp, pc, vp, vp, i32, i32, f64, f64, f64, vp,
                                  ctypes.POINTER(Info), vp]
        lib.or_pclsqr_var.restype = ctypes.c_int
        lib.or_pclsqr_var.argtypes = [pd, vp, vp, vp, vp, pc, vp, vp, i32, i32, f64, f64, f64,
                                      vp, vp, ctypes.POINTER(Info)]
        lib.or_lsqr_transposed.restype = ctypes.c_int
        lib.or_lsqr_transposed.argtypes = [pd, vp, vp, vp, vp, pc, vp, vp, i32, i32, f64, f64,
                                           f64, vp, ctypes.POINTER(Info)]
        lib.or_residual.restype = None
        lib.or_residual.argtypes = [pd, vp, vp, vp, vp, pc, vp, vp, vp]
        lib.or_refine.restype = i32
        lib.or_refine.argtypes = [pd, vp, vp, vp, vp, vp, pc, vp, i32, f64, i32, i32, i32, f64,
                                  f64, f64, vp, vp]
        lib.or_grad_vals.restype = None
        lib.or_grad_vals.argtypes = [pd, vp, vp, vp, vp, vp, vp, vp, vp]
        _lib = lib
    return _lib


def _p(a):
    if a is None:
        return None
    assert isinstance(a, np.ndarray) and a.flags["C_CONTIGUOUS"], "contiguous numpy array expected"
    return a.ctypes.data


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i32(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


class System:
    """A system in the compressed row format (Section 3): per row 24 coefficients in the
    slot order [5 astrometric | 3x4 attitude | 6 instrumental | 1 global], the star
    number, the attitude start t (relative to the attitude section) and 6 instrumental
    indices (relative to the instrumental section).

    `con` (optional): constraint equations appended below the observation rows, a dict
    with ``ptr`` [n_con+1] int64, ``col`` [nnz] int64 (absolute columns) and ``val`` [nnz]
    float64.  Row-space vectors (b, y, r, mu) then have n_rows + n_con entries."""

    def __init__(self, dims: dict, vals, star, att, instr, con: dict | None = None):
        self.d = Dims(int(dims["n_rows"]), int(dims["n_stars"]), int(dims["n_dfa"]),
                      int(dims["n_instr"]), int(dims.get("n_glob", 1)))
        assert self.d.n_glob == 1
        self.vals = _f64(vals)
        self.star = _i32(star)
        self.att = _i32(att)
        self.instr = _i32(instr)
        m = self.d.n_rows
        assert self.vals.size == 24 * m and self.star.size == m and self.att.size == m
        assert self.instr.size == 6 * m
        self.con = None
        self._con = None
        if con is not None:
            ptr, col, val = _i64(con["ptr"]), _i64(con["col"]), _f64(con["val"])
            assert ptr.size >= 1 and ptr[0] == 0 and col.size == val.size == ptr[-1]
            assert np.all(np.diff(ptr) >= 0)
            if col.size:
                assert col.min() >= 0 and col.max() < self.n
            self.con = dict(ptr=ptr, col=col, val=val)
            self._con = Con(ptr.size - 1, _p(ptr), _p(col) if col.size else None,
                            _p(val) if val.size else None)

    @property
    def m(self) -> int:
        """Rows of the operator: observation rows plus constraint rows."""
        return self.d.n_rows + self.n_con

    @property
    def n_con(self) -> int:
        return 0 if self._con is None else int(self._con.n_con)

    def _cp(self):
        return None if self._con is None else ctypes.addressof(self._con)

    @property
    def n(self) -> int:
        return int(_load().or_n_cols(ctypes.byref(self.d)))

    def _args(self, vals=None):
        return (ctypes.byref(self.d), _p(self.vals if vals is None else vals), _p(self.star),
                _p(self.att), _p(self.instr), self._cp())

    def with_vals(self, vals) -> "System":
        return System(dict(n_rows=self.d.n_rows, n_stars=self.d.n_stars, n_dfa=self.d.n_dfa,
                           n_instr=self.d.n_instr, n_glob=1), vals, self.star, self.att,
                      self.instr, con=self.con)

    # Algorithm 1
    def aprod1(self, x, y=None) -> np.ndarray:
        """y += A x (returns y; y = 0 if not given)."""
        x = _f64(x)
        assert x.size == self.n
        y = np.zeros(self.m) if y is None else _f64(y).copy()
        _load().or_aprod1(*self._args(), _p(x), _p(y))
        return y

    # Algorithm 2
    def aprod2(self, y, x=None) -> np.ndarray:
        """x += A^T y (returns x; x = 0 if not given)."""
        y = _f64(y)
        assert y.size == self.m
        x = np.zeros(self.n) if x is None else _f64(x).copy()
        _load().or_aprod2(*self._args(), _p(y), _p(x))
        return x

    def colnorm(self) -> np.ndarray:
        p = np.empty(self.n)
        _load().or_colnorm(*self._args(), _p(p))
        return p

    def lsqr(self, b, itnlim=100, fixed=True, atol=1e-14, btol=1e-14, precond=True, p=None,
             hist=False, conlim=0.0):
        """PC-LSQR.  Returns (x, info dict[, per-iteration rnorm estimates])."""
        b = _f64(b)
        assert b.size == self.m
        if precond and p is None:
            p = self.colnorm()
        x = np.empty(self.n)
        info = Info()
        h = np.zeros(max(itnlim, 1)) if hist else None
        _load().or_pclsqr(*self._args(), _p(p) if precond else None, _p(b), int(itnlim),
                          int(bool(fixed)), float(atol), float(btol), float(conlim), _p(x),
                          ctypes.byref(info), _p(h))
        if hist:
            return x, info.as_dict(), h[: info.itn]
        return x, info.as_dict()

    def lsqr_var(self, b, itnlim=100, fixed=True, atol=1e-14, btol=1e-14, p=None, conlim=0.0):
        """PC-LSQR with the variance estimate: returns (x, var, info dict); var estimates
        diag((A^T A)^-1)."""
        b = _f64(b)
        assert b.size == self.m
        if p is None:
            p = self.colnorm()
        x, var = np.empty(self.n), np.empty(self.n)
        info = Info()
        _load().or_pclsqr_var(*self._args(), _p(_f64(p)), _p(b), int(itnlim), int(bool(fixed)),
                              float(atol), float(btol), float(conlim), _p(x), _p(var),
                              ctypes.byref(info))
        return x, var, info.as_dict()

    def lsqr_transposed(self, g, itnlim=1000, fixed=False, atol=1e-14, btol=1e-14, p=None,
                        precond=True, conlim=0.0):
        """Minimum-norm mu with A^T mu = g (LSQR on D A^T)."""
        g = _f64(g)
        assert g.size == self.n
        if precond and p is None:
            p = self.colnorm()
        mu = np.empty(self.m)
        info = Info()
        _load().or_lsqr_transposed(*self._args(), _p(p) if precond else None, _p(g),
                                   int(itnlim), int(bool(fixed)), float(atol), float(btol),
                                   float(conlim), _p(mu), ctypes.byref(info))
        return mu, info.as_dict()

    def residual(self, b, x) -> np.ndarray:
        b, x = _f64(b), _f64(x)
        r = np.empty(self.m)
        _load().or_residual(*self._args(), _p(b), _p(x), _p(r))
        return r

    def refine(self, b, vals_lo, max_outer=5, refine_tol=1e-10, inner_itnlim=200,
               inner_fixed=False, inner_atol=1e-14, inner_btol=1e-14, later_itnlim=0,
               first_tol=0.0):
        """Mixed-precision residual correction; vals_lo = binary32-rounded coefficients
        (any float array; widened exactly to double); the correction solves after the first
        take later_itnlim iterations at most (0: inner_itnlim); the first inner solve stops
        at atol = btol = first_tol when first_tol > 0.  Returns (x, outer, inner_itns)."""
        b = _f64(b)
        lo = np.ascontiguousarray(np.asarray(vals_lo, dtype=np.float32).astype(np.float64))
        x = np.empty(self.n)
        inner = np.zeros(max(max_outer, 1), dtype=np.int32)
        k = _load().or_refine(ctypes.byref(self.d), _p(self.vals), _p(lo), _p(self.star),
                              _p(self.att), _p(self.instr), self._cp(), _p(b), int(max_outer),
                              float(refine_tol), int(inner_itnlim), int(later_itnlim),
                              int(bool(inner_fixed)),
                              float(inner_atol), float(inner_btol), float(first_tol), _p(x),
                              _p(inner))
        return x, int(k), inner[:k].tolist()

    def grad_vals(self, r, mu, x, lam) -> np.ndarray:
        r, mu, x, lam = _f64(r), _f64(mu), _f64(x), _f64(lam)
        dv = np.empty(24 * self.d.n_rows)
        _load().or_grad_vals(ctypes.byref(self.d), _p(self.star), _p(self.att), _p(self.instr),
                             _p(r), _p(mu), _p(x), _p(lam), _p(dv))
        return dv

    def solve_and_grad(self, b, g, itnlim=2000, atol=1e-15, btol=1e-15):
        """Converged forward solve x*, then the adjoint: mu = dL/db (min-norm solution of
        A^T mu = g), lam = argmin ||A lam - mu|| = (A^T A)^{-1} g, and dL/dvals."""
        x, _ = self.lsqr(b, itnlim=itnlim, fixed=False, atol=atol, btol=btol)
        r = self.residual(b, x)
        mu, _ = self.lsqr_transposed(g, itnlim=itnlim, fixed=False, atol=atol, btol=btol)
        lam, _ = self.lsqr(mu, itnlim=itnlim, fixed=False, atol=atol, btol=btol)
        return dict(x=x, r=r, mu=mu, lam=lam, dvals=self.grad_vals(r, mu, x, lam))
