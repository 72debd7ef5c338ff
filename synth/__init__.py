"""Seeded synthetic inputs shaped like the Gaia AVU-GSR observation matrix.

The paper's data are confidential; these generators stand in for them with
the structure of Section 3: one row per observation, rows sorted by star,
24 non-zero coefficients per row laid out as 5 astrometric (star block),
3 x 4 attitude (one 4-wide block per axis, axis stride N_DFA), 6 instrumental
(no regular pattern) and 1 global (PPN gamma) coefficient.

This module only draws random numbers (see ``synth.c`` for the generator's
definition).  It holds none of the solver's arithmetic: the right-hand side
b = A x_true + e is formed by the consumer (the oracle in tests, the library
itself in the benchmark).  Both the oracle and the GPU path read their
inputs from here; nothing here imports either of them.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "synth.c")
_LIB = os.path.join(_HERE, "libsynth.so")

SIGMA_NOISE = 1e-3  # standard deviation of the observation noise

STREAM_XTRUE = 4
STREAM_NOISE = 5
STREAM_XREF = 7
STREAM_STARS = 8
STREAM_CON_VALS = 10
STREAM_RHS_X = 64
STREAM_RHS_NOISE = 4096


def build(force: bool = True) -> str:
    """Compile ``libsynth.so`` with gcc (plain C, OpenMP over index ranges)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        u64, i64, i32, u32 = ctypes.c_uint64, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32
        vp = ctypes.c_void_p
        lib.syn_key.restype = u64
        lib.syn_key.argtypes = [u64, u64]
        lib.syn_uniform.restype = ctypes.c_double
        lib.syn_uniform.argtypes = [u64, u64]
        lib.syn_normal.restype = ctypes.c_double
        lib.syn_normal.argtypes = [u64, u64]
        lib.syn_below.restype = u32
        lib.syn_below.argtypes = [u64, u64, u32]
        lib.syn_fill_normal.restype = None
        lib.syn_fill_normal.argtypes = [u64, u64, i64, i64, ctypes.c_double, vp]
        lib.syn_star_counts.restype = None
        lib.syn_star_counts.argtypes = [u64, i64, i32, i32, vp]
        lib.syn_rows.restype = None
        lib.syn_rows.argtypes = [u64, i32, i32, i64, i64, vp, vp, vp]
        lib.syn_primary_stars.restype = i64
        lib.syn_primary_stars.argtypes = [u64, i64, ctypes.c_double, vp]
        lib.syn_star_of_rows.restype = None
        lib.syn_star_of_rows.argtypes = [vp, i64, i64, i64, vp]
        _lib = lib
    return _lib


def _ptr(a: np.ndarray | None):
    if a is None:
        return None
    assert a.flags["C_CONTIGUOUS"]
    return a.ctypes.data


@dataclass(frozen=True)
class Shape:
    """Sizes and seed of one synthetic system.

    n_stars stars, each observed obs_lo..obs_hi times (equal bounds: fixed),
    n_dfa attitude degrees of freedom per axis, n_instr instrumental columns,
    one global column.
    """

    n_stars: int
    obs_lo: int
    obs_hi: int
    n_dfa: int
    n_instr: int
    seed: int
    name: str = ""

    @property
    def n_glob(self) -> int:
        return 1

    @property
    def n_cols(self) -> int:
        return 5 * self.n_stars + 3 * self.n_dfa + self.n_instr + 1

    def star_counts(self) -> np.ndarray:
        c = np.empty(self.n_stars, dtype=np.int32)
        _load().syn_star_counts(self.seed, self.n_stars, self.obs_lo, self.obs_hi, _ptr(c))
        return c

    def row_ptr(self) -> np.ndarray:
        rp = np.zeros(self.n_stars + 1, dtype=np.int64)
        np.cumsum(self.star_counts(), out=rp[1:])
        return rp

    @property
    def n_rows(self) -> int:
        if self.obs_lo == self.obs_hi:
            return self.n_stars * self.obs_lo
        return int(self.star_counts().sum(dtype=np.int64))

    def dims(self) -> dict:
        return dict(n_rows=self.n_rows, n_stars=self.n_stars, n_dfa=self.n_dfa,
                    n_instr=self.n_instr, n_glob=1)


def rows(shape: Shape, r0: int, r1: int, *, star=True, att=True, instr=True, vals=True,
         row_ptr: np.ndarray | None = None) -> dict:
    """Arrays of rows [r0, r1): star[int32], att[int32], instr[int32 x6], vals[f64 x24]."""
    n = r1 - r0
    out = {}
    lib = _load()
    if star:
        rp = shape.row_ptr() if row_ptr is None else row_ptr
        s = np.empty(n, dtype=np.int32)
        lib.syn_star_of_rows(_ptr(rp), shape.n_stars, r0, r1, _ptr(s))
        out["star"] = s
    a = np.empty(n, dtype=np.int32) if att else None
    ins = np.empty(n * 6, dtype=np.int32) if instr else None
    v = np.empty(n * 24, dtype=np.float64) if vals else None
    lib.syn_rows(shape.seed, shape.n_dfa, shape.n_instr, r0, r1, _ptr(a), _ptr(ins), _ptr(v))
    if att:
        out["att"] = a
    if instr:
        out["instr"] = ins
    if vals:
        out["vals"] = v
    return out


def system(shape: Shape) -> dict:
    """The whole matrix of ``shape``: dict with star, att, instr, vals and dims."""
    rp = shape.row_ptr()
    m = int(rp[-1])
    out = rows(shape, 0, m, row_ptr=rp)
    out["dims"] = dict(n_rows=m, n_stars=shape.n_stars, n_dfa=shape.n_dfa,
                       n_instr=shape.n_instr, n_glob=1)
    out["row_ptr"] = rp
    return out


def normals(seed: int, stream: int, count: int, scale: float = 1.0, first: int = 0) -> np.ndarray:
    out = np.empty(count, dtype=np.float64)
    _load().syn_fill_normal(seed, stream, first, count, scale, _ptr(out))
    return out


def x_true(shape: Shape) -> np.ndarray:
    """Reference unknowns, N(0, 1) per column."""
    return normals(shape.seed, STREAM_XTRUE, shape.n_cols)


def noise(shape: Shape, n_rows: int | None = None) -> np.ndarray:
    """Observation noise, N(0, SIGMA_NOISE^2) per row."""
    m = shape.n_rows if n_rows is None else n_rows
    return normals(shape.seed, STREAM_NOISE, m, SIGMA_NOISE)


def x_ref(shape: Shape) -> np.ndarray:
    """Target of the loss ||x* - x_ref||^2 in the differentiation workload, N(0, 1)."""
    return normals(shape.seed, STREAM_XREF, shape.n_cols)


def rhs_x(shape: Shape, j: int) -> np.ndarray:
    """Unknowns of right-hand side j of a multi-RHS system, N(0, 1)."""
    return normals(shape.seed, STREAM_RHS_X + j, shape.n_cols)


def rhs_noise(shape: Shape, j: int, n_rows: int | None = None) -> np.ndarray:
    m = shape.n_rows if n_rows is None else n_rows
    return normals(shape.seed, STREAM_RHS_NOISE + j, m, SIGMA_NOISE)


def primary_stars(shape: Shape, frac: float) -> np.ndarray:
    """Stars selected (each with probability `frac`) for the constraint rows."""
    lib = _load()
    n = int(lib.syn_primary_stars(shape.seed, shape.n_stars, float(frac), None))
    out = np.empty(n, dtype=np.int32)
    if n:
        lib.syn_primary_stars(shape.seed, shape.n_stars, float(frac), _ptr(out))
    return out


def frame_constraints(shape: Shape, n_con: int = 6, frac: float = 0.1) -> dict:
    """Constraint rows shaped like the reference-frame conditions of a global astrometric
    solution: every row touches two astrometric unknowns of each selected ("primary") star
    -- slots 1, 2 (position-like) in the first half of the rows, slots 3, 4 (motion-like)
    in the second half -- with N(0, 1) coefficients.  Returns ptr [n_con+1] int64, col
    [nnz] int64 (absolute columns, ascending within a row), val [nnz] float64."""
    prim = primary_stars(shape, frac).astype(np.int64)
    per = 2 * prim.size
    ptr = np.arange(n_con + 1, dtype=np.int64) * per
    col = np.empty(n_con * per, dtype=np.int64)
    for k in range(n_con):
        a = 1 if k < (n_con + 1) // 2 else 3
        blk = col[k * per:(k + 1) * per].reshape(-1, 2)
        blk[:, 0] = 5 * prim + a
        blk[:, 1] = 5 * prim + a + 1
    val = normals(shape.seed, STREAM_CON_VALS, n_con * per)
    return dict(ptr=ptr, col=col, val=val)


# --- the workloads -----------------------------------------------------------------------

#: 1,000 stars x 60 obs, N_DFA 1,000, 500 instrumental columns (6.0e4 rows, 8,501 cols).
S1K_O60 = Shape(1000, 60, 60, 1000, 500, seed=1, name="stars1e3_obs60_dfa1e3_instr500")
#: 1e6 stars x 20 obs, N_DFA 30,000, 6,000 instrumental columns (2.0e7 rows, 5,096,001 cols).
S1M_O20 = Shape(1_000_000, 20, 20, 30_000, 6_000, seed=2, name="stars1e6_obs20_dfa3e4_instr6e3")
#: 5e6 stars x 40 obs, N_DFA 100,000, 10,000 instrumental columns (2.0e8 rows, 25,310,001 cols).
S5M_O40 = Shape(5_000_000, 40, 40, 100_000, 10_000, seed=3, name="stars5e6_obs40_dfa1e5_instr1e4")

#: one GPU's share of the 2e8-row system split over 8 GPUs by star-aligned row blocks:
#: 625,000 stars x 40 obs (2.5e7 rows) with the full attitude and instrumental widths.
S625K_O40 = Shape(625_000, 40, 40, 100_000, 10_000, seed=101,
                  name="stars625k_obs40_dfa1e5_instr1e4")

WORKLOADS = {s.name: s for s in (S1K_O60, S1M_O20, S5M_O40, S625K_O40)}


def batch_shapes(n_sys: int = 64, seed: int = 4, s_lo: float = 1e3, s_hi: float = 2e5,
                 obs_lo: int = 10, obs_hi: int = 60, n_instr: int = 500) -> list[Shape]:
    """Independent systems of the multi-system workload.

    Star counts log-uniform in [s_lo, s_hi] (drawn from stream STARS of ``seed``),
    obs_lo..obs_hi observations per star, N_DFA = n_stars // 10, n_instr
    instrumental columns; system k uses seed ``seed + k``.
    """
    lib = _load()
    key = lib.syn_key(seed, STREAM_STARS)
    out = []
    for k in range(n_sys):
        u = lib.syn_uniform(key, k)
        s = int(round(math.exp(math.log(s_lo) + u * (math.log(s_hi) - math.log(s_lo)))))
        out.append(Shape(s, obs_lo, obs_hi, max(4, s // 10), n_instr, seed=seed + k,
                         name=f"batch{k}_stars{s}"))
    return out
