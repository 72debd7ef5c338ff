"""Pins of the oracle's constraint equations against things other than itself.

Reading (Section 3: extra equations make the solution unique; Algorithms 1 and 2 end with
a "constraints computation" region): caller-given sparse rows C appended below the
observation rows, so the operator is the stacked [A; C] and the right-hand side [b; c].

- the stacked matrix built here with numpy from the rows' definition (products, column
  norms, adjoint identity), including repeated columns and an empty constraint row;
- a system that is rank deficient by construction (stars with fewer than five
  observations) made unique by constraint rows on those stars: dense least squares of the
  stacked matrix, and exact recovery of x_true from consistent data, which the
  unconstrained minimum-norm solution misses;
- scipy's LSQR on the stacked operator for the step-by-step PC-LSQR iterates;
- the residual correction reaching the binary64 constrained solution.
"""
import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

import oracle
import synth
from sparse_ref import csr, dense


def con_dense(con, n):
    """Dense C from the compressed rows (repeated columns add up)."""
    ptr, col, val = con["ptr"], con["col"], con["val"]
    C = np.zeros((len(ptr) - 1, n))
    for k in range(len(ptr) - 1):
        np.add.at(C[k], col[ptr[k]:ptr[k + 1]], val[ptr[k]:ptr[k + 1]])
    return C


def random_con(n, n_con, per_row, seed, empty_row=None, repeat=True):
    """Random constraint rows over all columns; optionally a row with no entries and a
    repeated column inside a row."""
    rng = np.random.default_rng(seed)
    counts = np.full(n_con, per_row)
    if empty_row is not None:
        counts[empty_row] = 0
    ptr = np.concatenate([[0], np.cumsum(counts)]).astype(np.int64)
    col = rng.integers(0, n, size=int(ptr[-1])).astype(np.int64)
    if repeat and ptr[-1] >= 2:
        col[1] = col[0]  # repeated column in the first non-empty row
    val = rng.standard_normal(int(ptr[-1]))
    return dict(ptr=ptr, col=col, val=val)


def _sys(shape, con):
    s = synth.system(shape)
    return s, oracle.System(s["dims"], s["vals"], s["star"], s["att"], s["instr"], con=con)


def test_products_colnorm_vs_stacked_dense():
    shape = synth.Shape(9, 10, 40, 12, 15, seed=31)
    n = shape.n_cols
    for con in (random_con(n, 5, 17, seed=1, empty_row=2),
                synth.frame_constraints(shape, n_con=6, frac=0.5)):
        s, S = _sys(shape, con)
        A = dense(s["dims"], s["vals"], s["star"], s["att"], s["instr"])
        B = np.vstack([A, con_dense(con, n)])
        assert S.m == B.shape[0] and S.n == n
        rng = np.random.default_rng(2)
        x, y0 = rng.standard_normal(n), rng.standard_normal(S.m)
        np.testing.assert_allclose(S.aprod1(x, y0), y0 + B @ x, rtol=1e-13, atol=1e-12)
        y, x0 = rng.standard_normal(S.m), rng.standard_normal(n)
        np.testing.assert_allclose(S.aprod2(y, x0), x0 + B.T @ y, rtol=1e-13, atol=1e-12)
        # column norms over the stored coefficients: the norm of the column of [A; C] when
        # no row repeats a column (the first constraint row here repeats one: there the
        # two stored coefficients count separately)
        ss = (dense(s["dims"], np.asarray(s["vals"]) ** 2, s["star"], s["att"], s["instr"])
              .sum(axis=0))
        np.add.at(ss, con["col"], con["val"] ** 2)
        p = S.colnorm()
        np.testing.assert_allclose(p[ss > 0], 1.0 / np.sqrt(ss[ss > 0]), rtol=1e-14)
        assert np.all(p[ss == 0] == 0.0)
        if len(np.unique(con["col"])) == len(con["col"]):
            cn = np.sqrt((B ** 2).sum(axis=0))
            np.testing.assert_allclose(p[cn > 0], 1.0 / cn[cn > 0], rtol=1e-14)
        # adjoint identity of the stacked operator
        lhs, rhs = S.aprod1(x) @ y, x @ S.aprod2(y)
        assert abs(lhs - rhs) <= 1e-13 * np.linalg.norm(S.aprod1(x)) * np.linalg.norm(y)


def test_residual_over_constraint_rows():
    shape = synth.Shape(6, 8, 20, 9, 11, seed=32)
    con = random_con(shape.n_cols, 4, 9, seed=3)
    s, S = _sys(shape, con)
    B = np.vstack([dense(s["dims"], s["vals"], s["star"], s["att"], s["instr"]),
                   con_dense(con, shape.n_cols)])
    rng = np.random.default_rng(4)
    b, x = rng.standard_normal(S.m), rng.standard_normal(S.n)
    np.testing.assert_allclose(S.residual(b, x), b - B @ x, rtol=1e-13, atol=1e-12)


def _deficient_system(seed=33):
    """Stars with 2..9 observations: every star with fewer than five observations leaves its
    astrometric block rank deficient.  One constraint row per missing rank on each such star,
    over its five astrometric columns (N(0, 1) coefficients)."""
    shape = synth.Shape(24, 2, 9, 6, 8, seed=seed)
    counts = shape.star_counts()
    deficient = np.nonzero(counts < 5)[0]
    rng = np.random.default_rng(seed)
    ptr, col = [0], []
    for st in deficient:
        for _ in range(5 - int(counts[st])):
            col.extend(5 * int(st) + np.arange(5))
            ptr.append(len(col))
    con = dict(ptr=np.array(ptr, dtype=np.int64), col=np.array(col, dtype=np.int64),
               val=rng.standard_normal(len(col)))
    return shape, deficient, con


def test_rank_deficient_system_made_unique():
    shape, deficient, con = _deficient_system()
    assert deficient.size >= 3
    s, S = _sys(shape, con)
    n = shape.n_cols
    A = dense(s["dims"], s["vals"], s["star"], s["att"], s["instr"])
    C = con_dense(con, n)
    B = np.vstack([A, C])
    assert np.linalg.matrix_rank(A) < n
    assert np.linalg.matrix_rank(B) == n
    xt = synth.x_true(shape)
    # consistent data: the constrained solution is x_true itself
    bc = B @ xt
    x, info = S.lsqr(bc, itnlim=5000, fixed=False, atol=1e-15, btol=1e-15)
    assert np.linalg.norm(x - xt) <= 1e-9 * np.linalg.norm(xt)
    # ... which the unconstrained minimum-norm solution of the same observations misses
    S0 = oracle.System(s["dims"], s["vals"], s["star"], s["att"], s["instr"])
    x0, _ = S0.lsqr(A @ xt, itnlim=5000, fixed=False, atol=1e-15, btol=1e-15)
    assert np.linalg.norm(x0 - xt) >= 1e-3 * np.linalg.norm(xt)
    # noisy observations, zero constraint right-hand side: dense least squares
    rng = np.random.default_rng(5)
    bn = np.concatenate([A @ xt + 1e-3 * rng.standard_normal(A.shape[0]), np.zeros(C.shape[0])])
    x, _ = S.lsqr(bn, itnlim=5000, fixed=False, atol=1e-15, btol=1e-15)
    xd = np.linalg.lstsq(B, bn, rcond=None)[0]
    assert np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)


def test_pclsqr_iterates_with_constraints_match_scipy():
    shape = synth.S1K_O60
    con = synth.frame_constraints(shape, n_con=6, frac=0.1)
    s, S = _sys(shape, con)
    n = shape.n_cols
    ptr, col, val = con["ptr"], con["col"], con["val"]
    rows = np.repeat(np.arange(len(ptr) - 1), np.diff(ptr))
    C = sp.csr_matrix((val, (rows, col)), shape=(len(ptr) - 1, n))
    B = sp.vstack([csr(s["dims"], s["vals"], s["star"], s["att"], s["instr"]), C]).tocsr()
    rng = np.random.default_rng(6)
    b = B @ synth.x_true(shape) + 1e-3 * rng.standard_normal(B.shape[0])
    p = S.colnorm()
    cn = np.sqrt(np.asarray(B.multiply(B).sum(axis=0)).ravel())
    np.testing.assert_allclose(p, 1.0 / cn, rtol=1e-14)
    Bp = spla.LinearOperator(B.shape, matvec=lambda z: B @ (p * z),
                             rmatvec=lambda y: p * (B.T @ y), dtype=np.float64)
    for k in (1, 2, 5, 10, 20):
        x, info = S.lsqr(b, itnlim=k, fixed=True)
        xs = p * spla.lsqr(Bp, b, atol=0.0, btol=0.0, conlim=0.0, iter_lim=k)[0]
        assert np.linalg.norm(x - xs) <= 1e-11 * np.linalg.norm(xs), k
        assert info["itn"] == k


def test_refine_with_constraints_reaches_fp64_solution():
    shape, deficient, con = _deficient_system(seed=34)
    s, S = _sys(shape, con)
    rng = np.random.default_rng(7)
    A = dense(s["dims"], s["vals"], s["star"], s["att"], s["instr"])
    b = np.concatenate([A @ synth.x_true(shape) + 1e-3 * rng.standard_normal(A.shape[0]),
                        np.zeros(S.n_con)])
    x64, _ = S.lsqr(b, itnlim=5000, fixed=False, atol=1e-15, btol=1e-15)
    lo = s["vals"].astype(np.float32)
    xr, outer, _ = S.refine(b, lo, max_outer=8, refine_tol=1e-12, inner_itnlim=5000,
                            inner_atol=1e-14, inner_btol=1e-14)
    assert outer >= 2
    assert np.linalg.norm(xr - x64) <= 1e-9 * np.linalg.norm(x64)
