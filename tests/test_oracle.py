"""Pins of the oracle against things other than itself.

- a hand-worked placement of the 24 coefficients (tests/golden/tiny_structure.txt);
- an independent scipy.sparse construction from the Section 3 description;
- scipy.sparse.linalg.lsqr (a library implementation of Paige & Saunders' LSQR) for
  the step-by-step iterates of PC-LSQR and its variance estimate;
- diag((A^T A)^-1) for the variance estimate after a full Krylov space;
- dense least squares / normal equations for converged solutions;
- invariants: adjoint identity, exact recovery of x_true, monotone residual,
  finite termination, preconditioner invariance of the converged solution;
- closed-form and finite-difference gradients for the adjoint.
"""
import os

import numpy as np
import pytest
import scipy.sparse.linalg as spla

import oracle
import synth
from sparse_ref import column_table, csr, dense, n_cols

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "tiny_structure.txt")


def _system(shape):
    s = synth.system(shape)
    return s, oracle.System(s["dims"], s["vals"], s["star"], s["att"], s["instr"])


def _load_golden():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        head, ins, cols = line.split("|")
        i, star, t = map(int, head.split())
        rows.append((i, star, t, list(map(int, ins.split())), list(map(int, cols.split()))))
    return rows


def test_golden_structure():
    g = _load_golden()
    dims = dict(n_rows=len(g), n_stars=2, n_dfa=5, n_instr=7, n_glob=1)
    star = np.array([r[1] for r in g], dtype=np.int32)
    att = np.array([r[2] for r in g], dtype=np.int32)
    instr = np.array([r[3] for r in g], dtype=np.int32).ravel()
    hand_cols = np.array([r[4] for r in g])
    assert hand_cols.shape == (len(g), 24)
    # the tests' own sparse builder agrees with the hand-worked placement
    assert np.array_equal(column_table(dims, star, att, instr), hand_cols)
    vals = np.array([[100.0 * (i + 1) + k for k in range(24)] for i in range(len(g))]).ravel()
    Ad = np.zeros((len(g), 33))
    for i in range(len(g)):
        for k in range(24):
            Ad[i, hand_cols[i, k]] += vals[24 * i + k]
    S = oracle.System(dims, vals, star, att, instr)
    assert S.n == 33
    rng = np.random.default_rng(0)
    x = rng.standard_normal(33)
    y0 = rng.standard_normal(len(g))
    np.testing.assert_allclose(S.aprod1(x, y0), y0 + Ad @ x, rtol=1e-13, atol=1e-11)
    y = rng.standard_normal(len(g))
    x0 = rng.standard_normal(33)
    np.testing.assert_allclose(S.aprod2(y, x0), x0 + Ad.T @ y, rtol=1e-13, atol=1e-11)
    cn = np.sqrt((Ad ** 2).sum(axis=0))
    p = S.colnorm()
    np.testing.assert_allclose(p[cn > 0], 1.0 / cn[cn > 0], rtol=1e-15)
    assert np.all(p[cn == 0] == 0.0)


@pytest.mark.parametrize("shape", [synth.Shape(3, 30, 30, 6, 8, seed=5),
                                   synth.Shape(7, 10, 60, 9, 13, seed=6),
                                   synth.Shape(1, 50, 50, 4, 6, seed=7)])
def test_aprod_vs_dense(shape):
    s, S = _system(shape)
    A = dense(s["dims"], s["vals"], s["star"], s["att"], s["instr"])
    rng = np.random.default_rng(1)
    x = rng.standard_normal(S.n)
    y0 = rng.standard_normal(S.m)
    np.testing.assert_allclose(S.aprod1(x, y0), y0 + A @ x, rtol=1e-13, atol=1e-13)
    y = rng.standard_normal(S.m)
    x0 = rng.standard_normal(S.n)
    np.testing.assert_allclose(S.aprod2(y, x0), x0 + A.T @ y, rtol=1e-13, atol=1e-13)


def test_aprod_small_workload_vs_scipy_and_adjoint():
    s, S = _system(synth.S1K_O60)
    A = csr(s["dims"], s["vals"], s["star"], s["att"], s["instr"])
    rng = np.random.default_rng(2)
    x = rng.standard_normal(S.n)
    y = rng.standard_normal(S.m)
    Ax = S.aprod1(x)
    Aty = S.aprod2(y)
    np.testing.assert_allclose(Ax, A @ x, rtol=1e-12, atol=1e-12 * np.abs(Ax).max())
    np.testing.assert_allclose(Aty, A.T @ y, rtol=1e-12, atol=1e-12 * np.abs(Aty).max())
    # adjoint identity <Ax, y> = <x, A^T y>
    lhs, rhs = Ax @ y, x @ Aty
    assert abs(lhs - rhs) <= 1e-12 * np.linalg.norm(Ax) * np.linalg.norm(y)


def test_colnorm_vs_scipy_and_empty_column():
    shape = synth.Shape(5, 12, 12, 8, 200, seed=8)  # 60 rows x 6 draws from 200: some unused
    s, S = _system(shape)
    A = csr(s["dims"], s["vals"], s["star"], s["att"], s["instr"])
    cn = np.sqrt(np.asarray(A.multiply(A).sum(axis=0)).ravel())
    p = S.colnorm()
    assert np.any(cn == 0)
    np.testing.assert_allclose(p[cn > 0], 1.0 / cn[cn > 0], rtol=1e-14)
    assert np.all(p[cn == 0] == 0)


def _scipy_pclsqr_iterate(A, p, b, k):
    """k iterations of scipy's LSQR on A diag(p), mapped back by p."""
    Ab = spla.LinearOperator(A.shape, matvec=lambda z: A @ (p * z), rmatvec=lambda y: p * (A.T @ y),
                             dtype=np.float64)
    z = spla.lsqr(Ab, b, atol=0.0, btol=0.0, conlim=0.0, iter_lim=k)[0]
    return p * z


@pytest.mark.parametrize("shape,ks", [
    (synth.Shape(4, 30, 30, 7, 9, seed=9), [1, 2, 3, 5, 8, 13]),
    (synth.S1K_O60, [1, 2, 5, 10, 20]),
])
def test_lsqr_iterates_match_scipy_lsqr(shape, ks):
    s, S = _system(shape)
    A = csr(s["dims"], s["vals"], s["star"], s["att"], s["instr"])
    xt = synth.x_true(shape)
    b = A @ xt + synth.noise(shape)
    p = S.colnorm()
    for k in ks:
        x, info = S.lsqr(b, itnlim=k, fixed=True)
        assert info["itn"] == k
        xs = _scipy_pclsqr_iterate(A, p, b, k)
        assert np.linalg.norm(x - xs) <= 1e-11 * np.linalg.norm(xs), k


@pytest.mark.parametrize("shape,ks", [
    (synth.Shape(4, 30, 30, 7, 9, seed=9), [1, 2, 3, 5, 8, 13]),
    (synth.S1K_O60, [1, 2, 5, 20]),
])
def test_variance_estimate_matches_scipy_lsqr(shape, ks):
    """Variance estimate: scipy's LSQR (calc_var) on A diag(p) gives the preconditioned sum of
    (w_i / rho_i)^2 step by step; the oracle returns it times p^2."""
    s, S = _system(shape)
    A = csr(s["dims"], s["vals"], s["star"], s["att"], s["instr"])
    b = A @ synth.x_true(shape) + synth.noise(shape)
    p = S.colnorm()
    Ab = spla.LinearOperator(A.shape, matvec=lambda z: A @ (p * z),
                             rmatvec=lambda y: p * (A.T @ y), dtype=np.float64)
    for k in ks:
        x, var, info = S.lsqr_var(b, itnlim=k, fixed=True)
        res = spla.lsqr(Ab, b, atol=0.0, btol=0.0, conlim=0.0, iter_lim=k, calc_var=True)
        vs = p * p * res[-1]
        assert np.linalg.norm(var - vs) <= 1e-11 * np.linalg.norm(vs), k
        x0, _ = S.lsqr(b, itnlim=k, fixed=True)
        assert np.array_equal(x, x0)  # the estimate does not change the iterate


def test_variance_estimate_exact_after_n_steps():
    """After exactly n steps (full Krylov space) the estimate is diag((A^T A)^-1) up to rounding
    and loss of orthogonality; 29 unknowns."""
    shape = synth.Shape(2, 30, 30, 4, 6, seed=93)
    s, S = _system(shape)
    A = dense(s["dims"], s["vals"], s["star"], s["att"], s["instr"])
    assert S.n == 29
    b = A @ synth.x_true(shape) + synth.noise(shape)
    x, var, info = S.lsqr_var(b, itnlim=S.n, fixed=True)
    ref = np.diag(np.linalg.inv(A.T @ A))
    assert np.max(np.abs(var - ref) / ref) <= 1e-3
    # far from complete after a third of the steps: the sum only grows towards the diagonal
    _, var10, _ = S.lsqr_var(b, itnlim=10, fixed=True)
    assert np.all(var10 <= ref * (1 + 1e-9)) and np.max(np.abs(var10 - ref) / ref) > 0.1


# scipy numbers the stopping reasons 1 compatible, 2 least squares, 3 conlim, 4/5/6 the same
# three at machine precision; the oracle keeps 3/4 for an exact breakdown and a zero b
_SCIPY_ISTOP = {1: 1, 2: 2, 3: 5, 4: 6, 5: 7, 6: 8}


@pytest.mark.parametrize("shape", [synth.Shape(40, 10, 60, 30, 40, seed=23),
                                   synth.Shape(4, 25, 40, 6, 10, seed=10)])
@pytest.mark.parametrize("noise", [True, False])
@pytest.mark.parametrize("atol,btol,conlim", [(0.0, 0.0, 0.0), (1e-8, 1e-8, 0.0),
                                              (0.0, 0.0, 30.0), (1e-14, 1e-14, 0.0)])
def test_stopping_rules_match_scipy_lsqr(shape, noise, atol, btol, conlim):
    """Every Paige & Saunders stopping test (tolerances, condition limit, machine precision):
    the same step and the same reason as scipy's LSQR on A diag(p), and the same condition
    estimate."""
    s, S = _system(shape)
    A = csr(s["dims"], s["vals"], s["star"], s["att"], s["instr"])
    b = A @ synth.x_true(shape) + (synth.noise(shape) if noise else 0.0)
    p = S.colnorm()
    Ab = spla.LinearOperator(A.shape, matvec=lambda z: A @ (p * z),
                             rmatvec=lambda y: p * (A.T @ y), dtype=np.float64)
    x, info = S.lsqr(b, itnlim=2000, fixed=False, atol=atol, btol=btol, conlim=conlim)
    res = spla.lsqr(Ab, b, atol=atol, btol=btol, conlim=conlim if conlim > 0 else 1e300,
                    iter_lim=2000)
    assert info["itn"] == res[2]
    assert info["istop"] == _SCIPY_ISTOP[res[1]]
    assert abs(info["acond"] - res[6]) <= 1e-3 * res[6]
    assert np.linalg.norm(x - p * res[0]) <= 1e-8 * np.linalg.norm(x)


def test_condition_estimate_after_n_steps():
    """acond = ||B|| (sum ||w_i / rho_i||^2)^(1/2) is ||B||_F ||B^+||_F once the Krylov space is
    complete (B = A D, 29 unknowns), and grows towards it."""
    shape = synth.Shape(2, 30, 30, 4, 6, seed=93)
    s, S = _system(shape)
    A = dense(s["dims"], s["vals"], s["star"], s["att"], s["instr"])
    p = S.colnorm()
    B = A * p
    sv = np.linalg.svd(B, compute_uv=False)
    ref = np.sqrt((sv ** 2).sum()) * np.sqrt((sv ** -2.0).sum())
    b = A @ synth.x_true(shape) + synth.noise(shape)
    _, info = S.lsqr(b, itnlim=S.n, fixed=True)
    assert abs(info["acond"] - ref) <= 1e-3 * ref
    _, info10 = S.lsqr(b, itnlim=10, fixed=True)
    assert info10["acond"] < 0.9 * ref
    # a condition limit below the estimate stops at the first step that exceeds it
    _, ic = S.lsqr(b, itnlim=S.n, fixed=False, atol=0.0, btol=0.0, conlim=info10["acond"])
    assert ic["istop"] == 5 and ic["itn"] <= 10 and ic["acond"] >= info10["acond"] * (1 - 1e-12)


def test_lsqr_converged_vs_lstsq_and_precond_invariance():
    shape = synth.Shape(4, 25, 40, 6, 10, seed=10)
    s, S = _system(shape)
    A = dense(s["dims"], s["vals"], s["star"], s["att"], s["instr"])
    rng = np.random.default_rng(3)
    b = rng.standard_normal(S.m)
    x_ls = np.linalg.lstsq(A, b, rcond=None)[0]
    x_pc, info = S.lsqr(b, itnlim=2000, fixed=False, atol=1e-15, btol=1e-15)
    assert info["istop"] in (1, 2, 3)
    assert np.linalg.norm(x_pc - x_ls) <= 1e-11 * np.linalg.norm(x_ls)
    x_pl, _ = S.lsqr(b, itnlim=5000, fixed=False, atol=1e-15, btol=1e-15, precond=False)
    assert np.linalg.norm(x_pl - x_ls) <= 1e-10 * np.linalg.norm(x_ls)
    # rnorm estimate at convergence equals the true least-squares residual
    assert abs(info["rnorm"] - np.linalg.norm(b - A @ x_ls)) <= 1e-10 * np.linalg.norm(b)


def test_x_true_recovery_noiseless():
    shape = synth.S1K_O60
    s, S = _system(shape)
    xt = synth.x_true(shape)
    b = S.aprod1(xt)
    x, info = S.lsqr(b, itnlim=100, fixed=True)
    assert np.linalg.norm(x - xt) <= 1e-13 * np.linalg.norm(xt)


def test_residual_estimate_and_monotone():
    shape = synth.Shape(50, 20, 20, 30, 40, seed=12)
    s, S = _system(shape)
    A = csr(s["dims"], s["vals"], s["star"], s["att"], s["instr"])
    b = A @ synth.x_true(shape) + 0.1 * synth.noise(shape) * 1e3
    _, _, hist = S.lsqr(b, itnlim=40, fixed=True, hist=True)
    assert np.all(np.diff(hist) <= 1e-12 * hist[0])
    for k in (1, 3, 10, 40):
        x, info = S.lsqr(b, itnlim=k, fixed=True)
        direct = np.linalg.norm(b - A @ x)
        assert abs(info["rnorm"] - direct) <= 1e-10 * np.linalg.norm(b), k
        assert abs(hist[k - 1] - direct) <= 1e-10 * np.linalg.norm(b), k
        # ||A_bar^T r|| estimate
        p = S.colnorm()
        ar = np.linalg.norm(p * (A.T @ (b - A @ x)))
        assert abs(info["arnorm"] - ar) <= 1e-8 * max(ar, 1e-300) + 1e-12 * np.linalg.norm(b)


def test_finite_termination():
    # one star: n = 5 + 12 + 6 + 1 = 24 columns, 40 rows; exact arithmetic ends in <= n steps
    shape = synth.Shape(1, 40, 40, 4, 6, seed=13)
    s, S = _system(shape)
    A = dense(s["dims"], s["vals"], s["star"], s["att"], s["instr"])
    assert S.n == 24
    b = np.random.default_rng(4).standard_normal(S.m)
    x_ls = np.linalg.lstsq(A, b, rcond=None)[0]
    # in floating point the termination is delayed by a few steps (loss of orthogonality)
    err = {k: np.linalg.norm(S.lsqr(b, itnlim=k, fixed=True)[0] - x_ls) / np.linalg.norm(x_ls)
           for k in (S.n // 2, S.n, S.n + 6)}
    assert err[S.n // 2] > 1e-3
    assert err[S.n] < 1e-6
    assert err[S.n + 6] < 1e-13


def test_zero_rhs_and_empty_columns():
    shape = synth.Shape(6, 30, 30, 8, 12, seed=8)
    s, S = _system(shape)
    x, info = S.lsqr(np.zeros(S.m), itnlim=10, fixed=True)
    assert info["istop"] == 4 and np.all(x == 0)
    # make two columns numerically empty: an instrumental one and an astrometric one
    cols = column_table(s["dims"], s["star"], s["att"], s["instr"])
    dead = [5 * 6 + 3 * 8 + 5, 5 * 2 + 3]
    vals = s["vals"].reshape(-1, 24).copy()
    vals[np.isin(cols, dead)] = 0.0
    S = S.with_vals(vals.ravel())
    A = dense(s["dims"], vals.ravel(), s["star"], s["att"], s["instr"])
    used = np.abs(A).sum(axis=0) > 0
    assert (~used).sum() == 2 and A.shape[0] > used.sum()
    assert np.all(S.colnorm()[~used] == 0)
    b = np.random.default_rng(5).standard_normal(S.m)
    x_ls = np.linalg.lstsq(A[:, used], b, rcond=None)[0]
    x, info = S.lsqr(b, itnlim=3000, fixed=False, atol=1e-15, btol=1e-15)
    assert np.all(x[~used] == 0)
    assert np.linalg.norm(x[used] - x_ls) <= 1e-11 * np.linalg.norm(x_ls)


def test_row_permutation_invariance():
    shape = synth.Shape(20, 15, 15, 12, 20, seed=14)
    s, S = _system(shape)
    b = np.random.default_rng(6).standard_normal(S.m)
    x1, _ = S.lsqr(b, itnlim=500, fixed=False, atol=1e-15, btol=1e-15)
    perm = np.random.default_rng(7).permutation(S.m)
    P = oracle.System(s["dims"], s["vals"].reshape(-1, 24)[perm].ravel(), s["star"][perm],
                      s["att"][perm], s["instr"].reshape(-1, 6)[perm].ravel())
    x2, _ = P.lsqr(b[perm], itnlim=500, fixed=False, atol=1e-15, btol=1e-15)
    assert np.linalg.norm(x1 - x2) <= 1e-12 * np.linalg.norm(x1)


# ---- mixed precision -------------------------------------------------------------------

def test_refine_reaches_fp64_solution():
    shape = synth.S1K_O60
    s, S = _system(shape)
    xt = synth.x_true(shape)
    b = S.aprod1(xt) + synth.noise(shape)
    x64, _ = S.lsqr(b, itnlim=300, fixed=False, atol=1e-15, btol=1e-15)
    lo = s["vals"].astype(np.float32)
    # before refinement: the FP32-coefficient solution is ~1e-8 away
    S32 = S.with_vals(lo.astype(np.float64))
    x32, _ = S32.lsqr(b, itnlim=300, fixed=False, atol=1e-15, btol=1e-15)
    pre = np.linalg.norm(x32 - x64) / np.linalg.norm(x64)
    assert 1e-10 < pre < 1e-6
    xr, outer, inner = S.refine(b, lo, max_outer=6, refine_tol=1e-10, inner_itnlim=300,
                                inner_atol=1e-12, inner_btol=1e-12)
    assert outer >= 2
    assert np.linalg.norm(xr - x64) <= 1e-9 * np.linalg.norm(x64)
    # noiseless: refinement recovers x_true
    b0 = S.aprod1(xt)
    xr0, _, _ = S.refine(b0, lo, max_outer=8, refine_tol=1e-13, inner_itnlim=300,
                         inner_atol=1e-12, inner_btol=1e-12)
    assert np.linalg.norm(xr0 - xt) <= 1e-12 * np.linalg.norm(xt)


def test_refine_schedule_with_short_correction_solves():
    """A first inner solve of k1 steps, then correction solves of k2 steps: the composition
    written out with scipy's sparse residual, and the binary64 solution reached with short
    corrections."""
    shape = synth.S1K_O60
    s, S = _system(shape)
    A = csr(s["dims"], s["vals"], s["star"], s["att"], s["instr"])
    b = A @ synth.x_true(shape) + synth.noise(shape)
    lo = s["vals"].astype(np.float32)
    S32 = S.with_vals(lo.astype(np.float64))
    x1, _ = S32.lsqr(b, itnlim=30, fixed=True)
    d1, _ = S32.lsqr(b - A @ x1, itnlim=6, fixed=True)
    xr, outer, inner = S.refine(b, lo, max_outer=2, refine_tol=0.0, inner_itnlim=30,
                                later_itnlim=6, inner_fixed=True)
    assert (outer, inner) == (2, [30, 6])
    assert np.linalg.norm(xr - (x1 + d1)) <= 1e-13 * np.linalg.norm(xr)
    x64, _ = S.lsqr(b, itnlim=300, fixed=False, atol=1e-15, btol=1e-15)
    xr, outer, inner = S.refine(b, lo, max_outer=3, refine_tol=0.0, inner_itnlim=300,
                                later_itnlim=12, inner_atol=1e-12, inner_btol=1e-12)
    assert inner[0] > 12 and all(k <= 12 for k in inner[1:])
    assert np.linalg.norm(xr - x64) <= 1e-9 * np.linalg.norm(x64)


def test_refine_with_loose_first_solve():
    """A first inner solve stopped at a loose tolerance, then correction solves at the final
    one: the composition written out with scipy's sparse residual, and the binary64 solution
    reached."""
    shape = synth.S1K_O60
    s, S = _system(shape)
    A = csr(s["dims"], s["vals"], s["star"], s["att"], s["instr"])
    b = A @ synth.x_true(shape) + synth.noise(shape)
    lo = s["vals"].astype(np.float32)
    S32 = S.with_vals(lo.astype(np.float64))
    x1, i1 = S32.lsqr(b, itnlim=300, fixed=False, atol=1e-4, btol=1e-4)
    d1, i2 = S32.lsqr(b - A @ x1, itnlim=300, fixed=False, atol=1e-12, btol=1e-12)
    xr, outer, inner = S.refine(b, lo, max_outer=2, refine_tol=0.0, inner_itnlim=300,
                                inner_atol=1e-12, inner_btol=1e-12, first_tol=1e-4)
    assert (outer, inner) == (2, [i1["itn"], i2["itn"]])
    assert i1["itn"] < i2["itn"]
    assert np.linalg.norm(xr - (x1 + d1)) <= 1e-13 * np.linalg.norm(xr)
    x64, _ = S.lsqr(b, itnlim=300, fixed=False, atol=1e-15, btol=1e-15)
    assert np.linalg.norm(xr - x64) <= 1e-9 * np.linalg.norm(x64)


def test_refine_with_exact_low_precision_is_one_solve():
    shape = synth.Shape(10, 20, 20, 10, 12, seed=15)
    s, S = _system(shape)
    vals = s["vals"].astype(np.float32).astype(np.float64)  # exactly representable
    S = S.with_vals(vals)
    b = np.random.default_rng(8).standard_normal(S.m)
    x1, _ = S.lsqr(b, itnlim=40, fixed=True)
    xr, outer, inner = S.refine(b, vals.astype(np.float32), max_outer=1, inner_itnlim=40,
                                inner_fixed=True)
    assert outer == 1 and inner == [40]
    assert np.array_equal(x1, xr)


# ---- differentiation -------------------------------------------------------------------

def _dense_grad(A, b, xr):
    """Closed form: x* = (A^T A)^-1 A^T b, L = ||x* - xr||^2, g = 2 (x* - xr),
    lam = (A^T A)^-1 g, mu = A lam, dL/db = mu, dL/dA = r lam^T - mu x*^T."""
    N = A.T @ A
    x = np.linalg.solve(N, A.T @ b)
    g = 2 * (x - xr)
    lam = np.linalg.solve(N, g)
    mu = A @ lam
    r = b - A @ x
    return x, g, mu, lam, np.outer(r, lam) - np.outer(mu, x)


def test_adjoint_gradient_vs_dense_closed_form():
    shape = synth.Shape(6, 20, 30, 8, 12, seed=16)
    s, S = _system(shape)
    A = dense(s["dims"], s["vals"], s["star"], s["att"], s["instr"])
    b = A @ synth.x_true(shape) + synth.noise(shape)
    xr = synth.x_ref(shape)
    x, g, mu, lam, dA = _dense_grad(A, b, xr)
    out = S.solve_and_grad(b, 2 * (S.lsqr(b, itnlim=3000, fixed=False, atol=1e-15,
                                            btol=1e-15)[0] - xr))
    assert np.linalg.norm(out["x"] - x) <= 1e-12 * np.linalg.norm(x)
    assert np.linalg.norm(out["mu"] - mu) <= 1e-10 * np.linalg.norm(mu)
    assert np.linalg.norm(out["lam"] - lam) <= 1e-10 * np.linalg.norm(lam)
    cols = column_table(s["dims"], s["star"], s["att"], s["instr"])
    dvals_ref = dA[np.arange(S.m)[:, None], cols].ravel()
    assert np.linalg.norm(out["dvals"] - dvals_ref) <= 1e-10 * np.linalg.norm(dvals_ref)
    # mu is the minimum-norm solution of A^T mu = g: it lies in range(A)
    np.testing.assert_allclose(A.T @ out["mu"], g, rtol=0, atol=1e-10 * np.linalg.norm(g))


def test_adjoint_gradient_vs_finite_differences():
    shape = synth.Shape(5, 20, 20, 8, 10, seed=17)
    s, S = _system(shape)
    A = csr(s["dims"], s["vals"], s["star"], s["att"], s["instr"])
    b = A @ synth.x_true(shape) + synth.noise(shape)
    xr = synth.x_ref(shape)

    def solve(vals, bb):
        T = S.with_vals(vals)
        return T.lsqr(bb, itnlim=3000, fixed=False, atol=1e-16, btol=1e-16)[0]

    x = solve(s["vals"], b)
    out = S.solve_and_grad(b, 2 * (x - xr))
    rng = np.random.default_rng(9)
    h = 1e-6
    # directional derivative along random +-1 directions, L(+) - L(-) written without
    # cancellation as sum (x+ - x-)(x+ + x- - 2 xr)
    eb = rng.choice([-1.0, 1.0], size=S.m)
    xp, xm = solve(s["vals"], b + h * eb), solve(s["vals"], b - h * eb)
    fd = np.sum((xp - xm) * (xp + xm - 2 * xr)) / (2 * h)
    an = out["mu"] @ eb
    assert abs(fd - an) <= 1e-6 * abs(an)
    ev = rng.choice([-1.0, 1.0], size=24 * S.m)
    xp, xm = solve(s["vals"] + h * ev, b), solve(s["vals"] - h * ev, b)
    fd = np.sum((xp - xm) * (xp + xm - 2 * xr)) / (2 * h)
    an = out["dvals"] @ ev
    assert abs(fd - an) <= 1e-6 * abs(an)
