"""Constraint equations on the GPU (gsr_set_constraints) against the oracle, through the C ABI.

The operator is the stacked [A; C] (C: caller-given sparse rows below the observation rows),
the reading the oracle takes of Section 3's extra equations and of the constraints
computation that closes Algorithms 1 and 2.  Products, preconditioner and residual are
compared elementwise (1e-13 of the largest entry); PC-LSQR iterates to 1e-10 relative
(binary64), the refined precision form to 1e-8; fused and unfused row passes both.
"""
import numpy as np
import pytest
import torch

import synth
from gpu_util import assert_close_scaled, cuda, host, open_system, rel
from paper_2212_11675_amd import gsr
from test_oracle_constraints import _deficient_system, con_dense, random_con

import oracle

pytestmark = pytest.mark.gpu

FUSED = synth.Shape(300, 10, 60, 40, 50, seed=141, name="fused")
UNFUSED = synth.Shape(200, 10, 40, 30, 10600, seed=142, name="unfused_instr10600")


def con_dev(con):
    return (torch.from_numpy(np.ascontiguousarray(con["ptr"], dtype=np.int64)).to("cuda"),
            torch.from_numpy(np.ascontiguousarray(con["col"], dtype=np.int64)).to("cuda"),
            torch.from_numpy(np.ascontiguousarray(con["val"], dtype=np.float64)).to("cuda"))


def setup(shape, con, **kw):
    sysd = synth.system(shape)
    S = oracle.System(sysd["dims"], sysd["vals"], sysd["star"], sysd["att"], sysd["instr"],
                      con=con)
    h, t = open_system(sysd, allow_empty_cols=True, **kw)
    cd = con_dev(con)
    gsr.gsr_set_constraints(h, *cd)
    assert h.m == S.m == sysd["dims"]["n_rows"] + len(con["ptr"]) - 1
    return sysd, S, h, (t, cd)


def cons_for(shape):
    n = shape.n_cols
    return [random_con(n, 7, 23, seed=shape.seed, empty_row=3),
            synth.frame_constraints(shape, n_con=6, frac=0.3),
            random_con(n, 300, 2, seed=shape.seed + 1)]  # many short rows


@pytest.mark.parametrize("shape", [FUSED, UNFUSED], ids=lambda s: s.name)
def test_products_preconditioner_residual_with_constraints(shape):
    for ci, con in enumerate(cons_for(shape)):
        print(f"[con products] {shape.name} constraint set {ci}", flush=True)
        sysd, S, h, keep = setup(shape, con, build_f32=True)
        rng = np.random.default_rng(ci)
        x, y0 = rng.standard_normal(S.n), rng.standard_normal(S.m)
        yd = cuda(y0)
        gsr.gsr_aprod1(h, cuda(x), yd)
        assert_close_scaled(host(yd), S.aprod1(x, y0), 1e-13)
        y, x0 = rng.standard_normal(S.m), rng.standard_normal(S.n)
        xd = cuda(x0)
        gsr.gsr_aprod2(h, cuda(y), xd)
        assert_close_scaled(host(xd), S.aprod2(y, x0), 1e-13)
        p = torch.empty(S.n, dtype=torch.float64, device="cuda")
        gsr.gsr_precond(h, p)
        np.testing.assert_allclose(host(p), S.colnorm(), rtol=1e-12, atol=0)
        # binary32 observation coefficients, binary64 constraint rows
        S32 = S.with_vals(sysd["vals"].astype(np.float32).astype(np.float64))
        yd = cuda(y0)
        gsr.gsr_aprod1_f32v(h, cuda(x), yd)
        assert_close_scaled(host(yd), S32.aprod1(x, y0), 1e-13)
        xd = cuda(x0)
        gsr.gsr_aprod2_f32v(h, cuda(y), xd)
        assert_close_scaled(host(xd), S32.aprod2(y, x0), 1e-13)
        gsr.gsr_precond(h, p, precision=gsr.GSR_F32V)
        np.testing.assert_allclose(host(p), S32.colnorm(), rtol=1e-12, atol=0)
        b = rng.standard_normal(S.m)
        r = torch.empty(S.m, dtype=torch.float64, device="cuda")
        gsr.gsr_residual(h, cuda(b), cuda(x), r)
        assert_close_scaled(host(r), S.residual(b, x), 1e-13)
        h.close()


@pytest.mark.parametrize("shape", [FUSED, UNFUSED], ids=lambda s: s.name)
def test_pclsqr_iterates_with_constraints(shape):
    con = synth.frame_constraints(shape, n_con=6, frac=0.3)
    sysd, S, h, keep = setup(shape, con)
    rng = np.random.default_rng(5)
    b = S.aprod1(synth.x_true(shape)) + 1e-3 * rng.standard_normal(S.m)
    # Step by step up to 10 steps.  The six frame rows put a few singular values of A D far
    # above the rest; once the recurrence has found them it amplifies rounding (Lanczos
    # vectors lose orthogonality): the oracle's own iterate moves by 2e-11 at 20 steps and
    # 3e-8 at 40 when one entry of b changes by one ulp (1e-16 without the rows).  Past that
    # the converged solutions are compared.
    for k in (1, 2, 5, 10):
        print(f"[con lsqr] {shape.name} k={k}", flush=True)
        x = torch.empty(S.n, dtype=torch.float64, device="cuda")
        info = gsr.gsr_lsqr_solve(h, cuda(b), x, gsr.solve_opts(itnlim=k, fixed_iters=True))
        assert info["fused"] == int(shape.n_instr <= 10240)
        xo, io = S.lsqr(b, itnlim=k, fixed=True)
        assert info["itn"] == io["itn"] == k
        assert rel(host(x), xo) <= 1e-10, k
        for key in ("rnorm", "arnorm", "anorm"):
            assert abs(info[key] - io[key]) <= 1e-10 * abs(io[key]), (k, key)
    o = gsr.solve_opts(itnlim=2000, fixed_iters=False, atol=1e-14, btol=1e-14)
    info = gsr.gsr_lsqr_solve(h, cuda(b), x, o)
    xo, io = S.lsqr(b, itnlim=2000, fixed=False, atol=1e-14, btol=1e-14)
    print(f"[con lsqr] converged: GPU {info['itn']} its, oracle {io['itn']}", flush=True)
    assert info["istop"] in (1, 2) and io["istop"] in (1, 2)
    assert rel(host(x), xo) <= 1e-10
    # adjoint solve: mu has n_rows + n_con entries
    g = rng.standard_normal(S.n)
    mu = torch.empty(S.m, dtype=torch.float64, device="cuda")
    lam = torch.empty(S.n, dtype=torch.float64, device="cuda")
    o = gsr.solve_opts(itnlim=7, fixed_iters=True)
    gsr.gsr_lsqr_solve_adjoint(h, cuda(g), mu, lam, o)
    muo, _ = S.lsqr_transposed(g, itnlim=7, fixed=True)
    assert rel(host(mu), muo) <= 1e-10
    lamo, _ = S.lsqr(muo, itnlim=7, fixed=True)
    assert rel(host(lam), lamo) <= 1e-9
    # variance estimate over the stacked operator
    var = torch.empty(S.n, dtype=torch.float64, device="cuda")
    gsr.gsr_lsqr_solve_var(h, cuda(b), x, var, gsr.solve_opts(itnlim=10, fixed_iters=True))
    xo, vo, _ = S.lsqr_var(b, itnlim=10, fixed=True)
    assert rel(host(x), xo) <= 1e-10
    np.testing.assert_allclose(host(var), vo, rtol=1e-10, atol=0)
    # stream-ordered solve: the same iterates
    xa = torch.empty_like(x)
    infod = gsr.solve_info_buffer()
    gsr.gsr_lsqr_solve_async(h, cuda(b), xa, infod, gsr.solve_opts(itnlim=5, fixed_iters=True))
    xo, _ = S.lsqr(b, itnlim=5, fixed=True)
    assert rel(host(xa), xo) <= 1e-10
    # removing the constraint rows restores the plain system
    gsr.gsr_set_constraints(h)
    assert h.m == sysd["dims"]["n_rows"]
    S0 = oracle.System(sysd["dims"], sysd["vals"], sysd["star"], sysd["att"], sysd["instr"])
    b0 = b[: S0.m]
    gsr.gsr_lsqr_solve(h, cuda(b0), x, gsr.solve_opts(itnlim=5, fixed_iters=True))
    xo, _ = S0.lsqr(b0, itnlim=5, fixed=True)
    assert rel(host(x), xo) <= 1e-10
    h.close()


def test_rank_deficient_system_made_unique_on_gpu():
    """Stars with fewer than five observations leave A rank deficient; constraint rows on
    those stars make [A; C] full rank: consistent data give x_true back, noisy data the dense
    least-squares solution of the stacked matrix, both as the oracle."""
    shape, deficient, con = _deficient_system(seed=35)
    sysd, S, h, keep = setup(shape, con, build_f32=True)
    from sparse_ref import dense
    A = dense(sysd["dims"], sysd["vals"], sysd["star"], sysd["att"], sysd["instr"])
    B = np.vstack([A, con_dense(con, shape.n_cols)])
    assert np.linalg.matrix_rank(A) < shape.n_cols == np.linalg.matrix_rank(B)
    xt = synth.x_true(shape)
    x = torch.empty(S.n, dtype=torch.float64, device="cuda")
    o = gsr.solve_opts(itnlim=5000, fixed_iters=False, atol=1e-15, btol=1e-15)
    gsr.gsr_lsqr_solve(h, cuda(B @ xt), x, o)
    assert rel(host(x), xt) <= 1e-9
    rng = np.random.default_rng(9)
    bn = np.concatenate([A @ xt + 1e-3 * rng.standard_normal(A.shape[0]), np.zeros(S.n_con)])
    info = gsr.gsr_lsqr_solve(h, cuda(bn), x, o)
    xd = np.linalg.lstsq(B, bn, rcond=None)[0]
    xo, io = S.lsqr(bn, itnlim=5000, fixed=False, atol=1e-15, btol=1e-15)
    print(f"[con deficient] GPU {info['itn']} its, oracle {io['itn']}", flush=True)
    assert rel(host(x), xd) <= 1e-9 and rel(host(x), xo) <= 1e-9
    # the precision form refines to the same constrained solution
    xr = torch.empty_like(x)
    o32 = gsr.solve_opts(itnlim=5000, fixed_iters=False, atol=1e-14, btol=1e-14,
                         precision=gsr.GSR_F32V, max_refine=8, refine_tol=1e-12)
    gsr.gsr_lsqr_solve(h, cuda(bn), xr, o32)
    xro, outer, _ = S.refine(bn, sysd["vals"].astype(np.float32), max_outer=8,
                             refine_tol=1e-12, inner_itnlim=5000, inner_atol=1e-14,
                             inner_btol=1e-14)
    assert rel(host(xr), xro) <= 1e-8 and rel(host(xr), xd) <= 1e-8
    # the stream-ordered precision form on the stacked system: the same correction steps and
    # solution.  Its ~600 inner steps on this ill-conditioned system may end a step or two
    # apart from the synchronous run's: the products add in an order that varies from run to
    # run (atomic sums), and a stopping test that sits at its threshold can flip.
    xa = torch.empty_like(x)
    infod = gsr.solve_info_buffer()
    ref = gsr.gsr_lsqr_solve(h, cuda(bn), xr, o32)
    gsr.gsr_lsqr_solve_async(h, cuda(bn), xa, infod, o32)
    f = gsr.read_solve_info(infod)
    assert f["n_refine"] == ref["n_refine"] and abs(f["itn"] - ref["itn"]) <= 0.02 * ref["itn"]
    assert rel(host(xa), xro) <= 1e-8 and rel(host(xa), xd) <= 1e-8
    h.close()


def test_constraint_rows_only():
    """A system with no observation rows and only constraint rows: the minimum-norm solution
    of C x ~ c over the columns C touches, as the oracle (the other columns are empty)."""
    shape = synth.Shape(6, 10, 10, 8, 12, seed=144)
    sysd = synth.system(shape)
    sys0 = dict(sysd)
    sys0["dims"] = dict(sysd["dims"], n_rows=0)
    for key in ("vals", "star", "att", "instr"):
        sys0[key] = sysd[key][:0]
    con = random_con(shape.n_cols, 5, 9, seed=145, repeat=False)
    S = oracle.System(sys0["dims"], sys0["vals"], sys0["star"], sys0["att"], sys0["instr"],
                      con=con)
    h, _ = open_system(sys0, allow_empty_cols=True)
    cd = con_dev(con)
    gsr.gsr_set_constraints(h, *cd)
    assert h.m == 5
    c = np.random.default_rng(146).standard_normal(5)
    x = torch.empty(S.n, dtype=torch.float64, device="cuda")
    o = gsr.solve_opts(itnlim=200, fixed_iters=False, atol=1e-14, btol=1e-14)
    gsr.gsr_lsqr_solve(h, cuda(c), x, o)
    xo, _ = S.lsqr(c, itnlim=200, fixed=False, atol=1e-14, btol=1e-14)
    assert rel(host(x), xo) <= 1e-10
    y = torch.zeros(5, dtype=torch.float64, device="cuda")
    gsr.gsr_aprod1(h, x, y)
    assert_close_scaled(host(y), S.aprod1(host(x)), 1e-13)
    h.close()


def test_constraint_layout_errors():
    shape = synth.Shape(20, 10, 10, 12, 30, seed=143)
    sysd = synth.system(shape)
    h, _ = open_system(sysd)
    n = shape.n_cols
    dev = lambda a, dt: torch.tensor(a, dtype=dt, device="cuda")  # noqa: E731
    with pytest.raises(gsr.GsrError, match="ptr\\[0\\]"):
        gsr.gsr_set_constraints(h, dev([1, 2], torch.int64), dev([0, 1], torch.int64),
                                dev([1.0, 1.0], torch.float64))
    with pytest.raises(gsr.GsrError, match="decreases"):
        gsr.gsr_set_constraints(h, dev([0, 2, 1, 2], torch.int64), dev([0, 1], torch.int64),
                                dev([1.0, 1.0], torch.float64))
    with pytest.raises(gsr.GsrError, match="column"):
        gsr.gsr_set_constraints(h, dev([0, 2], torch.int64), dev([0, n], torch.int64),
                                dev([1.0, 1.0], torch.float64))
    assert h.m == sysd["dims"]["n_rows"]  # after an error: no constraint rows
    # constraint rows with no entries at all
    gsr.gsr_set_constraints(h, dev([0, 0, 0], torch.int64), dev([], torch.int64),
                            dev([], torch.float64))
    assert h.m == sysd["dims"]["n_rows"] + 2
    S = oracle.System(sysd["dims"], sysd["vals"], sysd["star"], sysd["att"], sysd["instr"],
                      con=dict(ptr=np.array([0, 0, 0]), col=np.array([], dtype=np.int64),
                               val=np.array([])))
    y = torch.zeros(S.m, dtype=torch.float64, device="cuda")
    x = np.random.default_rng(1).standard_normal(S.n)
    gsr.gsr_aprod1(h, cuda(x), y)
    assert_close_scaled(host(y), S.aprod1(x), 1e-13)
    h.close()


def test_full_size_with_frame_constraints():
    """The 2e7-row system with six reference-frame-like constraint rows over a tenth of the
    stars (2e5 coefficients each): products and the first iterates against the oracle."""
    shape = synth.S1M_O20
    print(f"[con full] {shape.name}: generating", flush=True)
    con = synth.frame_constraints(shape, n_con=6, frac=0.1)
    sysd, S, h, keep = setup(shape, con)
    rng = np.random.default_rng(64)
    x = rng.standard_normal(S.n)
    yd = torch.zeros(S.m, dtype=torch.float64, device="cuda")
    gsr.gsr_aprod1(h, cuda(x), yd)
    assert_close_scaled(host(yd), S.aprod1(x), 1e-13)
    y = rng.standard_normal(S.m)
    xd = torch.zeros(S.n, dtype=torch.float64, device="cuda")
    gsr.gsr_aprod2(h, cuda(y), xd)
    assert_close_scaled(host(xd), S.aprod2(y), 1e-12)
    b = S.aprod1(synth.x_true(shape)) + 1e-3 * rng.standard_normal(S.m)
    for k in (1, 2):
        xg = torch.empty(S.n, dtype=torch.float64, device="cuda")
        gsr.gsr_lsqr_solve(h, cuda(b), xg, gsr.solve_opts(itnlim=k, fixed_iters=True))
        print(f"[con full] lsqr {k} oracle", flush=True)
        xo, _ = S.lsqr(b, itnlim=k, fixed=True)
        assert rel(host(xg), xo) <= 1e-10
    h.close()
