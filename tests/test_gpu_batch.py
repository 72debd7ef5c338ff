"""Batched form (many systems x k right-hand sides) vs the oracle, through the C ABI.

Every (system, right-hand side) pair must match the oracle's solo PC-LSQR on that system
and right-hand side (binary64: ||x - x_oracle|| / ||x_oracle|| <= 1e-10); the multi-RHS
products must match the oracle's single-RHS products column by column.
"""
import numpy as np
import pytest
import torch

import synth
from gpu_util import assert_close_scaled, cuda, host, oracle_system, rel
from paper_2212_11675_amd import gsr

pytestmark = pytest.mark.gpu

SHAPES = [
    synth.Shape(1, 7, 7, 4, 6, seed=71, name="tiny"),
    synth.Shape(300, 10, 60, 30, 40, seed=72, name="s300"),
    synth.Shape(57, 10, 60, 5, 500, seed=73, name="s57_instr500"),
    synth.Shape(1000, 20, 20, 100, 500, seed=74, name="s1000"),
    synth.Shape(33, 10, 60, 30, 9, seed=75, name="s33"),
]


def make_batch(shapes, k):
    systems = [synth.system(sh) for sh in shapes]
    dims = [gsr.make_dims(s["dims"]["n_rows"], s["dims"]["n_stars"], s["dims"]["n_dfa"],
                          s["dims"]["n_instr"]) for s in systems]
    row_offset = np.concatenate([[0], np.cumsum([s["dims"]["n_rows"] for s in systems])])
    cat = {key: np.concatenate([s[key] for s in systems]) for key in ("vals", "star", "att",
                                                                      "instr")}
    dev = {key: torch.from_numpy(v).to("cuda:0") for key, v in cat.items()}
    b = gsr.gsr_batch_setup(dims, row_offset.tolist(), dev["vals"], dev["star"], dev["att"],
                            dev["instr"], k, allow_empty_cols=True)
    return b, systems, dev


@pytest.mark.parametrize("k", [1, 2, 4, 8])
def test_batched_products_vs_oracle(k):
    print(f"[batch products] k={k}", flush=True)
    b, systems, _ = make_batch(SHAPES, k)
    rng = np.random.default_rng(81 + k)
    X = rng.standard_normal((b.n, k))
    Y0 = rng.standard_normal((b.m, k))
    Yd = cuda(Y0.ravel())
    gsr.gsr_batch_aprod1(b, cuda(X.ravel()), Yd)
    Yg = host(Yd).reshape(b.m, k)
    Y = rng.standard_normal((b.m, k))
    X0 = rng.standard_normal((b.n, k))
    Xd = cuda(X0.ravel())
    gsr.gsr_batch_aprod2(b, cuda(Y.ravel()), Xd)
    Xg = host(Xd).reshape(b.n, k)
    for s, sysd in enumerate(systems):
        S = oracle_system(sysd)
        r0, r1 = b.row_offset[s], b.row_offset[s + 1]
        c0, c1 = b.col_offset[s], b.col_offset[s + 1]
        assert c1 - c0 == S.n
        for j in range(k):
            assert_close_scaled(Yg[r0:r1, j], S.aprod1(X[c0:c1, j], Y0[r0:r1, j]), 1e-13)
            assert_close_scaled(Xg[c0:c1, j], S.aprod2(Y[r0:r1, j], X0[c0:c1, j]), 1e-13)
    b.close()


@pytest.mark.parametrize("k,iters", [(8, 1), (8, 7), (8, 40), (4, 12), (2, 15), (1, 9)])
def test_batched_solve_matches_solo_oracle(k, iters):
    print(f"[batch solve] k={k} iters={iters}", flush=True)
    b, systems, _ = make_batch(SHAPES, k)
    B = np.zeros((b.m, k))
    oracles = []
    for s, sysd in enumerate(systems):
        S = oracle_system(sysd)
        shape = SHAPES[s]
        r0, r1 = b.row_offset[s], b.row_offset[s + 1]
        for j in range(k):
            B[r0:r1, j] = S.aprod1(synth.rhs_x(shape, j)) + synth.rhs_noise(shape, j, S.m)
        oracles.append(S)
    Xd = torch.empty(b.n * k, dtype=torch.float64, device="cuda")
    infos = gsr.gsr_batch_solve(b, cuda(B.ravel()), Xd,
                                gsr.solve_opts(itnlim=iters, fixed_iters=True))
    Xg = host(Xd).reshape(b.n, k)
    for s, S in enumerate(oracles):
        r0, r1 = b.row_offset[s], b.row_offset[s + 1]
        c0, c1 = b.col_offset[s], b.col_offset[s + 1]
        for j in range(k):
            xo, io = S.lsqr(B[r0:r1, j], itnlim=iters, fixed=True)
            assert infos[s * k + j]["itn"] == io["itn"], (s, j)
            assert rel(Xg[c0:c1, j], xo) <= 1e-10, (s, j)
    # a second solve into new buffers (graph captured again) gives the same answer
    Bd = cuda(B.ravel())
    Xd2 = torch.empty_like(Xd)
    gsr.gsr_batch_solve(b, Bd, Xd2, gsr.solve_opts(itnlim=iters, fixed_iters=True))
    first = host(Xd2)
    assert rel(first, host(Xd)) <= 1e-13
    # replays of the cached graph (same buffers), with eager work of the library and of torch
    # on the same stream in between: every replay matches
    rng = np.random.default_rng(90 + iters)
    for rep in range(3):
        Yd = cuda(rng.standard_normal(b.m * k))
        gsr.gsr_batch_aprod1(b, cuda(rng.standard_normal(b.n * k)), Yd)
        Xd2.mul_(-3.0).add_(Yd.sum())
        torch.cuda.synchronize()
        gsr.gsr_batch_solve(b, Bd, Xd2, gsr.solve_opts(itnlim=iters, fixed_iters=True))
        assert rel(host(Xd2), first) <= 1e-13, rep
    b.close()


def test_batched_converged_solve():
    k = 8
    b, systems, _ = make_batch(SHAPES[1:], k)
    B = np.zeros((b.m, k))
    for s, sysd in enumerate(systems):
        S = oracle_system(sysd)
        r0, r1 = b.row_offset[s], b.row_offset[s + 1]
        for j in range(k):
            B[r0:r1, j] = S.aprod1(synth.rhs_x(SHAPES[1 + s], j)) + synth.rhs_noise(
                SHAPES[1 + s], j, S.m)
    Xd = torch.empty(b.n * k, dtype=torch.float64, device="cuda")
    infos = gsr.gsr_batch_solve(b, cuda(B.ravel()), Xd,
                                gsr.solve_opts(itnlim=3000, fixed_iters=False, atol=1e-12,
                                               btol=1e-12))
    Xg = host(Xd).reshape(b.n, k)
    for s, sysd in enumerate(systems):
        S = oracle_system(sysd)
        r0, r1 = b.row_offset[s], b.row_offset[s + 1]
        c0, c1 = b.col_offset[s], b.col_offset[s + 1]
        for j in range(k):
            xo, io = S.lsqr(B[r0:r1, j], itnlim=3000, fixed=False, atol=1e-12, btol=1e-12)
            assert infos[s * k + j]["istop"] in (1, 2)
            # near the tolerance the test ratios move with rounding: the stop iteration may
            # drift by a few iterations, the solutions agree to the tolerance
            assert abs(infos[s * k + j]["itn"] - io["itn"]) <= max(3, io["itn"] // 10)
            assert rel(Xg[c0:c1, j], xo) <= 1e-9
    b.close()


def test_batched_nonfinite_pair_is_reported():
    """A non-finite right-hand side in one (system, rhs) pair: the call reports a breakdown,
    the solve information names that pair, and every other pair still matches the oracle."""
    k, iters = 4, 9
    print(f"[batch nonfinite] k={k} iters={iters}", flush=True)
    b, systems, _ = make_batch(SHAPES, k)
    B = np.zeros((b.m, k))
    oracles = []
    for s, sysd in enumerate(systems):
        S = oracle_system(sysd)
        r0, r1 = b.row_offset[s], b.row_offset[s + 1]
        for j in range(k):
            B[r0:r1, j] = S.aprod1(synth.rhs_x(SHAPES[s], j)) + synth.rhs_noise(SHAPES[s], j,
                                                                               S.m)
        oracles.append(S)
    bad_s, bad_j = 3, 2
    B[b.row_offset[bad_s] + 5, bad_j] = np.nan
    Xd = torch.empty(b.n * k, dtype=torch.float64, device="cuda")
    with pytest.raises(gsr.GsrError) as ei:
        gsr.gsr_batch_solve(b, cuda(B.ravel()), Xd, gsr.solve_opts(itnlim=iters, fixed_iters=True))
    assert ei.value.status == -5
    infos = ei.value.info
    Xg = host(Xd).reshape(b.n, k)
    for s, S in enumerate(oracles):
        r0, r1 = b.row_offset[s], b.row_offset[s + 1]
        c0, c1 = b.col_offset[s], b.col_offset[s + 1]
        for j in range(k):
            f = infos[s * k + j]
            if (s, j) == (bad_s, bad_j):
                assert f["nonfinite"] == 1
                continue
            assert f["nonfinite"] == 0 and f["fused"] == 1, (s, j)
            xo, io = S.lsqr(B[r0:r1, j], itnlim=iters, fixed=True)
            assert f["itn"] == io["itn"], (s, j)
            assert rel(Xg[c0:c1, j], xo) <= 1e-10, (s, j)
    b.close()


def test_batched_condition_limit_stops_every_pair():
    """conlim: each (system, right-hand side) pair stops on its own condition estimate at the
    step the oracle's solo solve does."""
    k = 2
    b, systems, _ = make_batch(SHAPES[1:], k)
    B = np.zeros((b.m, k))
    for s, sysd in enumerate(systems):
        S = oracle_system(sysd)
        r0, r1 = b.row_offset[s], b.row_offset[s + 1]
        for j in range(k):
            B[r0:r1, j] = S.aprod1(synth.rhs_x(SHAPES[1 + s], j)) + synth.rhs_noise(
                SHAPES[1 + s], j, S.m)
    Xd = torch.empty(b.n * k, dtype=torch.float64, device="cuda")
    o = gsr.solve_opts(itnlim=500, fixed_iters=False, atol=0.0, btol=0.0, conlim=25.0)
    infos = gsr.gsr_batch_solve(b, cuda(B.ravel()), Xd, o)
    Xg = host(Xd).reshape(b.n, k)
    for s, sysd in enumerate(systems):
        S = oracle_system(sysd)
        r0, r1 = b.row_offset[s], b.row_offset[s + 1]
        c0, c1 = b.col_offset[s], b.col_offset[s + 1]
        for j in range(k):
            xo, io = S.lsqr(B[r0:r1, j], itnlim=500, fixed=False, atol=0.0, btol=0.0,
                            conlim=25.0)
            f = infos[s * k + j]
            assert (f["istop"], f["itn"]) == (io["istop"], io["itn"]), (s, j)
            assert abs(f["acond"] - io["acond"]) <= 1e-10 * io["acond"], (s, j)
            assert rel(Xg[c0:c1, j], xo) <= 1e-10, (s, j)
    b.close()


def test_batched_argument_errors():
    sh = SHAPES[1]
    sysd = synth.system(sh)
    dev = {key: torch.from_numpy(sysd[key]).to("cuda:0") for key in ("vals", "star", "att",
                                                                     "instr")}
    d = gsr.make_dims(sysd["dims"]["n_rows"], sh.n_stars, sh.n_dfa, sh.n_instr)
    with pytest.raises(gsr.GsrError, match="k must be"):
        gsr.gsr_batch_setup([d], [0, sysd["dims"]["n_rows"]], dev["vals"], dev["star"],
                            dev["att"], dev["instr"], 3)
    with pytest.raises(gsr.GsrError, match="row_offset"):
        gsr.gsr_batch_setup([d], [0, sysd["dims"]["n_rows"] - 1], dev["vals"][:-24],
                            dev["star"][:-1], dev["att"][:-1], dev["instr"][:-6], 8)


def test_batched_extreme_systems_of_the_64_system_workload():
    """The smallest and the largest system of the 64-system workload (1,007 and 198,336 stars,
    3.5e4 and 6.9e6 rows), at their real sizes, batched with k = 8 right-hand sides: products
    and 5 PC-LSQR iterations of every (system, rhs) pair against the oracle's solo solve."""
    shapes = synth.batch_shapes()
    order = sorted(range(len(shapes)), key=lambda i: shapes[i].n_stars)
    pick = [shapes[order[0]], shapes[order[-1]]]
    k, iters = 8, 5
    print(f"[batch extremes] {[(s.n_stars, s.n_rows) for s in pick]}", flush=True)
    b, systems, _ = make_batch(pick, k)
    rng = np.random.default_rng(97)
    X = rng.standard_normal((b.n, k))
    Yd = torch.zeros(b.m * k, dtype=torch.float64, device="cuda")
    gsr.gsr_batch_aprod1(b, cuda(X.ravel()), Yd)
    Yg = host(Yd).reshape(b.m, k)
    B = np.zeros((b.m, k))
    oracles = []
    for s, sysd in enumerate(systems):
        S = oracle_system(sysd)
        r0, r1 = b.row_offset[s], b.row_offset[s + 1]
        c0, c1 = b.col_offset[s], b.col_offset[s + 1]
        for j in range(k):
            assert_close_scaled(Yg[r0:r1, j], S.aprod1(X[c0:c1, j]), 1e-13)
            B[r0:r1, j] = S.aprod1(synth.rhs_x(pick[s], j)) + synth.rhs_noise(pick[s], j, S.m)
        oracles.append(S)
    Xd = torch.empty(b.n * k, dtype=torch.float64, device="cuda")
    infos = gsr.gsr_batch_solve(b, cuda(B.ravel()), Xd,
                                gsr.solve_opts(itnlim=iters, fixed_iters=True))
    Xg = host(Xd).reshape(b.n, k)
    for s, S in enumerate(oracles):
        r0, r1 = b.row_offset[s], b.row_offset[s + 1]
        c0, c1 = b.col_offset[s], b.col_offset[s + 1]
        p = S.colnorm()
        for j in range(k):
            print(f"[batch extremes] system {s} rhs {j}", flush=True)
            xo, io = S.lsqr(B[r0:r1, j], itnlim=iters, fixed=True, p=p)
            assert infos[s * k + j]["itn"] == io["itn"] == iters
            assert rel(Xg[c0:c1, j], xo) <= 1e-10, (s, j)
    b.close()
