"""The 2e8-row workload (5e6 stars x 40 observations, 1e5 attitude knots per axis, 1e4
instrumental columns: the largest LDS footprint of the fused row pass, more than 2^31
coefficients) at its real size, set up as the benchmark sets it up, against the oracle on
the whole system held in host memory (45 GB):
  - aprod 1, aprod 2 and the preconditioner, every entry;
  - the binary32 products, every entry, against the oracle on the binary32-rounded
    coefficients (row chunks of the system, so that only one rounded chunk is in memory);
  - the first two PC-LSQR iterates and their residual estimate;
  - the adjoint identity and the residual estimate after 5 iterations against the oracle's
    residual.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import assert_close_scaled, cuda, host, open_system, oracle_system, rel
from paper_2212_11675_amd import gsr

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]

SHAPE = synth.S5M_O40


@pytest.fixture(scope="module")
def big():
    print(f"[2e8] {SHAPE.name}: generating on the host", flush=True)
    sysd = synth.system(SHAPE)
    S = oracle_system(sysd)
    print("[2e8] uploading and setting up", flush=True)
    h, t = open_system(sysd, build_f32=True)
    yield dict(sysd=sysd, S=S, h=h, t=t)
    h.close()


def test_2e8_products_and_preconditioner_vs_oracle(big):
    S, h = big["S"], big["h"]
    rng = np.random.default_rng(2208)
    x = rng.standard_normal(S.n)
    yd = torch.zeros(S.m, dtype=torch.float64, device="cuda")
    gsr.gsr_aprod1(h, cuda(x), yd)
    print("[2e8] aprod1 vs oracle", flush=True)
    y = host(yd)
    assert_close_scaled(y, S.aprod1(x), 1e-13)
    yr = rng.standard_normal(S.m)
    xd = torch.zeros(S.n, dtype=torch.float64, device="cuda")
    gsr.gsr_aprod2(h, cuda(yr), xd)
    print("[2e8] aprod2 vs oracle", flush=True)
    xs = host(xd)
    assert_close_scaled(xs, S.aprod2(yr), 1e-12)
    # adjoint identity of the library's own products
    lhs, rhs = float(np.dot(y, yr)), float(np.dot(x, xs))
    assert abs(lhs - rhs) <= 1e-12 * float(np.linalg.norm(y) * np.linalg.norm(yr))
    p = torch.empty(S.n, dtype=torch.float64, device="cuda")
    gsr.gsr_precond(h, p)
    print("[2e8] preconditioner vs oracle", flush=True)
    np.testing.assert_allclose(host(p), S.colnorm(), rtol=1e-12, atol=0)


def test_2e8_binary32_products_vs_oracle(big):
    sysd, S, h = big["sysd"], big["S"], big["h"]
    rng = np.random.default_rng(2210)
    x = rng.standard_normal(S.n)
    yr = rng.standard_normal(S.m)
    yd = torch.zeros(S.m, dtype=torch.float64, device="cuda")
    gsr.gsr_aprod1_f32v(h, cuda(x), yd)
    xd = torch.zeros(S.n, dtype=torch.float64, device="cuda")
    gsr.gsr_aprod2_f32v(h, cuda(yr), xd)
    y32, x32 = host(yd), host(xd)
    d = sysd["dims"]
    rp = sysd["row_ptr"]
    xo = np.zeros(S.n)
    step = 500_000  # stars per chunk (2e7 rows)
    for s0 in range(0, d["n_stars"], step):
        r0, r1 = int(rp[s0]), int(rp[min(s0 + step, d["n_stars"])])
        print(f"[2e8] binary32 rows {r0}..{r1}", flush=True)
        lo = sysd["vals"][24 * r0: 24 * r1].astype(np.float32).astype(np.float64)
        C = oracle.System(dict(d, n_rows=r1 - r0), lo, sysd["star"][r0:r1], sysd["att"][r0:r1],
                          sysd["instr"][6 * r0: 6 * r1])
        assert_close_scaled(y32[r0:r1], C.aprod1(x), 1e-13)
        xo = C.aprod2(yr[r0:r1], xo)
    assert_close_scaled(x32, xo, 1e-12)


def test_2e8_first_iterations_and_residual_vs_oracle(big):
    S, h = big["S"], big["h"]
    b = S.aprod1(synth.x_true(SHAPE)) + synth.noise(SHAPE)
    p = S.colnorm()
    bd = cuda(b)
    for k in (1, 2):
        xg = torch.empty(S.n, dtype=torch.float64, device="cuda")
        info = gsr.gsr_lsqr_solve(h, bd, xg, gsr.solve_opts(itnlim=k, fixed_iters=True))
        assert info["fused"] == 1
        print(f"[2e8] PC-LSQR {k} vs oracle", flush=True)
        xo, io = S.lsqr(b, itnlim=k, fixed=True, p=p)
        assert rel(host(xg), xo) <= 1e-10, k
        for key in ("rnorm", "arnorm", "anorm", "znorm"):
            assert abs(info[key] - io[key]) <= 1e-10 * abs(io[key]), (k, key)
    # residual estimate after 5 iterations against the oracle's residual of the GPU iterate
    x5 = torch.empty(S.n, dtype=torch.float64, device="cuda")
    info = gsr.gsr_lsqr_solve(h, bd, x5, gsr.solve_opts(itnlim=5, fixed_iters=True))
    r = S.residual(b, host(x5))
    rn = float(np.linalg.norm(r))
    rg = torch.empty(S.m, dtype=torch.float64, device="cuda")
    gsr.gsr_residual(h, bd, x5, rg)
    print(f"[2e8] rnorm estimate {info['rnorm']:.12e} oracle residual {rn:.12e}", flush=True)
    assert abs(info["rnorm"] - rn) <= 1e-10 * rn
    assert_close_scaled(host(rg), r, 1e-12)
