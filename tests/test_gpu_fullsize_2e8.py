"""The 2e8-row workload (5e6 stars x 40 observations, 1e5 attitude knots per axis, 1e4
instrumental columns: the largest LDS footprint of the fused row pass) at its real size,
set up as the benchmark sets it up.  The CPU oracle cannot take the whole system, so:
  - aprod 1 on 2,000 sampled rows, computed by the oracle on the sub-system of those rows;
  - the adjoint identity <A x, y> = <x, A^T y>;
  - the first PC-LSQR iterate against its closed form, the minimizer of ||A D z - b|| along
    z = D A^T b (LSQR's first step), built from the library's products;
  - LSQR's residual estimate against the directly computed residual after 5 iterations.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from gpu_util import assert_close_scaled, host, rel, upload_chunked
from paper_2212_11675_amd import gsr

pytestmark = pytest.mark.gpu


def test_full_size_2e8_sampled_rows_adjoint_and_first_iterate():
    shape = synth.S5M_O40
    print(f"[2e8] {shape.name}: generating and uploading", flush=True)
    t, d, rp = upload_chunked(shape)
    m, n = d["n_rows"], shape.n_cols
    h = gsr.gsr_lsqr_setup(gsr.make_dims(m, d["n_stars"], d["n_dfa"], d["n_instr"]), t["vals"],
                           t["star"], t["att"], t["instr"])
    dev = torch.device("cuda:0")
    gen = torch.Generator(device=dev)
    gen.manual_seed(2208)
    # aprod 1 on sampled rows
    x = torch.randn(n, dtype=torch.float64, device=dev, generator=gen)
    y = torch.zeros(m, dtype=torch.float64, device=dev)
    gsr.gsr_aprod1(h, x, y)
    rows = np.sort(np.random.default_rng(2209).choice(m, size=2000, replace=False))
    parts = [synth.rows(shape, int(r), int(r) + 1, row_ptr=rp) for r in rows]
    sub = {k: np.concatenate([p[k] for p in parts]) for k in ("vals", "star", "att", "instr")}
    S = oracle.System(dict(n_rows=len(rows), n_stars=d["n_stars"], n_dfa=d["n_dfa"],
                           n_instr=d["n_instr"], n_glob=1),
                      sub["vals"], sub["star"], sub["att"], sub["instr"])
    print("[2e8] sampled rows vs oracle", flush=True)
    assert_close_scaled(host(y)[rows], S.aprod1(host(x)), 1e-13)
    # adjoint identity
    yr = torch.randn(m, dtype=torch.float64, device=dev, generator=gen)
    xs = torch.zeros(n, dtype=torch.float64, device=dev)
    gsr.gsr_aprod2(h, yr, xs)
    lhs, rhs = float(torch.dot(y, yr)), float(torch.dot(x, xs))
    scale = float(torch.linalg.norm(y) * torch.linalg.norm(yr))
    print(f"[2e8] <Ax,y> {lhs:.12e} <x,A^T y> {rhs:.12e}", flush=True)
    assert abs(lhs - rhs) <= 1e-12 * scale
    # right-hand side b = A x_true + e (library product, noise from the generator)
    b = torch.from_numpy(synth.noise(shape)).to(dev)
    gsr.gsr_aprod1(h, torch.from_numpy(synth.x_true(shape)).to(dev), b)
    # first iterate: x1 = tau D^2 A^T b with tau = <A D g, b> / ||A D g||^2, g = D A^T b
    p = torch.empty(n, dtype=torch.float64, device=dev)
    gsr.gsr_precond(h, p)
    s = torch.zeros(n, dtype=torch.float64, device=dev)
    gsr.gsr_aprod2(h, b, s)
    g = p * s
    w = torch.zeros(m, dtype=torch.float64, device=dev)
    gsr.gsr_aprod1(h, p * g, w)
    tau = float(torch.dot(w, b) / torch.dot(w, w))
    x1 = torch.empty(n, dtype=torch.float64, device=dev)
    info = gsr.gsr_lsqr_solve(h, b, x1, gsr.solve_opts(itnlim=1, fixed_iters=True))
    assert info["fused"] == 1
    print("[2e8] first iterate vs closed form", flush=True)
    assert rel(host(x1), host(tau * p * g)) <= 1e-12
    # residual estimate after 5 iterations
    x5 = torch.empty(n, dtype=torch.float64, device=dev)
    info = gsr.gsr_lsqr_solve(h, b, x5, gsr.solve_opts(itnlim=5, fixed_iters=True))
    r = torch.empty(m, dtype=torch.float64, device=dev)
    gsr.gsr_residual(h, b, x5, r)
    rn = float(torch.linalg.norm(r))
    print(f"[2e8] rnorm estimate {info['rnorm']:.12e} direct {rn:.12e}", flush=True)
    assert abs(info["rnorm"] - rn) <= 1e-10 * rn
    h.close()
