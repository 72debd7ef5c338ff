"""gsr_aprod2_noalloc (x += A^T y on the caller's arrays, no handle, no allocation: the block
partial sums live in the library's fixed device scratch) against the handle's gsr_aprod2 and
the oracle, through the C ABI, on two calls in a row, the second with a smaller system; and
its size limit."""
import numpy as np
import pytest
import torch

import synth
from gpu_util import assert_close_scaled, cuda, host, open_system, oracle_system
from paper_2212_11675_amd import gsr

pytestmark = pytest.mark.gpu


def _dims(sysd):
    d = sysd["dims"]
    return gsr.make_dims(d["n_rows"], d["n_stars"], d["n_dfa"], d["n_instr"])


def test_aprod2_noalloc_matches_handle_product_twice():
    shapes = [synth.Shape(3000, 10, 60, 300, 6000, seed=151, name="larger"),
              synth.Shape(40, 10, 60, 30, 40, seed=152, name="smaller")]
    for shape in shapes:
        print(f"[noalloc] {shape.name}", flush=True)
        sysd = synth.system(shape)
        S = oracle_system(sysd)
        h, t = open_system(sysd, allow_empty_cols=True)
        rng = np.random.default_rng(shape.seed)
        y, x0 = rng.standard_normal(S.m), rng.standard_normal(S.n)
        xh = cuda(x0)
        gsr.gsr_aprod2(h, cuda(y), xh)
        xn = cuda(x0)
        gsr.gsr_aprod2_noalloc(_dims(sysd), t["vals"], t["star"], t["att"], t["instr"],
                               cuda(y), xn)
        assert_close_scaled(host(xn), host(xh), 1e-13)
        assert_close_scaled(host(xn), S.aprod2(y, x0), 1e-13)
        h.close()


def test_aprod2_noalloc_refuses_sizes_beyond_its_maximum():
    big = synth.Shape(5, 10, 10, 8, 10241, seed=153)
    sysd = synth.system(big)
    t = {k: torch.from_numpy(np.ascontiguousarray(sysd[k])).to("cuda")
         for k in ("vals", "star", "att", "instr")}
    x = torch.zeros(big.n_cols, dtype=torch.float64, device="cuda")
    y = torch.zeros(sysd["dims"]["n_rows"], dtype=torch.float64, device="cuda")
    with pytest.raises(gsr.GsrError, match="beyond the maximum") as ei:
        gsr.gsr_aprod2_noalloc(_dims(sysd), t["vals"], t["star"], t["att"], t["instr"], y, x)
    assert ei.value.status == -6
    assert float(x.abs().max()) == 0.0
