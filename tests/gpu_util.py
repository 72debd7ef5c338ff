"""Helpers of the GPU tests: upload generated systems, open handles, compare with the oracle."""
import numpy as np
import torch

import oracle
import synth
from paper_2212_11675_amd import gsr


def upload(sysd: dict) -> dict:
    dev = torch.device("cuda:0")
    return {k: torch.from_numpy(np.ascontiguousarray(sysd[k])).to(dev)
            for k in ("vals", "star", "att", "instr")}


def open_system(sysd: dict, **kw):
    d = sysd["dims"]
    t = upload(sysd)
    h = gsr.gsr_lsqr_setup(gsr.make_dims(d["n_rows"], d["n_stars"], d["n_dfa"], d["n_instr"]),
                           t["vals"], t["star"], t["att"], t["instr"], **kw)
    return h, t


def oracle_system(sysd: dict) -> oracle.System:
    return oracle.System(sysd["dims"], sysd["vals"], sysd["star"], sysd["att"], sysd["instr"])


def cuda(a) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to("cuda:0")


def host(t: torch.Tensor) -> np.ndarray:
    torch.cuda.synchronize()
    return t.cpu().numpy()


def rel(a, b) -> float:
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / (nb if nb > 0 else 1.0))


def assert_close_scaled(got, ref, tol):
    """Elementwise |got - ref| <= tol * max|ref| (products with rounding-order differences)."""
    got, ref = np.asarray(got), np.asarray(ref)
    scale = max(np.abs(ref).max(), 1e-300)
    err = np.abs(got - ref).max() / scale
    assert err <= tol, f"max scaled error {err:.3e} > {tol:.1e}"


SMALL_SHAPES = [
    synth.Shape(1, 7, 7, 4, 6, seed=21, name="one_star_7rows"),
    synth.Shape(3, 10, 60, 9, 13, seed=22, name="ragged_97rows"),
    synth.Shape(40, 10, 60, 30, 40, seed=23, name="stars40_ragged"),
    synth.Shape(300, 20, 20, 100, 50, seed=24, name="stars300_obs20"),
    synth.Shape(2000, 10, 60, 200, 500, seed=25, name="stars2000_obs10to60"),
]


def upload_chunked(shape, chunk_rows: int = 10_000_000):
    """Generate `shape` on the host in row chunks and copy it to the GPU (bounded host
    memory); returns the device arrays, the dims and the star row pointer."""
    rp = shape.row_ptr()
    m = int(rp[-1])
    dev = torch.device("cuda:0")
    t = {"vals": torch.empty(24 * m, dtype=torch.float64, device=dev),
         "star": torch.empty(m, dtype=torch.int32, device=dev),
         "att": torch.empty(m, dtype=torch.int32, device=dev),
         "instr": torch.empty(6 * m, dtype=torch.int32, device=dev)}
    for r0 in range(0, m, chunk_rows):
        r1 = min(m, r0 + chunk_rows)
        part = synth.rows(shape, r0, r1, row_ptr=rp)
        t["vals"][24 * r0: 24 * r1].copy_(torch.from_numpy(part["vals"]))
        t["star"][r0:r1].copy_(torch.from_numpy(part["star"]))
        t["att"][r0:r1].copy_(torch.from_numpy(part["att"]))
        t["instr"][6 * r0: 6 * r1].copy_(torch.from_numpy(part["instr"]))
    torch.cuda.synchronize()
    dims = dict(n_rows=m, n_stars=shape.n_stars, n_dfa=shape.n_dfa, n_instr=shape.n_instr,
                n_glob=1)
    return t, dims, rp
