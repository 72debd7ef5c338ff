"""The seeded input generators: structure, determinism, counter-based slicing."""
import numpy as np

import synth


def test_structure_small():
    sh = synth.S1K_O60
    s = synth.system(sh)
    m = s["dims"]["n_rows"]
    assert m == 60_000
    assert sh.n_cols == 5 * 1000 + 3 * 1000 + 500 + 1
    star, att, instr = s["star"], s["att"], s["instr"].reshape(m, 6)
    assert np.all(np.diff(star) >= 0) and star[0] == 0 and star[-1] == 999
    assert np.all(np.bincount(star) == 60)
    assert att.min() == 0 and att.max() == 996  # t ~ U[0, n_dfa - 4]
    assert instr.min() >= 0 and instr.max() < 500
    assert np.all(np.diff(instr, axis=1) > 0)  # 6 distinct, ascending
    v = s["vals"]
    assert abs(v.mean()) < 0.01 and abs(v.std() - 1.0) < 0.01


def test_deterministic_and_sliceable():
    sh = synth.Shape(300, 10, 60, 30, 40, seed=11)
    a = synth.system(sh)
    b = synth.system(sh)
    for k in ("star", "att", "instr", "vals"):
        assert np.array_equal(a[k], b[k])
    m = a["dims"]["n_rows"]
    r0, r1 = m // 3, m // 3 + 777
    part = synth.rows(sh, r0, r1)
    assert np.array_equal(part["star"], a["star"][r0:r1])
    assert np.array_equal(part["att"], a["att"][r0:r1])
    assert np.array_equal(part["instr"], a["instr"][6 * r0: 6 * r1])
    assert np.array_equal(part["vals"], a["vals"][24 * r0: 24 * r1])
    counts = sh.star_counts()
    assert counts.min() >= 10 and counts.max() <= 60 and counts.sum() == m


def test_batch_shapes():
    shapes = synth.batch_shapes()
    assert len(shapes) == 64
    s = np.array([x.n_stars for x in shapes])
    assert s.min() >= 1000 and s.max() <= 200_000
    assert len({x.seed for x in shapes}) == 64
    for x in shapes:
        assert x.n_dfa == x.n_stars // 10 and x.n_instr == 500


def test_noise_scale():
    e = synth.noise(synth.S1K_O60)
    assert abs(e.std() - 1e-3) < 2e-5
