"""Differentiation form: gradients through the GPU least-squares solve.

Checked against (1) the oracle's adjoint (same definition, CPU), (2) the dense closed form
from the normal equations on the 60,000-row system, (3) central finite differences with
h = 1e-6 along random +-1 directions (loss differences written without cancellation), and
(4) torch.autograd.gradcheck on a tiny system.
"""
import numpy as np
import pytest
import torch

import synth
from gpu_util import host, oracle_system, rel, upload
from paper_2212_11675_amd import autograd as gad

pytestmark = pytest.mark.gpu


def _structure(sysd, shape):
    t = upload(sysd)
    return t, gad.Structure(t["star"], t["att"], t["instr"], shape.n_stars, shape.n_dfa,
                            shape.n_instr)


def _loss_grads(vals, b, st, xr):
    vals = vals.clone().requires_grad_(True)
    b = b.clone().requires_grad_(True)
    x = gad.lstsq(vals, b, st)
    loss = ((x - xr) ** 2).sum()
    loss.backward()
    return x.detach(), loss.detach(), vals.grad, b.grad


def test_grad_vs_oracle_and_dense_closed_form():
    shape = synth.S1K_O60
    sysd = synth.system(shape)
    S = oracle_system(sysd)
    b = S.aprod1(synth.x_true(shape)) + synth.noise(shape)
    xr = synth.x_ref(shape)
    t, st = _structure(sysd, shape)
    dev = torch.device("cuda:0")
    x, loss, gv, gb = _loss_grads(t["vals"], torch.from_numpy(b).to(dev), st,
                                  torch.from_numpy(xr).to(dev))
    ref = S.solve_and_grad(b, 2 * (host(x) - xr))
    assert rel(host(x), ref["x"]) <= 1e-10
    assert rel(host(gb), ref["mu"]) <= 1e-8
    assert rel(host(gv), ref["dvals"]) <= 1e-8
    # dense normal equations (n = 8,501): dL/db = A (A^T A)^-1 g
    from sparse_ref import csr
    A = csr(sysd["dims"], sysd["vals"], sysd["star"], sysd["att"], sysd["instr"])
    N = (A.T @ A).toarray()
    xs = np.linalg.solve(N, A.T @ b)
    g = 2 * (xs - xr)
    lam = np.linalg.solve(N, g)
    mu = A @ lam
    assert rel(host(x), xs) <= 1e-10
    assert rel(host(gb), mu) <= 1e-8


def test_grad_vs_central_differences():
    shape = synth.Shape(200, 20, 20, 40, 30, seed=91, name="fd")
    sysd = synth.system(shape)
    S = oracle_system(sysd)
    b = S.aprod1(synth.x_true(shape)) + synth.noise(shape)
    xr = synth.x_ref(shape)
    t, st = _structure(sysd, shape)
    dev = torch.device("cuda:0")
    bd, xrd = torch.from_numpy(b).to(dev), torch.from_numpy(xr).to(dev)
    x, loss, gv, gb = _loss_grads(t["vals"], bd, st, xrd)
    rng = np.random.default_rng(92)
    h = 1e-6

    def solve(vals, bb):
        with torch.no_grad():
            return gad.lstsq(vals, bb, st)

    eb = torch.from_numpy(rng.choice([-1.0, 1.0], size=S.m)).to(dev)
    xp, xm = solve(t["vals"], bd + h * eb), solve(t["vals"], bd - h * eb)
    fd = float(((xp - xm) * (xp + xm - 2 * xrd)).sum() / (2 * h))
    an = float((gb * eb).sum())
    print(f"dL/db directional: analytic {an:.12e} fd {fd:.12e}")
    assert abs(fd - an) <= 1e-6 * abs(an)
    ev = torch.from_numpy(rng.choice([-1.0, 1.0], size=24 * S.m)).to(dev)
    xp, xm = solve(t["vals"] + h * ev, bd), solve(t["vals"] - h * ev, bd)
    fd = float(((xp - xm) * (xp + xm - 2 * xrd)).sum() / (2 * h))
    an = float((gv * ev).sum())
    print(f"dL/dvals directional: analytic {an:.12e} fd {fd:.12e}")
    assert abs(fd - an) <= 1e-6 * abs(an)


def test_gradcheck_tiny():
    # 2 stars x 30 rows, 29 unknowns: full column rank
    shape = synth.Shape(2, 30, 30, 4, 6, seed=93, name="gc")
    sysd = synth.system(shape)
    t, st = _structure(sysd, shape)
    S = oracle_system(sysd)
    dev = torch.device("cuda:0")
    b = torch.from_numpy(S.aprod1(synth.x_true(shape)) + 0.1 * np.random.default_rng(94)
                         .standard_normal(S.m)).to(dev)
    vals = t["vals"].clone().requires_grad_(True)
    b = b.clone().requires_grad_(True)
    # device atomics reorder the column sums: repeated backward passes agree to rounding only
    assert torch.autograd.gradcheck(lambda v, bb: gad.lstsq(v, bb, st), (vals, b), eps=1e-6,
                                    atol=1e-6, rtol=1e-5, nondet_tol=1e-12)


def test_one_handle_reused_in_training_loop():
    """The structure's handle is set up once; coefficients changed in place between steps
    (as by an optimizer) are brought into it with gsr_update_values.  Every step's gradients
    match those of a fresh structure on the same values, device memory stays flat over the
    steps, and a backward pass run after another solve changed the values gets its own."""
    shape = synth.Shape(400, 10, 60, 60, 50, seed=95, name="loop")
    sysd = synth.system(shape)
    S = oracle_system(sysd)
    dev = torch.device("cuda:0")
    b = torch.from_numpy(S.aprod1(synth.x_true(shape)) + synth.noise(shape)).to(dev)
    xr = torch.from_numpy(synth.x_ref(shape)).to(dev)
    t, st = _structure(sysd, shape)
    vals = t["vals"].clone().requires_grad_(True)
    rng = np.random.default_rng(96)
    free, ptr0 = [], None
    for step in range(6):
        x = gad.lstsq(vals, b, st, atol=1e-14, btol=1e-14)
        loss = ((x - xr) ** 2).sum()
        loss.backward()
        if ptr0 is None:
            ptr0 = st._handle.ptr.value
        assert st._handle.ptr.value == ptr0  # no new handle
        # the same step on a fresh structure
        t2, st2 = _structure(sysd, shape)
        v2 = vals.detach().clone().requires_grad_(True)
        x2 = gad.lstsq(v2, b, st2, atol=1e-14, btol=1e-14)
        ((x2 - xr) ** 2).sum().backward()
        assert rel(host(x.detach()), host(x2.detach())) <= 1e-12, step
        assert rel(host(vals.grad), host(v2.grad)) <= 1e-10, step
        st2.close()
        del t2, st2, v2, x2
        with torch.no_grad():  # an optimizer-like step in place
            vals.add_(torch.from_numpy(1e-3 * rng.standard_normal(vals.numel())).to(dev))
            vals.grad = None
        torch.cuda.synchronize()
        free.append(torch.cuda.mem_get_info()[0])
    print(f"[loop] free device memory over the steps (MiB): {[f >> 20 for f in free]}")
    assert max(free[1:]) - min(free[1:]) <= 64 << 20
    # two solves on different values, then the first one's backward
    va = vals.detach().clone().requires_grad_(True)
    vb = (vals.detach() * 1.01).requires_grad_(True)
    xa = gad.lstsq(va, b, st, atol=1e-14, btol=1e-14)
    xb = gad.lstsq(vb, b, st, atol=1e-14, btol=1e-14)
    ((xa - xr) ** 2).sum().backward()
    ((xb - xr) ** 2).sum().backward()
    for v, xv in ((va, xa), (vb, xb)):
        t3, st3 = _structure(sysd, shape)
        v3 = v.detach().clone().requires_grad_(True)
        x3 = gad.lstsq(v3, b, st3, atol=1e-14, btol=1e-14)
        ((x3 - xr) ** 2).sum().backward()
        assert rel(host(xv.detach()), host(x3.detach())) <= 1e-12
        assert rel(host(v.grad), host(v3.grad)) <= 1e-10
        st3.close()
    st.close()
