"""Differentiation through the least-squares solve x* = argmin ||A x - b|| (PC-LSQR).

Forward: the library's PC-LSQR (binary64) run to convergence.
Backward, for g = dL/dx*: differentiating the normal equations A^T A x = A^T b gives
    dL/db    = mu,            mu  = minimum-norm solution of A^T mu = g (= A (A^T A)^-1 g),
    dL/dA_ic = r_i lam_c - mu_i x*_c,  r = b - A x*,  lam = (A^T A)^-1 g = argmin ||A lam - mu||,
restricted to the stored pattern.  mu and lam come from two LSQR solves on the same product
kernels (gsr_lsqr_solve_adjoint); the pattern gradient from gsr_grad_vals.  All arithmetic
runs in the HIP library; this module only marshals tensors.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import torch

from . import gsr


@dataclass
class Structure:
    """Index map of a system (Section 3): star number, attitude start and instrumental
    indices per row, as int32 CUDA tensors, plus the section sizes.

    The structure owns one library handle, set up at the first solve and reused after it:
    every later solve brings its coefficients into the handle with gsr_update_values (the
    handle's copies and preconditioner rebuilt in place, no sort, no allocation) -- whether
    they changed or not cannot be told reliably (writes through .data leave no trace) -- and a
    backward pass does the same when another solve used the handle after its forward.
    close() releases the handle; so does dropping the structure."""

    star: torch.Tensor
    att: torch.Tensor
    instr: torch.Tensor
    n_stars: int
    n_dfa: int
    n_instr: int
    _handle: gsr.Handle | None = field(default=None, init=False, repr=False)
    _gen: int = field(default=0, init=False, repr=False)  # solves that loaded values
    _vals: torch.Tensor | None = field(default=None, init=False, repr=False)

    @property
    def n_rows(self) -> int:
        return self.star.numel()

    @property
    def n_cols(self) -> int:
        return 5 * self.n_stars + 3 * self.n_dfa + self.n_instr + 1

    def dims(self) -> gsr.Dims:
        return gsr.make_dims(self.n_rows, self.n_stars, self.n_dfa, self.n_instr)

    def load(self, vals: torch.Tensor) -> int:
        """Bring the coefficients `vals` (contiguous float64 CUDA tensor) into the handle
        (set up at the first call); returns the generation that identifies this load.  The
        tensor is referenced, not copied: the structure keeps it alive while it is loaded."""
        if self._handle is None:
            self._handle = gsr.gsr_lsqr_setup(self.dims(), vals, self.star, self.att,
                                              self.instr, allow_empty_cols=True)
        else:
            gsr.gsr_update_values(self._handle, vals)
        self._vals = vals
        self._gen += 1
        return self._gen

    def handle(self, vals: torch.Tensor | None = None, gen: int | None = None) -> gsr.Handle:
        """The handle; with `vals` and the generation `gen` of an earlier load, the values
        are loaded again unless that load is still the current one."""
        if vals is not None and (self._handle is None or gen != self._gen):
            self.load(vals)
        return self._handle

    def close(self):
        if self._handle is not None:
            self._handle.close()
        self._handle, self._vals = None, None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class LstsqSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, vals, b, structure: Structure, itnlim: int, atol: float, btol: float):
        vals_c = vals.detach().contiguous()
        b_c = b.detach().contiguous()
        ctx.gen = structure.load(vals_c)
        h = structure.handle()
        opts = gsr.solve_opts(itnlim=itnlim, fixed_iters=False, atol=atol, btol=btol)
        x = torch.empty(structure.n_cols, dtype=torch.float64, device=vals.device)
        info = gsr.gsr_lsqr_solve(h, b_c, x, opts)
        ctx.structure = structure
        ctx.opts = opts
        ctx.info = info
        ctx.save_for_backward(vals_c, b_c, x)
        return x

    @staticmethod
    def backward(ctx, g):
        vals_c, b_c, x = ctx.saved_tensors
        # the coefficients of this forward, loaded again if another solve used the handle since
        h = ctx.structure.handle(vals_c, ctx.gen)
        g = g.detach().contiguous().to(torch.float64)
        m, n = h.m, h.n
        mu = torch.empty(m, dtype=torch.float64, device=g.device)
        lam = torch.empty(n, dtype=torch.float64, device=g.device)
        gsr.gsr_lsqr_solve_adjoint(h, g, mu, lam, ctx.opts)
        grad_vals = None
        if ctx.needs_input_grad[0]:
            r = torch.empty(m, dtype=torch.float64, device=g.device)
            gsr.gsr_residual(h, b_c, x, r)
            grad_vals = torch.empty(24 * m, dtype=torch.float64, device=g.device)
            gsr.gsr_grad_vals(h, r, mu, x, lam, grad_vals)
        grad_b = mu if ctx.needs_input_grad[1] else None
        return grad_vals, grad_b, None, None, None, None


def lstsq(vals: torch.Tensor, b: torch.Tensor, structure: Structure, itnlim: int = 5000,
          atol: float = 1e-15, btol: float = 1e-15) -> torch.Tensor:
    """x* = argmin ||A x - b|| for the matrix with stored coefficients `vals` ([n_rows*24],
    float64, CUDA) and index map `structure`; differentiable in vals and b."""
    return LstsqSolve.apply(vals, b, structure, itnlim, atol, btol)
