"""torch.autograd Functions for the Wilson-Dirac apply and solve.

Gradients follow PyTorch's complex convention (grad = dL/dRe + i dL/dIm of a
real loss).  Every derivative is computed by the library's kernels:

WilsonApply  y = D psi
    grad_psi = D^dagger g          (dirac_apply with the adjoint hopping sign,
                                    equal to gamma5 D gamma5 g)
    grad_U   = link_force(g, psi, coeff = -1/2)
    grad_m0  = Re <g, psi>         (block_dot)
WilsonSolve  x = A^-1 eta, A = D (or D^dagger with dagger=True; batched GMRES)
    lambda   = A^-dagger g         (the adjoint solve: gmres_solve with the
                                    opposite dagger flag)
    grad_eta = lambda
    grad_U   = link_force(lambda, x, coeff = +1/2) for A = D; for A = D^dagger
               dL = -Re <lambda, dD^dagger x> = -Re <x, dD lambda>, i.e.
               link_force(x, lambda, coeff = +1/2)
    grad_m0  = -Re <lambda, x>     (dA/dm0 = 1 either way)

Blocks are FP64 full-lattice tensors in the rhs-innermost layout
[N0, N1, N2, N3, 4, 3, nrhs]; U is [4, N0, N1, N2, N3, 3, 3].
"""
from __future__ import annotations

import torch

from . import LAYOUT2, NOT_CONVERGED, block_dot, dirac_apply, gmres_solve, link_force


def _m0(m0):
    return float(m0.detach().cpu()) if isinstance(m0, torch.Tensor) else float(m0)


def _dims(U):
    return tuple(U.shape[1:5])


class WilsonApply(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, psi, m0):
        m = _m0(m0)
        ctx.m0 = m
        ctx.save_for_backward(U, psi)
        return dirac_apply(U.contiguous(), psi.contiguous(), m, layout=LAYOUT2)

    @staticmethod
    def backward(ctx, g):
        U, psi = ctx.saved_tensors
        g = g.contiguous()
        gU = gpsi = gm0 = None
        if ctx.needs_input_grad[1]:
            gpsi = dirac_apply(U, g, ctx.m0, layout=LAYOUT2, dagger=True)
        if ctx.needs_input_grad[0]:
            gU = link_force(U, g, psi, -0.5)
        if ctx.needs_input_grad[2]:
            gm0 = block_dot(g, psi, _dims(U)).real.sum()
        return gU, gpsi, gm0


class WilsonSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, U, eta, m0, params=None):
        m = _m0(m0)
        kw = dict(params or {})
        kw.setdefault("tol", 1e-10)
        x, st, rc = gmres_solve(U.contiguous(), eta.contiguous(), m, layout=LAYOUT2, **kw)
        if rc == NOT_CONVERGED:
            raise RuntimeError(f"WilsonSolve: GMRES did not converge (true residuals {st['true_relres']})")
        ctx.m0 = m
        ctx.kw = kw
        ctx.save_for_backward(U, x)
        return x

    @staticmethod
    def backward(ctx, g):
        U, x = ctx.saved_tensors
        kw = dict(ctx.kw)
        fwd_dagger = bool(kw.pop("dagger", False))
        kw.pop("x_is_guess", None)
        lam, st, rc = gmres_solve(U, g.contiguous(), ctx.m0, layout=LAYOUT2, dagger=not fwd_dagger, **kw)
        if rc == NOT_CONVERGED:
            raise RuntimeError(f"WilsonSolve backward: adjoint GMRES did not converge ({st['true_relres']})")
        gU = None
        if ctx.needs_input_grad[0]:
            gU = link_force(U, x, lam, 0.5) if fwd_dagger else link_force(U, lam, x, 0.5)
        gm0 = -block_dot(lam, x, _dims(U)).real.sum() if ctx.needs_input_grad[2] else None
        return gU, lam, gm0, None


def wilson_apply(U, psi, m0):
    return WilsonApply.apply(U, psi, m0)


def wilson_solve(U, eta, m0, **params):
    return WilsonSolve.apply(U, eta, m0, params)
