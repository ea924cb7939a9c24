"""Gradients of the apply and of the solve (derived; the paper has no
differentiation).  Complex gradients follow PyTorch's convention
grad = dL/dRe z + i dL/dIm z, so that for a real loss dL = Re <grad, dz>.

Apply, y = D_W psi with upstream gradient g:
  grad_psi = D_W^dagger g,   grad_m0 = Re <g, psi>,
  grad_U_mu(x) = -1/2 sum_{rhs, spin} { [(1 - gamma_mu) g(x)] (x) psi(x + mu)^*
                                        + psi(x) (x) [(1 + gamma_mu) g(x + mu)]^* }
  where (x) is the colour outer product (a, b) -> p_a q_b^*.
Solve, x = D_W^{-1} eta with upstream gradient g:
  lambda = D_W^{-dagger} g,  grad_eta = lambda,  grad_m0 = -Re <lambda, x>,
  grad_U = -(apply gradient with g -> lambda, psi -> x).
su(3) force for left multiplication U -> exp(h Q) U, Q in su(3):
  F_mu(x) = TA(G_mu(x) U_mu(x)^dagger), TA(X) = (X - X^dag)/2 - tr(X - X^dag)/6 I,
  and dL/dh = Re tr(F^dagger Q).
"""
from __future__ import annotations

import numpy as np

from .gamma import gammas


def _spin(g, psi):
    return np.einsum("st,nTZYXta->nTZYXsa", g, psi)


def apply_link_grad(U: np.ndarray, g: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """grad_U of L with y = D_W psi and dL/dy = g (both blocks, summed over rhs)."""
    gm = gammas()
    one = np.eye(4, dtype=np.complex128)
    G = np.zeros_like(U)
    for mu in range(4):
        p = _spin(one - gm[mu], g)                       # (1 - gamma) g(x)
        q = np.roll(psi, -1, axis=1 + mu)                # psi(x + mu)
        G[mu] += -0.5 * np.einsum("nTZYXsa,nTZYXsb->TZYXab", p, np.conj(q))
        r = np.roll(_spin(one + gm[mu], g), -1, axis=1 + mu)   # (1 + gamma) g(x + mu)
        G[mu] += -0.5 * np.einsum("nTZYXsa,nTZYXsb->TZYXab", psi, np.conj(r))
    return G


def traceless_antihermitian(X: np.ndarray) -> np.ndarray:
    a = (X - np.conj(np.swapaxes(X, -1, -2))) / 2
    tr = np.trace(a, axis1=-2, axis2=-1)
    return a - (tr / 3)[..., None, None] * np.eye(3)


def su3_force(U: np.ndarray, G: np.ndarray) -> np.ndarray:
    """F = TA(G U^dagger) per link."""
    return traceless_antihermitian(G @ np.conj(np.swapaxes(U, -1, -2)))
