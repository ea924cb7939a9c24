"""Closed forms used to pin the apply (derived from the operator's definition,
not from any implementation of it).

Free field (U = 1): a plane wave psi(x) = exp(i p.x) u with p_mu = 2 pi n_mu / N_mu
and a 4x3 spin-colour amplitude u is mapped by D_W to exp(i p.x) M(p) u with the
4x4 spin symbol
    M(p) = (4 + m0) - sum_mu cos p_mu + i sum_mu gamma_mu sin p_mu,
since the forward hop contributes -1/2 (1 - gamma_mu) e^{i p_mu} and the backward
hop -1/2 (1 + gamma_mu) e^{-i p_mu}.  M(p) has the eigenvalues
m0 + sum_mu (1 - cos p_mu) +- i (sum_mu sin^2 p_mu)^{1/2}, each six-fold
(two spins x three colours).

Pure gauge U_mu(x) = G(x) G(x + mu)^dagger: psi(x) = G(x) exp(i p.x) u is mapped
to G(x) exp(i p.x) M(p) u, at any lattice size.

Free Schur complement: with h(p) = -sum cos p_mu + i sum gamma_mu sin p_mu the
hopping symbol, h(p + (pi,pi,pi,pi)) = -h(p), and the even projection of a
plane wave mixes p with p + pi; the Schur complement on even sites then acts on
P_e exp(i p.x) u as multiplication by (4 + m0) - h(p)^2 / (4 + m0).
"""
from __future__ import annotations

import numpy as np

from .gamma import gammas


def momenta(n, dims) -> np.ndarray:
    return 2 * np.pi * np.asarray(n, dtype=np.float64) / np.asarray(dims, dtype=np.float64)


def free_symbol(p, m0: float) -> np.ndarray:
    g = gammas()
    M = (4.0 + m0 - np.sum(np.cos(p))) * np.eye(4, dtype=np.complex128)
    for mu in range(4):
        M = M + 1j * np.sin(p[mu]) * g[mu]
    return M


def hopping_symbol(p) -> np.ndarray:
    g = gammas()
    h = -np.sum(np.cos(p)) * np.eye(4, dtype=np.complex128)
    for mu in range(4):
        h = h + 1j * np.sin(p[mu]) * g[mu]
    return h


def free_eigenvalues(p, m0: float) -> np.ndarray:
    re = m0 + np.sum(1 - np.cos(p))
    im = np.sqrt(np.sum(np.sin(p) ** 2))
    return np.array([re + 1j * im, re - 1j * im])


def plane_wave(dims, p, u) -> np.ndarray:
    """exp(i p.x) u on the lattice, shape (N0, N1, N2, N3, 4, 3)."""
    grids = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    phase = np.exp(1j * sum(p[mu] * grids[mu] for mu in range(4)))
    return phase[..., None, None] * u


def pure_gauge_links(G: np.ndarray) -> np.ndarray:
    """U_mu(x) = G(x) G(x + mu)^dagger for a site field G (N0..N3, 3, 3)."""
    out = np.empty((4,) + G.shape, dtype=np.complex128)
    for mu in range(4):
        Gp = np.roll(G, -1, axis=mu)
        out[mu] = G @ np.conj(np.swapaxes(Gp, -1, -2))
    return out


def colour_rotate(G: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(G psi)(x)_{s a} = sum_b G(x)_{ab} psi(x)_{s b} for psi (..., N0..N3, 4, 3)."""
    return np.einsum("TZYXab,...TZYXsb->...TZYXsa", G, psi)
