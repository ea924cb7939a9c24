"""Euclidean gamma matrices (Sec. III-A.1 projectors pi^{+-}_mu).

The paper does not print a gamma basis; the reading taken is the chiral basis
gamma_mu = [[0, B_mu], [B_mu^dagger, 0]] with B_0 = I_2 (mu = 0, time) and
B_k = -i sigma_k (mu = k = 1, 2, 3).  These are Hermitian, satisfy
{gamma_mu, gamma_nu} = 2 delta_{mu nu}, and gamma_5 = gamma_1 gamma_2 gamma_3
gamma_0 = diag(1, 1, -1, -1).  Every property the solver relies on
(gamma_5-hermiticity, the projector algebra) is basis independent.

The spin-colour index of a site is spin-major: component 3*spin + colour.
"""
from __future__ import annotations

import numpy as np

_SIGMA = (
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
)


def _block(b: np.ndarray) -> np.ndarray:
    g = np.zeros((4, 4), dtype=np.complex128)
    g[0:2, 2:4] = b
    g[2:4, 0:2] = b.conj().T
    return g


def gammas() -> np.ndarray:
    """(4, 4, 4): gamma_0 .. gamma_3."""
    bs = [np.eye(2, dtype=np.complex128)] + [-1j * s for s in _SIGMA]
    return np.stack([_block(b) for b in bs])


def gamma5() -> np.ndarray:
    g = gammas()
    return g[1] @ g[2] @ g[3] @ g[0]
