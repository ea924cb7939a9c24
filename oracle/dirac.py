"""Wilson-Dirac operator on a block of right-hand sides (Sec. III-A.1).

D_W psi(x) = (4 + m0) psi(x)
             - 1/2 sum_mu [ (1 - gamma_mu) U_mu(x) psi(x + mu_hat)
                            + (1 + gamma_mu) U_mu(x - mu_hat)^dagger psi(x - mu_hat) ]

with lattice spacing a = 1, the projectors pi^{-+}_mu read as (1 -+ gamma_mu)/2
and no clover term (C = 0).  Algorithm 1 evaluates the same sum through
half-spinor projections and halo exchange; this oracle instead multiplies the
full 4x4 spin matrices, one direction at a time, so that nothing of the
projection trick is shared with the kernels.  Every right-hand side is treated
independently (the block form of eq. (1)).

Array shapes: U (4, N0, N1, N2, N3, 3, 3); psi (nrhs, N0, N1, N2, N3, 4, 3).
"""
from __future__ import annotations

import numpy as np

from .gamma import gammas, gamma5


def _shift_fwd(a: np.ndarray, mu: int, lead: int) -> np.ndarray:
    """out[x] = a[x + mu_hat] (periodic); lattice axes start at `lead`."""
    return np.roll(a, -1, axis=lead + mu)


def _shift_bwd(a: np.ndarray, mu: int, lead: int) -> np.ndarray:
    """out[x] = a[x - mu_hat] (periodic)."""
    return np.roll(a, 1, axis=lead + mu)


def _colour(u: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(U psi)_{s a} = sum_b U_{a b} psi_{s b}, per site and rhs."""
    return np.einsum("TZYXab,nTZYXsb->nTZYXsa", u, psi)


def _colour_dag(u: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(U^dagger psi)_{s a} = sum_b conj(U_{b a}) psi_{s b}."""
    return np.einsum("TZYXba,nTZYXsb->nTZYXsa", np.conj(u), psi)


def _spin(g: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(g psi)_{s a} = sum_t g_{s t} psi_{t a}."""
    return np.einsum("st,nTZYXta->nTZYXsa", g, psi)


def hopping(U: np.ndarray, psi: np.ndarray, sign: float = 1.0) -> np.ndarray:
    """H psi = sum_mu [ (1 - s gamma_mu) U_mu(x) psi(x+mu) + (1 + s gamma_mu) U_mu(x-mu)^dag psi(x-mu) ]
    with s = sign (s = +1 is the Wilson hopping term of D_W)."""
    g = gammas()
    one = np.eye(4, dtype=np.complex128)
    out = np.zeros(np.broadcast_shapes(psi.shape), dtype=np.result_type(U, psi))
    for mu in range(4):
        fwd = _colour(U[mu], _shift_fwd(psi, mu, 1))
        out += _spin((one - sign * g[mu]).astype(out.dtype), fwd)
        ub = _shift_bwd(U[mu], mu, 0)
        bwd = _colour_dag(ub, _shift_bwd(psi, mu, 1))
        out += _spin((one + sign * g[mu]).astype(out.dtype), bwd)
    return out


def apply_dw(U: np.ndarray, psi: np.ndarray, m0: float) -> np.ndarray:
    """eta = D_W psi for every rhs of the block."""
    return (4.0 + m0) * psi - 0.5 * hopping(U, psi, 1.0)


def apply_dw_dagger(U: np.ndarray, psi: np.ndarray, m0: float) -> np.ndarray:
    """eta = D_W^dagger psi, from the adjoint of each hopping term: the adjoint
    of psi -> (1-gamma) U(x) psi(x+mu) is g -> (1-gamma) U(x-mu)^dag g(x-mu),
    and of psi -> (1+gamma) U(x-mu)^dag psi(x-mu) it is g -> (1+gamma) U(x) g(x+mu).
    Both together are the hopping term with gamma_mu -> -gamma_mu."""
    return (4.0 + m0) * psi - 0.5 * hopping(U, psi, -1.0)


def apply_gamma5(psi: np.ndarray) -> np.ndarray:
    return _spin(gamma5().astype(psi.dtype), psi)


def dense(U: np.ndarray, m0: float) -> np.ndarray:
    """Dense matrix of D_W in the site-major, spin-major, colour-minor basis,
    assembled column by column from unit vectors (12 V x 12 V)."""
    dims = U.shape[1:5]
    n = 12 * int(np.prod(dims))
    eye = np.eye(n, dtype=np.complex128).reshape((n,) + tuple(dims) + (4, 3))
    cols = apply_dw(U, eye, m0).reshape(n, n)
    return cols.T.copy()


def apply_dw_sites(U: np.ndarray, psi: np.ndarray, m0: float, sites) -> np.ndarray:
    """(D_W psi) at the listed site numbers only, evaluated one site at a time
    from the definition (for checking a full-size result on a sample).
    Returns (nrhs, len(sites), 4, 3)."""
    dims = U.shape[1:5]
    g = gammas()
    one = np.eye(4, dtype=np.complex128)
    out = np.empty((psi.shape[0], len(sites), 4, 3), dtype=np.complex128)
    for k, s in enumerate(sites):
        x = np.array(np.unravel_index(int(s), dims))
        acc = (4.0 + m0) * psi[(slice(None),) + tuple(x)].astype(np.complex128)
        for mu in range(4):
            xp = x.copy(); xp[mu] = (xp[mu] + 1) % dims[mu]
            xm = x.copy(); xm[mu] = (xm[mu] - 1) % dims[mu]
            uf = U[(mu,) + tuple(x)]
            ub = U[(mu,) + tuple(xm)]
            fwd = np.einsum("ab,nsb->nsa", uf, psi[(slice(None),) + tuple(xp)])
            bwd = np.einsum("ba,nsb->nsa", np.conj(ub), psi[(slice(None),) + tuple(xm)])
            acc = acc - 0.5 * (np.einsum("st,nta->nsa", one - g[mu], fwd) + np.einsum("st,nta->nsa", one + g[mu], bwd))
        out[:, k] = acc
    return out
