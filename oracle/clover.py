"""Clover term of the improved Wilson-Dirac operator.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU baseline, never by the library path.

The improved operator (Sec. III-A.1, the equation after eq. (1)) is

    D psi(x) = D_W psi(x) - C(x) psi(x),

and Algorithm 1 applies C in its first line together with the diagonal
(4 + m0).  Sec. III-A.1 (the paragraph on the projections) states that C(x)
is block-diagonal with Hermitian blocks, 42 complex numbers per site.
Readings taken (the paper does not spell them out):

* the two blocks act on the spin pairs (0, 1) and (2, 3) of the chiral basis
  (the pairs gamma5 = diag(1, 1, -1, -1) keeps apart), each a Hermitian 6x6
  matrix in the (spin-in-pair, colour) index 3 s + c;
* storage per site: block 0 then block 1, each as its 6 diagonal entries
  followed by the 15 entries above the diagonal in row-major order
  ((0,1), (0,2), ..., (0,5), (1,2), ..., (4,5)), 21 complex numbers per
  block; the imaginary parts of the diagonal entries are not used;
* C is an input field (the paper never derives it from U here).

Array shapes: packed C (N0, N1, N2, N3, 42); psi (nrhs, N0, N1, N2, N3, 4, 3).
"""
from __future__ import annotations

import numpy as np

from .dirac import apply_dw, apply_dw_dagger
from .geometry import from_half, to_half

EVEN, ODD = 0, 1
_UPPER = [(i, j) for i in range(6) for j in range(i + 1, 6)]


def unpack(cp: np.ndarray) -> np.ndarray:
    """Packed (..., 42) -> Hermitian blocks (..., 2, 6, 6)."""
    lead = cp.shape[:-1]
    out = np.zeros(lead + (2, 6, 6), dtype=np.complex128)
    for b in range(2):
        base = 21 * b
        for i in range(6):
            out[..., b, i, i] = cp[..., base + i].real
        for k, (i, j) in enumerate(_UPPER):
            out[..., b, i, j] = cp[..., base + 6 + k]
            out[..., b, j, i] = np.conj(cp[..., base + 6 + k])
    return out


def pack(blocks: np.ndarray) -> np.ndarray:
    """Hermitian blocks (..., 2, 6, 6) -> packed (..., 42)."""
    lead = blocks.shape[:-3]
    out = np.zeros(lead + (42,), dtype=np.complex128)
    for b in range(2):
        base = 21 * b
        for i in range(6):
            out[..., base + i] = blocks[..., b, i, i].real
        for k, (i, j) in enumerate(_UPPER):
            out[..., base + 6 + k] = blocks[..., b, i, j]
    return out


def site_matrix(cp: np.ndarray) -> np.ndarray:
    """The 12x12 matrix C(x) in the spin-major, colour-minor site basis
    (index 3 spin + colour): block 0 on components 0..5, block 1 on 6..11."""
    blk = unpack(cp)
    out = np.zeros(cp.shape[:-1] + (12, 12), dtype=np.complex128)
    out[..., 0:6, 0:6] = blk[..., 0, :, :]
    out[..., 6:12, 6:12] = blk[..., 1, :, :]
    return out


def apply_clover(cp: np.ndarray, psi: np.ndarray) -> np.ndarray:
    """(C psi)(x) = C(x) psi(x) for every rhs."""
    m = site_matrix(cp)
    v = psi.reshape(psi.shape[:-2] + (12,))
    return np.einsum("TZYXij,nTZYXj->nTZYXi", m, v).reshape(psi.shape)


def apply_dwc(U: np.ndarray, cp: np.ndarray, psi: np.ndarray, m0: float) -> np.ndarray:
    """D psi = D_W psi - C psi."""
    return apply_dw(U, psi, m0) - apply_clover(cp, psi)


def apply_dwc_dagger(U: np.ndarray, cp: np.ndarray, psi: np.ndarray, m0: float) -> np.ndarray:
    """D^dagger psi = D_W^dagger psi - C psi (C is Hermitian)."""
    return apply_dw_dagger(U, psi, m0) - apply_clover(cp, psi)


def diagonal_inverse(cp: np.ndarray, m0: float) -> np.ndarray:
    """Packed blocks of ((4 + m0) I - C(x))^{-1}, the site-local part of D
    inverted site by site (Hermitian, so the same storage applies)."""
    blk = unpack(cp)
    eye = np.eye(6, dtype=np.complex128)
    return pack(np.linalg.inv((4.0 + m0) * eye - blk))


def _apply_site_inverse(cp_half: np.ndarray, m0: float, v: np.ndarray) -> np.ndarray:
    """Solve ((4 + m0) I - C(x)) y(x) = v(x) site by site on compact vectors
    v (nrhs, V/2, 4, 3) with cp_half (V/2, 42)."""
    m = (4.0 + m0) * np.eye(12, dtype=np.complex128) - site_matrix(cp_half)
    rhs = v.reshape(v.shape[0], v.shape[1], 12)
    y = np.linalg.solve(m[None], rhs[..., None])[..., 0]
    return y.reshape(v.shape)


def _block(U, cp, m0, half, src, dst):
    """D_{dst,src} applied to a compact parity-src vector (through the full D)."""
    dims = U.shape[1:5]
    return to_half(apply_dwc(U, cp, from_half(half, dims, src), m0), dims, dst)


def _cp_half(cp: np.ndarray, p: int) -> np.ndarray:
    dims = cp.shape[:4]
    return to_half(cp.reshape((1,) + dims + (42, 1)), dims, p).reshape(-1, 42)


def apply_schur(U: np.ndarray, cp: np.ndarray, psi_e: np.ndarray, m0: float) -> np.ndarray:
    """S psi_e = D_ee psi_e - D_eo D_oo^{-1} D_oe psi_e (Sec. III-A.2), with
    D_oo = (4 + m0) - C on odd sites inverted site by site."""
    t_o = _apply_site_inverse(_cp_half(cp, ODD), m0, _block(U, cp, m0, psi_e, EVEN, ODD))
    return _block(U, cp, m0, psi_e, EVEN, EVEN) - _block(U, cp, m0, t_o, ODD, EVEN)


def prepare_source(U: np.ndarray, cp: np.ndarray, b: np.ndarray, m0: float) -> np.ndarray:
    """b'_e = b_e - D_eo D_oo^{-1} b_o."""
    dims = U.shape[1:5]
    b_e = to_half(b, dims, EVEN)
    t_o = _apply_site_inverse(_cp_half(cp, ODD), m0, to_half(b, dims, ODD))
    return b_e - _block(U, cp, m0, t_o, ODD, EVEN)


def reconstruct(U: np.ndarray, cp: np.ndarray, b: np.ndarray, x_e: np.ndarray, m0: float) -> np.ndarray:
    """x_o = D_oo^{-1} (b_o - D_oe x_e); returns the full-lattice solution."""
    dims = U.shape[1:5]
    x_o = _apply_site_inverse(_cp_half(cp, ODD), m0, to_half(b, dims, ODD) - _block(U, cp, m0, x_e, EVEN, ODD))
    return from_half(x_e, dims, EVEN) + from_half(x_o, dims, ODD)


def dense(U: np.ndarray, cp: np.ndarray, m0: float) -> np.ndarray:
    """Dense matrix of D = D_W - C, column by column (12 V x 12 V)."""
    dims = U.shape[1:5]
    n = 12 * int(np.prod(dims))
    eye = np.eye(n, dtype=np.complex128).reshape((n,) + tuple(dims) + (4, 3))
    return apply_dwc(U, cp, eye, m0).reshape(n, n).T.copy()
