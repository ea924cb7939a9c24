"""Odd-even (Schur complement) preconditioning (Sec. III-A.2, last paragraph).

Ordering sites as (even, odd), D = [[D_ee, D_eo], [D_oe, D_oo]] and the
even-site Schur complement is S = D_ee - D_eo D_oo^{-1} D_oe.  Reading taken:
"even" means parity 0 and the reduced system lives on even sites.  Without
a clover term the hopping part never connects two sites of equal parity, so
D_ee = D_oo = (4 + m0) I; the code below nevertheless evaluates every block
through the full operator D on vectors supported on one parity, so the block
structure is not assumed but applied.

Solving D x = b: b'_e = b_e - D_eo D_oo^{-1} b_o, solve S x_e = b'_e, then
x_o = D_oo^{-1} (b_o - D_oe x_e).

Compact vectors have shape (nrhs, V/2, 4, 3) in the order of
geometry.eo_sites.
"""
from __future__ import annotations

import numpy as np

from .dirac import apply_dw
from .geometry import from_half, to_half

EVEN, ODD = 0, 1


def _block(U, m0, half, src, dst):
    """D_{dst,src} applied to a compact parity-src vector."""
    dims = U.shape[1:5]
    return to_half(apply_dw(U, from_half(half, dims, src), m0), dims, dst)


def apply_schur(U: np.ndarray, psi_e: np.ndarray, m0: float) -> np.ndarray:
    """S psi_e = D_ee psi_e - D_eo D_oo^{-1} D_oe psi_e."""
    t_o = _block(U, m0, psi_e, EVEN, ODD) / (4.0 + m0)
    return _block(U, m0, psi_e, EVEN, EVEN) - _block(U, m0, t_o, ODD, EVEN)


def prepare_source(U: np.ndarray, b: np.ndarray, m0: float) -> np.ndarray:
    """b'_e = b_e - D_eo D_oo^{-1} b_o for a full-lattice block b."""
    dims = U.shape[1:5]
    b_e = to_half(b, dims, EVEN)
    b_o = to_half(b, dims, ODD)
    return b_e - _block(U, m0, b_o / (4.0 + m0), ODD, EVEN)


def reconstruct(U: np.ndarray, b: np.ndarray, x_e: np.ndarray, m0: float) -> np.ndarray:
    """Full solution from the even part: x_o = D_oo^{-1} (b_o - D_oe x_e)."""
    dims = U.shape[1:5]
    b_o = to_half(b, dims, ODD)
    x_o = (b_o - _block(U, m0, x_e, EVEN, ODD)) / (4.0 + m0)
    return from_half(x_e, dims, EVEN) + from_half(x_o, dims, ODD)
