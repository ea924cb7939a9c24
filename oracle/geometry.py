"""Lattice geometry (Sec. III-A.1, site numbering).

A lattice of size N0 x N1 x N2 x N3 numbers site (x0, x1, x2, x3) with the
positional system whose strides are the extents of the faster dimensions:
idx = ((x0*N1 + x1)*N2 + x2)*N3 + x3.  (The printed stride formula is garbled;
this mixed-radix form is the reading taken, and it equals the printed one when
N1 = N2 = N3.)  N0 is time.  Boundaries are periodic in all four directions.

Neighbour table columns: 0..3 hold x + mu_hat for mu = 0..3, 4..7 hold
x - mu_hat.  Parity of a site is (x0 + x1 + x2 + x3) mod 2; parity 0 is
"even".  The odd-even compact list of parity p holds the sites of that parity
in ascending site number.
"""
from __future__ import annotations

import numpy as np


def check_dims(dims):
    dims = tuple(int(d) for d in dims)
    if len(dims) != 4 or any(d < 2 or d % 2 for d in dims):
        raise ValueError(f"lattice extents must be four even numbers >= 2, got {dims}")
    return dims


def site_index(coords, dims) -> np.ndarray:
    """Site number of coordinates (..., 4)."""
    c = np.asarray(coords, dtype=np.int64)
    n0, n1, n2, n3 = dims
    return ((c[..., 0] * n1 + c[..., 1]) * n2 + c[..., 2]) * n3 + c[..., 3]


def coordinates(dims) -> np.ndarray:
    """Coordinates (V, 4) of every site in site-number order."""
    dims = check_dims(dims)
    grids = np.meshgrid(*[np.arange(d) for d in dims], indexing="ij")
    return np.stack([g.reshape(-1) for g in grids], axis=-1).astype(np.int64)


def neighbour_table(dims) -> np.ndarray:
    """int32 (V, 8): site numbers of x + mu_hat (cols 0..3) and x - mu_hat (cols 4..7)."""
    dims = check_dims(dims)
    c = coordinates(dims)
    out = np.empty((c.shape[0], 8), dtype=np.int64)
    for mu in range(4):
        for sgn, col in ((+1, mu), (-1, 4 + mu)):
            s = c.copy()
            s[:, mu] = (s[:, mu] + sgn) % dims[mu]
            out[:, col] = site_index(s, dims)
    return out.astype(np.int32)


def parity(dims) -> np.ndarray:
    """int32 (V,): (x0+x1+x2+x3) mod 2 per site."""
    return (coordinates(dims).sum(axis=1) % 2).astype(np.int32)


def eo_sites(dims) -> np.ndarray:
    """int32 (2, V/2): row p lists the sites of parity p in ascending order."""
    p = parity(dims)
    even = np.nonzero(p == 0)[0]
    odd = np.nonzero(p == 1)[0]
    return np.stack([even, odd]).astype(np.int32)


def to_half(field: np.ndarray, dims, p: int) -> np.ndarray:
    """Restrict a block (nrhs, N0, N1, N2, N3, 4, 3) to the parity-p sites,
    giving (nrhs, V/2, 4, 3) in compact order."""
    v = int(np.prod(dims))
    flat = field.reshape((field.shape[0], v) + field.shape[5:])
    return flat[:, eo_sites(dims)[p]]


def from_half(half: np.ndarray, dims, p: int) -> np.ndarray:
    """Embed a compact parity-p block (nrhs, V/2, 4, 3) into the full lattice
    (zeros on the other parity)."""
    v = int(np.prod(dims))
    out = np.zeros((half.shape[0], v) + half.shape[2:], dtype=half.dtype)
    out[:, eo_sites(dims)[p]] = half
    return out.reshape((half.shape[0],) + tuple(dims) + half.shape[2:])
