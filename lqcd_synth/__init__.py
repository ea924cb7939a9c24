"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module only draws random numbers and arranges them into gauge fields and
spinor blocks.  It holds none of the solver's arithmetic (no Dirac operator, no
projection, no Krylov step), so that the oracle and the HIP path can consume
the same arrays without sharing code.

Conventions (all arrays are numpy complex128, C order):

* lattice dims ``(N0, N1, N2, N3)`` with ``N0 = T`` slowest and ``N3`` fastest
  (the positional site numbering of Sec. III-A.1);
* gauge field ``U[mu, x0, x1, x2, x3, a, b]``: one 3x3 row-major colour matrix
  per direction and site, direction-major (Sec. III-A.1, storage of U_mu);
* spinor block ``psi[i, x0, x1, x2, x3, spin, colour]`` with one field per
  right-hand side ``i`` ("one column per rhs", eq. (1));
* random streams: ``numpy.random.default_rng([config, role, index])`` with
  role 0 = gauge field, 1 = source spinors, 2 = projection spinors (chi),
  3 = gauge transformation, 4 = batch composition draws, 5 = plane-wave
  polarisations, 6 = clover field.  Every rhs has its own stream, so any subset of right-hand
  sides can be regenerated on its own.
"""
from __future__ import annotations

import numpy as np

ROLE_GAUGE = 0
ROLE_SOURCE = 1
ROLE_CHI = 2
ROLE_GAUGE_TRANSFORM = 3
ROLE_BATCH = 4
ROLE_PLANE_WAVE = 5
ROLE_CLOVER = 6

# Gell-Mann matrices lambda_1..lambda_8 (standard normalisation tr(l_a l_b) = 2 delta_ab).
_GELL_MANN = np.zeros((8, 3, 3), dtype=np.complex128)
_GELL_MANN[0][0, 1] = _GELL_MANN[0][1, 0] = 1
_GELL_MANN[1][0, 1] = -1j
_GELL_MANN[1][1, 0] = 1j
_GELL_MANN[2][0, 0] = 1
_GELL_MANN[2][1, 1] = -1
_GELL_MANN[3][0, 2] = _GELL_MANN[3][2, 0] = 1
_GELL_MANN[4][0, 2] = -1j
_GELL_MANN[4][2, 0] = 1j
_GELL_MANN[5][1, 2] = _GELL_MANN[5][2, 1] = 1
_GELL_MANN[6][1, 2] = -1j
_GELL_MANN[6][2, 1] = 1j
_GELL_MANN[7][0, 0] = _GELL_MANN[7][1, 1] = 1 / np.sqrt(3)
_GELL_MANN[7][2, 2] = -2 / np.sqrt(3)


def gell_mann() -> np.ndarray:
    """The eight Gell-Mann matrices, shape (8, 3, 3)."""
    return _GELL_MANN.copy()


def rng(config: int, role: int, index: int = 0) -> np.random.Generator:
    return np.random.default_rng([int(config), int(role), int(index)])


def volume(dims) -> int:
    return int(np.prod(dims))


def _complex_normal(gen: np.random.Generator, shape) -> np.ndarray:
    """re and im drawn i.i.d. N(0, 1), real parts first, then imaginary parts."""
    re = gen.standard_normal(shape)
    im = gen.standard_normal(shape)
    return re + 1j * im


def haar_su3(gen: np.random.Generator, n: int) -> np.ndarray:
    """n Haar-distributed SU(3) matrices: QR of a complex Gaussian 3x3 matrix,
    phases of R's diagonal moved into Q (Mezzadri's fix), then the principal
    cube root of det Q divided out so that det U = 1."""
    z = _complex_normal(gen, (n, 3, 3))
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=-2, axis2=-1)
    q = q * (d / np.abs(d))[:, None, :]
    det = np.linalg.det(q)
    return q / (det ** (1.0 / 3.0))[:, None, None]


def near_identity_su3(gen: np.random.Generator, n: int, eps: float, chunk: int = 1 << 20) -> np.ndarray:
    """n matrices exp(i eps H), H = sum_a h_a lambda_a / 2 with h_a ~ N(0, 1),
    exponentiated through the eigen-decomposition of the Hermitian H."""
    h = gen.standard_normal((n, 8))
    out = np.empty((n, 3, 3), dtype=np.complex128)
    lam = _GELL_MANN / 2
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        hm = np.einsum("na,aij->nij", h[s:e], lam)
        hm = (hm + np.conj(np.swapaxes(hm, -1, -2))) / 2
        w, v = np.linalg.eigh(hm)
        ph = np.exp(1j * eps * w)
        out[s:e] = np.einsum("nik,nk,njk->nij", v, ph, np.conj(v))
    return out


def gauge_field(dims, kind: str, config: int, eps: float = 0.3, index: int = 0) -> np.ndarray:
    """Gauge field U[mu, x0..x3, a, b] drawn from stream (config, 0, index).

    kind = "haar" (uniform SU(3) links), "near_identity" (exp(i eps H)) or
    "unit" (U = 1, the free field)."""
    dims = tuple(int(d) for d in dims)
    v = volume(dims)
    if kind == "unit":
        u = np.broadcast_to(np.eye(3, dtype=np.complex128), (4 * v, 3, 3)).copy()
    elif kind == "haar":
        u = haar_su3(rng(config, ROLE_GAUGE, index), 4 * v)
    elif kind == "near_identity":
        u = near_identity_su3(rng(config, ROLE_GAUGE, index), 4 * v, eps)
    else:
        raise ValueError(f"unknown gauge field kind {kind!r}")
    return u.reshape((4,) + dims + (3, 3))


def gauge_transform(dims, config: int, index: int = 0) -> np.ndarray:
    """Random SU(3) matrix per site, G[x0..x3, a, b] (Haar), stream (config, 3, index)."""
    dims = tuple(int(d) for d in dims)
    return haar_su3(rng(config, ROLE_GAUGE_TRANSFORM, index), volume(dims)).reshape(dims + (3, 3))


def spinor_block(dims, nrhs: int, config: int, role: int = ROLE_SOURCE, first: int = 0,
                 dtype=np.complex128) -> np.ndarray:
    """Gaussian spinor block psi[i, x0..x3, spin, colour] for rhs first..first+nrhs-1.

    Right-hand side i is drawn from stream (config, role, i).  A complex64
    block is the complex128 draw rounded to single precision."""
    dims = tuple(int(d) for d in dims)
    out = np.empty((nrhs,) + dims + (4, 3), dtype=dtype)
    for k in range(nrhs):
        out[k] = _complex_normal(rng(config, role, first + k), dims + (4, 3))
    return out


def plane_wave_modes(dims, config: int, count: int = 1):
    """Random integer momenta n_mu in [0, N_mu) and unit 12-component
    polarisations u, drawn from stream (config, 5, k).  Returns a list of
    (n, u) with n an int array of 4 and u complex (4, 3)."""
    out = []
    for k in range(count):
        g = rng(config, ROLE_PLANE_WAVE, k)
        n = np.array([g.integers(0, d) for d in dims], dtype=np.int64)
        u = _complex_normal(g, (4, 3))
        out.append((n, u / np.linalg.norm(u)))
    return out


# Uneven batch of independent lattices (one per entry; L^3 x 2L with the
# spatial extents below), each with its own field strength and rhs count.
BATCH_L = (8, 12, 16, 20, 24, 12, 16, 20)


def batch_composition(config: int = 4):
    """List of dicts {dims, eps, nrhs, index} for the uneven multi-lattice batch:
    L from BATCH_L, T = 2L, eps_k = 0.2 + 0.3 k / 7, nrhs_k drawn uniformly in
    1..32 from stream (config, 4, k)."""
    out = []
    for k, L in enumerate(BATCH_L):
        nrhs = int(rng(config, ROLE_BATCH, k).integers(1, 33))
        out.append(dict(dims=(2 * L, L, L, L), eps=0.2 + 0.3 * k / 7, nrhs=nrhs, index=k))
    return out


def clover_field(dims, config: int, scale: float = 0.2, index: int = 0) -> np.ndarray:
    """Synthetic clover field, packed (N0, N1, N2, N3, 42) complex128: per site
    two Hermitian 6x6 blocks H = scale (Z + Z^dagger) / (2 sqrt 6) with Z a
    complex Gaussian 6x6 (stream (config, 6, index)), stored as each block's
    6 diagonal entries (real) then its 15 entries above the diagonal in
    row-major order.  Spectral radius about 2 scale, so (4 + m0) - C stays
    well away from singular for scale <= 0.5 and m0 > -1."""
    v = volume(dims)
    z = _complex_normal(rng(config, ROLE_CLOVER, index), (v, 2, 6, 6))
    h = scale * (z + np.conj(np.swapaxes(z, -1, -2))) / (2.0 * np.sqrt(6.0))
    out = np.zeros((v, 42), dtype=np.complex128)
    iu = np.triu_indices(6, 1)
    for b in range(2):
        out[:, 21 * b:21 * b + 6] = np.real(np.diagonal(h[:, b], axis1=-2, axis2=-1))
        out[:, 21 * b + 6:21 * b + 21] = h[:, b][:, iu[0], iu[1]]
    return out.reshape(tuple(dims) + (42,))
