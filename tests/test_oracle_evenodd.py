"""Pins for the oracle's odd-even preconditioning: the dense block-LU
identity, the free-field Schur symbol, and full solve = Schur solve +
reconstruction."""
import numpy as np
import pytest

import lqcd_synth as syn
from oracle import closed_forms as cf
from oracle import dirac, evenodd, geometry


def _perm(dims):
    """Row permutation of the dense D into (even sites, odd sites) order."""
    eo = geometry.eo_sites(dims)
    sites = np.concatenate([eo[0], eo[1]])
    return (sites[:, None] * 12 + np.arange(12)[None]).reshape(-1)


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 2, 2)])
def test_block_lu_identity(dims):
    m0 = 0.1
    U = syn.gauge_field(dims, "haar", config=11)
    D = dirac.dense(U, m0)
    P = _perm(dims)
    Dp = D[np.ix_(P, P)]
    h = Dp.shape[0] // 2
    Dee, Deo, Doe, Doo = Dp[:h, :h], Dp[:h, h:], Dp[h:, :h], Dp[h:, h:]
    # no clover: the diagonal blocks are multiples of the identity
    assert np.allclose(Dee, (4 + m0) * np.eye(h), atol=1e-15)
    assert np.allclose(Doo, (4 + m0) * np.eye(h), atol=1e-15)
    S_dense = Dee - Deo @ np.linalg.inv(Doo) @ Doe
    # block LU: D = [[1, Deo Doo^-1], [0, 1]] diag(S, Doo) [[1, 0], [Doo^-1 Doe, 1]]
    I = np.eye(h)
    L = np.block([[I, Deo @ np.linalg.inv(Doo)], [0 * I, I]])
    R = np.block([[I, 0 * I], [np.linalg.inv(Doo) @ Doe, I]])
    Mid = np.block([[S_dense, 0 * I], [0 * I, Doo]])
    assert np.allclose(L @ Mid @ R, Dp, atol=1e-13)
    # the oracle's Schur apply, column by column
    eye = np.eye(h, dtype=np.complex128).reshape(h, h // 12, 4, 3)
    S_or = evenodd.apply_schur(U, eye, m0).reshape(h, h).T
    assert np.allclose(S_or, S_dense, atol=1e-13)


def test_free_schur_symbol():
    dims = (4, 4, 4, 8)
    m0 = -0.05
    U = syn.gauge_field(dims, "unit", config=0)
    for n, u in syn.plane_wave_modes(dims, config=12, count=3):
        p = cf.momenta(n, dims)
        wave = cf.plane_wave(dims, p, u)[None]
        psi_e = geometry.to_half(wave, dims, 0)
        h = cf.hopping_symbol(p)
        sym = (4 + m0) * np.eye(4) - h @ h / (4 + m0)
        want = geometry.to_half(cf.plane_wave(dims, p, sym @ u)[None], dims, 0)
        assert np.max(np.abs(evenodd.apply_schur(U, psi_e, m0) - want)) < 1e-13
        # h(p + pi) = -h(p)
        assert np.allclose(cf.hopping_symbol(p + np.pi), -h, atol=1e-14)


def test_prepare_reconstruct_solves_full_system():
    dims = (4, 4, 2, 2)
    m0 = 0.1
    U = syn.gauge_field(dims, "haar", config=13)
    b = syn.spinor_block(dims, 2, config=13)
    D = dirac.dense(U, m0)
    x_ref = np.linalg.solve(D, b.reshape(2, -1).T).T.reshape(b.shape)
    # exact Schur solve through the dense Schur matrix
    h = D.shape[0] // 2
    eye = np.eye(h, dtype=np.complex128).reshape(h, h // 12, 4, 3)
    S = evenodd.apply_schur(U, eye, m0).reshape(h, h).T
    bp = evenodd.prepare_source(U, b, m0)
    xe = np.linalg.solve(S, bp.reshape(2, -1).T).T.reshape(bp.shape)
    x = evenodd.reconstruct(U, b, xe, m0)
    assert np.max(np.abs(x - x_ref)) < 1e-12
    # reconstruction zeroes the odd rows of the residual for any x_e
    xe_bad = xe + 0.1 * syn.spinor_block(dims, 2, config=14).reshape(2, -1)[:, : h].reshape(xe.shape)
    r = b - dirac.apply_dw(U, evenodd.reconstruct(U, b, xe_bad, m0), m0)
    assert np.max(np.abs(geometry.to_half(r, dims, 1))) < 1e-13
    assert np.allclose(geometry.to_half(r, dims, 0), bp - evenodd.apply_schur(U, xe_bad, m0), atol=1e-12)
