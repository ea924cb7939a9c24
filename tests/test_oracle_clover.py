"""Pins of the oracle's clover term (D = D_W - C, Sec. III-A.1): storage,
special cases that reduce to the plain operator, the chiral block structure,
gamma5-hermiticity, gauge covariance and the Schur complement with a
site-dependent D_oo, all against facts that do not go through the oracle's
own formulas."""
import numpy as np
import pytest

import lqcd_synth as syn
from oracle import clover, dirac, geometry
from oracle.gamma import gamma5


def _herm(gen, shape):
    z = gen.standard_normal(shape + (6, 6)) + 1j * gen.standard_normal(shape + (6, 6))
    return (z + np.conj(np.swapaxes(z, -1, -2))) / 2


def test_storage_roundtrip_and_hermitian():
    gen = np.random.default_rng(1)
    h = _herm(gen, (5, 2))
    np.testing.assert_array_equal(clover.unpack(clover.pack(h)), h)
    cp = syn.clover_field((2, 2, 2, 2), config=1)
    b = clover.unpack(cp)
    np.testing.assert_array_equal(b, np.conj(np.swapaxes(b, -1, -2)))
    np.testing.assert_array_equal(clover.pack(b), cp)
    # diagonal first, then the upper triangle row by row
    one = np.zeros(42, dtype=np.complex128)
    one[21 + 6 + 5] = 2 + 3j  # block 1, 6th upper entry = (1, 2)
    m = clover.unpack(one)
    assert m[1, 1, 2] == 2 + 3j and m[1, 2, 1] == 2 - 3j and np.count_nonzero(m) == 2


def test_zero_clover_is_wilson():
    dims = (4, 4, 2, 2)
    U = syn.gauge_field(dims, "haar", config=2)
    psi = syn.spinor_block(dims, 2, config=2)
    cp = np.zeros(dims + (42,), dtype=np.complex128)
    np.testing.assert_array_equal(clover.apply_dwc(U, cp, psi, 0.1), dirac.apply_dw(U, psi, 0.1))


def test_constant_clover_shifts_the_mass():
    """C = c I on every site: D_W(m0) - c = D_W(m0 - c)."""
    dims = (4, 2, 4, 2)
    U = syn.gauge_field(dims, "haar", config=3)
    psi = syn.spinor_block(dims, 3, config=3)
    c = 0.37
    cp = np.zeros(dims + (42,), dtype=np.complex128)
    cp[..., 0:6] = c
    cp[..., 21:27] = c
    want = dirac.apply_dw(U, psi, 0.1 - c)
    got = clover.apply_dwc(U, cp, psi, 0.1)
    assert np.abs(got - want).max() <= 1e-14 * np.abs(want).max()


def test_blocks_act_on_spin_pairs():
    """Block 0 mixes spins (0, 1) with colour, block 1 spins (2, 3); a block
    acts on the 6-vector (spin-in-pair, colour) = 3 s + c."""
    dims = (2, 2, 2, 2)
    gen = np.random.default_rng(4)
    blk = np.zeros(dims + (2, 6, 6), dtype=np.complex128)
    blk[..., 0, :, :] = _herm(gen, dims)
    cp = clover.pack(blk)
    psi = syn.spinor_block(dims, 1, config=4)
    lower = psi.copy()
    lower[..., 0:2, :] = 0
    assert np.abs(clover.apply_clover(cp, lower)).max() == 0.0
    upper = psi.copy()
    upper[..., 2:4, :] = 0
    out = clover.apply_clover(cp, upper)
    assert np.abs(out[..., 2:4, :]).max() == 0.0
    x = (1, 0, 1, 1)
    v = upper[(0,) + x][0:2].reshape(6)
    np.testing.assert_allclose(out[(0,) + x][0:2].reshape(6), blk[x][0] @ v, rtol=1e-14, atol=1e-14)


def test_gamma5_hermiticity_dense():
    dims = (2, 2, 2, 2)
    U = syn.gauge_field(dims, "haar", config=5)
    cp = syn.clover_field(dims, config=5, scale=0.4)
    D = clover.dense(U, cp, 0.2)
    g5 = np.kron(np.eye(int(np.prod(dims))), np.kron(gamma5(), np.eye(3)))
    assert np.linalg.norm(g5 @ D @ g5 - D.conj().T) <= 1e-14 * np.linalg.norm(D)
    # the adjoint apply agrees with the dense conjugate transpose
    psi = syn.spinor_block(dims, 1, config=6)
    got = clover.apply_dwc_dagger(U, cp, psi, 0.2).reshape(-1)
    np.testing.assert_allclose(got, D.conj().T @ psi.reshape(-1), rtol=1e-13, atol=1e-13)


def test_gauge_covariance():
    """U^G_mu(x) = G(x) U_mu(x) G(x+mu)^dag and C^G(x) = (1 x G(x)) C(x) (1 x G(x))^dag
    on each block: D[U^G, C^G] (G psi) = G D[U, C] psi."""
    dims = (4, 2, 2, 4)
    U = syn.gauge_field(dims, "haar", config=7)
    cp = syn.clover_field(dims, config=7, scale=0.3)
    G = syn.gauge_transform(dims, config=7)
    psi = syn.spinor_block(dims, 2, config=7)
    UG = np.empty_like(U)
    for mu in range(4):
        Gf = np.roll(G, -1, axis=mu)
        UG[mu] = G @ U[mu] @ np.conj(np.swapaxes(Gf, -1, -2))
    big = np.zeros(dims + (6, 6), dtype=np.complex128)
    big[..., 0:3, 0:3] = G
    big[..., 3:6, 3:6] = G
    blk = clover.unpack(cp)
    blkG = big[..., None, :, :] @ blk @ np.conj(np.swapaxes(big, -1, -2))[..., None, :, :]
    cpG = clover.pack(blkG)
    Gpsi = np.einsum("TZYXab,nTZYXsb->nTZYXsa", G, psi)
    lhs = clover.apply_dwc(UG, cpG, Gpsi, -0.1)
    rhs = np.einsum("TZYXab,nTZYXsb->nTZYXsa", G, clover.apply_dwc(U, cp, psi, -0.1))
    assert np.abs(lhs - rhs).max() <= 1e-13 * np.abs(rhs).max()


def test_diagonal_inverse():
    dims = (2, 2, 2, 2)
    cp = syn.clover_field(dims, config=8, scale=0.5)
    inv = clover.unpack(clover.diagonal_inverse(cp, -0.4))
    m = 3.6 * np.eye(6) - clover.unpack(cp)
    np.testing.assert_allclose(inv @ m, np.broadcast_to(np.eye(6), m.shape), atol=1e-14)


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 2, 2)])
def test_schur_complement_block_lu_dense(dims):
    """Even/odd blocks of the dense D: S = D_ee - D_eo D_oo^{-1} D_oe with a
    site-dependent D_oo; prepare + Schur solve + reconstruct = dense solve."""
    U = syn.gauge_field(dims, "haar", config=9)
    cp = syn.clover_field(dims, config=9, scale=0.4)
    m0 = 0.1
    D = clover.dense(U, cp, m0)
    eo = geometry.eo_sites(dims)
    idx = [np.concatenate([12 * s + np.arange(12) for s in eo[p]]) for p in (0, 1)]
    Dee, Deo = D[np.ix_(idx[0], idx[0])], D[np.ix_(idx[0], idx[1])]
    Doe, Doo = D[np.ix_(idx[1], idx[0])], D[np.ix_(idx[1], idx[1])]
    S = Dee - Deo @ np.linalg.solve(Doo, Doe)
    v = syn.spinor_block(dims, 2, config=10)
    ve = geometry.to_half(v, dims, 0)
    got = clover.apply_schur(U, cp, ve, m0).reshape(2, -1)
    want = (S @ ve.reshape(2, -1).T).T
    assert np.abs(got - want).max() <= 1e-13 * np.abs(want).max()
    b = syn.spinor_block(dims, 1, config=11)
    x = np.linalg.solve(D, b.reshape(-1)).reshape(b.shape)
    bp = clover.prepare_source(U, cp, b, m0)
    xe = np.linalg.solve(S, bp.reshape(-1)).reshape(bp.shape)
    full = clover.reconstruct(U, cp, b, xe, m0)
    assert np.abs(full - x).max() <= 1e-12 * np.abs(x).max()
