"""Pins for the oracle's Wilson-Dirac apply (Sec. III-A.1): gamma algebra,
field generation, gamma5-hermiticity, gauge covariance, free-field and
pure-gauge plane waves, the 2^4 spectrum, and a per-site loop evaluation."""
from math import comb

import numpy as np
import pytest

import lqcd_synth as syn
from oracle import closed_forms as cf
from oracle import dirac, geometry
from oracle.gamma import gamma5, gammas


def test_gamma_algebra():
    g = gammas()
    for mu in range(4):
        assert np.allclose(g[mu], g[mu].conj().T)
        for nu in range(4):
            assert np.allclose(g[mu] @ g[nu] + g[nu] @ g[mu], 2 * (mu == nu) * np.eye(4), atol=1e-15)
    g5 = gamma5()
    assert np.allclose(g5, np.diag([1, 1, -1, -1]), atol=1e-15)
    for mu in range(4):
        assert np.allclose(g5 @ g[mu] + g[mu] @ g5, 0, atol=1e-15)
        for s in (+1, -1):
            P = (np.eye(4) + s * g[mu]) / 2           # Hermitian rank-2 projector
            assert np.allclose(P @ P, P, atol=1e-15)
            assert np.linalg.matrix_rank(P) == 2


@pytest.mark.parametrize("kind", ["haar", "near_identity"])
def test_links_special_unitary(kind):
    U = syn.gauge_field((4, 4, 2, 2), kind, config=1)
    m = U.reshape(-1, 3, 3)
    eye = np.eye(3)
    assert np.max(np.abs(np.conj(np.swapaxes(m, 1, 2)) @ m - eye)) < 1e-13
    assert np.max(np.abs(np.linalg.det(m) - 1)) < 1e-13


def test_near_identity_mean_trace():
    # <Re tr U>/3 ~ 1 - eps^2 <tr H^2>/6 with tr H^2 = (1/2) sum h_a^2 ~ 4: 1 - eps^2 * 2/3
    U = syn.gauge_field((8, 8, 8, 8), "near_identity", config=2, eps=0.3)
    m = np.trace(U.reshape(-1, 3, 3), axis1=1, axis2=2).real.mean() / 3
    assert abs(m - (1 - 0.09 * 2 / 3)) < 2e-3


def _site_loop_apply(U, psi, m0):
    """Per-site evaluation with explicit loops and the neighbour table (used
    only on 2^4 / 4x2x2x2 where it runs in seconds)."""
    dims = U.shape[1:5]
    v = int(np.prod(dims))
    nbr = geometry.neighbour_table(dims)
    g = gammas()
    Uf = U.reshape(4, v, 3, 3)
    pf = psi.reshape(psi.shape[0], v, 4, 3)
    out = np.zeros_like(pf)
    for n in range(pf.shape[0]):
        for x in range(v):
            acc = (4 + m0) * pf[n, x]
            for mu in range(4):
                xp, xm = nbr[x, mu], nbr[x, 4 + mu]
                fwd = (np.eye(4) - g[mu]) @ (pf[n, xp] @ Uf[mu, x].T)
                bwd = (np.eye(4) + g[mu]) @ (pf[n, xm] @ np.conj(Uf[mu, xm]))
                acc = acc - 0.5 * (fwd + bwd)
            out[n, x] = acc
    return out.reshape(psi.shape)


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 2, 2)])
def test_site_loop_matches(dims):
    U = syn.gauge_field(dims, "haar", config=3)
    psi = syn.spinor_block(dims, 2, config=3)
    a = dirac.apply_dw(U, psi, 0.1)
    b = _site_loop_apply(U, psi, 0.1)
    assert np.max(np.abs(a - b)) < 1e-12


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 2, 2)])
def test_gamma5_hermiticity_dense(dims):
    U = syn.gauge_field(dims, "haar", config=4)
    D = dirac.dense(U, 0.1)
    v = int(np.prod(dims))
    G5 = np.kron(np.eye(v), np.kron(gamma5(), np.eye(3)))
    assert np.linalg.norm(G5 @ D @ G5 - D.conj().T) <= 1e-14 * np.linalg.norm(D)
    Dd = dirac.dense(U, 0.1)  # dagger apply vs conjugate transpose
    eye = np.eye(12 * v, dtype=np.complex128).reshape((12 * v,) + dims + (4, 3))
    cols = dirac.apply_dw_dagger(U, eye, 0.1).reshape(12 * v, 12 * v).T
    assert np.allclose(cols, Dd.conj().T, atol=1e-14)


def test_gamma5_hermiticity_inner_product():
    dims = (4, 4, 4, 8)
    U = syn.gauge_field(dims, "near_identity", config=5)
    phi = syn.spinor_block(dims, 1, config=5, role=syn.ROLE_CHI)
    psi = syn.spinor_block(dims, 1, config=5)
    m0 = -0.05
    lhs = np.vdot(phi, dirac.apply_gamma5(dirac.apply_dw(U, dirac.apply_gamma5(psi), m0)))
    rhs = np.vdot(dirac.apply_dw(U, phi, m0), psi)
    assert abs(lhs - rhs) <= 1e-12 * abs(rhs)


def test_gauge_covariance():
    dims = (4, 4, 4, 4)
    U = syn.gauge_field(dims, "haar", config=6)
    G = syn.gauge_transform(dims, config=6)
    psi = syn.spinor_block(dims, 2, config=6)
    UG = np.empty_like(U)
    for mu in range(4):
        UG[mu] = G @ U[mu] @ np.conj(np.swapaxes(np.roll(G, -1, axis=mu), -1, -2))
    lhs = dirac.apply_dw(UG, cf.colour_rotate(G, psi), 0.1)
    rhs = cf.colour_rotate(G, dirac.apply_dw(U, psi, 0.1))
    assert np.max(np.abs(lhs - rhs)) < 1e-12


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (8, 4, 6, 4)])
def test_free_plane_wave(dims):
    U = syn.gauge_field(dims, "unit", config=0)
    m0 = -0.05
    for n, u in syn.plane_wave_modes(dims, config=7, count=4):
        p = cf.momenta(n, dims)
        psi = cf.plane_wave(dims, p, u)[None]
        want = cf.plane_wave(dims, p, cf.free_symbol(p, m0) @ u)[None]
        assert np.max(np.abs(dirac.apply_dw(U, psi, m0) - want)) < 1e-13
        ev = np.linalg.eigvals(cf.free_symbol(p, m0))
        ref = cf.free_eigenvalues(p, m0)
        assert all(np.min(np.abs(ref - e)) < 1e-12 for e in ev)


def test_pure_gauge_plane_wave():
    dims = (4, 4, 6, 4)
    G = syn.gauge_transform(dims, config=8)
    U = cf.pure_gauge_links(G)
    m0 = 0.1
    for n, u in syn.plane_wave_modes(dims, config=8, count=3):
        p = cf.momenta(n, dims)
        psi = cf.colour_rotate(G, cf.plane_wave(dims, p, u))[None]
        want = cf.colour_rotate(G, cf.plane_wave(dims, p, cf.free_symbol(p, m0) @ u))[None]
        assert np.max(np.abs(dirac.apply_dw(U, psi, m0) - want)) < 1e-13


def test_free_spectrum_2x2x2x2():
    U = syn.gauge_field((2, 2, 2, 2), "unit", config=0)
    m0 = 0.1
    ev = np.sort(np.linalg.eigvals(dirac.dense(U, m0)).real)
    want = np.sort(np.concatenate([np.full(12 * comb(4, k), m0 + 2 * k) for k in range(5)]))
    assert np.allclose(ev, want, atol=1e-12)


def test_linearity_and_blocks_independent():
    dims = (4, 2, 2, 4)
    U = syn.gauge_field(dims, "haar", config=9)
    psi = syn.spinor_block(dims, 3, config=9)
    block = dirac.apply_dw(U, psi, 0.3)
    for i in range(3):
        assert np.allclose(dirac.apply_dw(U, psi[i:i + 1], 0.3)[0], block[i], atol=1e-14)


def test_site_sampled_apply_matches_block():
    dims = (4, 4, 2, 6)
    U = syn.gauge_field(dims, "near_identity", config=10)
    psi = syn.spinor_block(dims, 3, config=10)
    full = dirac.apply_dw(U, psi, -0.05).reshape(3, -1, 4, 3)
    sites = [0, 5, 17, 95, 191]
    assert np.max(np.abs(dirac.apply_dw_sites(U, psi, -0.05, sites) - full[:, sites])) < 1e-13
