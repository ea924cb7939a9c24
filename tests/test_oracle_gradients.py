"""Pins for the oracle's gradients: central finite differences of the loss
through the apply and through a dense-LU solve, and su(3) group directions."""
import numpy as np
import pytest
import scipy.linalg as sla

import lqcd_synth as syn
from oracle import dirac, gradients


def _loss_apply(U, psi, chi, m0):
    return float(np.real(np.vdot(chi, dirac.apply_dw(U, psi, m0))))


def _dense_solve(U, eta, m0):
    D = dirac.dense(U, m0)
    n = eta.shape[0]
    return np.linalg.solve(D, eta.reshape(n, -1).T).T.reshape(eta.shape)


def _loss_solve(U, eta, chi, m0):
    return float(np.real(np.vdot(chi, _dense_solve(U, eta, m0))))


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 2, 2)])
def test_apply_gradients_fd(dims):
    m0 = 0.1
    U = syn.gauge_field(dims, "haar", config=31)
    psi = syn.spinor_block(dims, 2, config=31)
    chi = syn.spinor_block(dims, 2, config=31, role=syn.ROLE_CHI)
    G = gradients.apply_link_grad(U, chi, psi)
    rng = np.random.default_rng(5)
    # the loss is linear in U, psi and m0, so central differences carry no
    # truncation error and a large step keeps rounding small
    h = 1e-3
    flatU = U.reshape(-1)
    for k in rng.choice(flatU.size, size=40, replace=False):
        for unit in (1.0, 1j):
            Up = flatU.copy(); Up[k] += h * unit
            Um = flatU.copy(); Um[k] -= h * unit
            fd = (_loss_apply(Up.reshape(U.shape), psi, chi, m0) - _loss_apply(Um.reshape(U.shape), psi, chi, m0)) / (2 * h)
            an = G.reshape(-1)[k].real if unit == 1.0 else G.reshape(-1)[k].imag
            assert abs(fd - an) < 1e-9 * max(1.0, abs(an))
    # grad_psi = D^dagger chi, grad_m0 = Re <chi, psi>
    gpsi = dirac.apply_dw_dagger(U, chi, m0)
    flatp = psi.reshape(-1)
    for k in rng.choice(flatp.size, size=10, replace=False):
        pp = flatp.copy(); pp[k] += h * 1j
        pm = flatp.copy(); pm[k] -= h * 1j
        fd = (_loss_apply(U, pp.reshape(psi.shape), chi, m0) - _loss_apply(U, pm.reshape(psi.shape), chi, m0)) / (2 * h)
        assert abs(fd - gpsi.reshape(-1)[k].imag) < 1e-9
    fd = (_loss_apply(U, psi, chi, m0 + h) - _loss_apply(U, psi, chi, m0 - h)) / (2 * h)
    assert abs(fd - np.real(np.vdot(chi, psi))) < 1e-9 * abs(np.vdot(chi, psi))


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 2, 2, 2)])
def test_solve_gradients_fd(dims):
    m0 = 0.05
    U = syn.gauge_field(dims, "near_identity", config=32)
    eta = syn.spinor_block(dims, 2, config=32)
    chi = syn.spinor_block(dims, 2, config=32, role=syn.ROLE_CHI)
    x = _dense_solve(U, eta, m0)
    # lambda = D^{-dagger} chi, by a dense solve with the conjugate transpose
    D = dirac.dense(U, m0)
    lam = np.linalg.solve(D.conj().T, chi.reshape(2, -1).T).T.reshape(chi.shape)
    # and equal to gamma5 D^{-1} gamma5 chi
    lam5 = dirac.apply_gamma5(_dense_solve(U, dirac.apply_gamma5(chi), m0))
    assert np.allclose(lam, lam5, atol=1e-12)
    G = -gradients.apply_link_grad(U, lam, x)
    gm0 = -np.real(np.vdot(lam, x))
    h = 1e-6
    rng = np.random.default_rng(6)
    flatU = U.reshape(-1)
    for k in rng.choice(flatU.size, size=24, replace=False):
        for unit in (1.0, 1j):
            Up = flatU.copy(); Up[k] += h * unit
            Um = flatU.copy(); Um[k] -= h * unit
            fd = (_loss_solve(Up.reshape(U.shape), eta, chi, m0) - _loss_solve(Um.reshape(U.shape), eta, chi, m0)) / (2 * h)
            an = G.reshape(-1)[k].real if unit == 1.0 else G.reshape(-1)[k].imag
            assert abs(fd - an) < 1e-6 * max(1.0, abs(an))
    fd = (_loss_solve(U, eta, chi, m0 + h) - _loss_solve(U, eta, chi, m0 - h)) / (2 * h)
    assert abs(fd - gm0) < 1e-6 * max(1.0, abs(gm0))
    flate = eta.reshape(-1)
    for k in rng.choice(flate.size, size=6, replace=False):
        ep = flate.copy(); ep[k] += h
        em = flate.copy(); em[k] -= h
        fd = (_loss_solve(U, ep.reshape(eta.shape), chi, m0) - _loss_solve(U, em.reshape(eta.shape), chi, m0)) / (2 * h)
        assert abs(fd - lam.reshape(-1)[k].real) < 1e-6


def test_su3_force_group_directions():
    dims = (4, 2, 2, 2)
    m0 = 0.05
    U = syn.gauge_field(dims, "near_identity", config=33)
    eta = syn.spinor_block(dims, 1, config=33)
    chi = syn.spinor_block(dims, 1, config=33, role=syn.ROLE_CHI)
    x = _dense_solve(U, eta, m0)
    D = dirac.dense(U, m0)
    lam = np.linalg.solve(D.conj().T, chi.reshape(1, -1).T).T.reshape(chi.shape)
    F = gradients.su3_force(U, -gradients.apply_link_grad(U, lam, x))
    # F is traceless anti-Hermitian
    assert np.allclose(F + np.conj(np.swapaxes(F, -1, -2)), 0, atol=1e-14)
    assert np.allclose(np.trace(F, axis1=-2, axis2=-1), 0, atol=1e-14)
    lam_a = syn.gell_mann()
    h = 1e-5
    for (mu, t, z) in [(0, 1, 0), (2, 3, 1), (3, 0, 1)]:
        for a in (0, 3, 7):
            Q = 1j * lam_a[a] / 2
            Up = U.copy(); Um = U.copy()
            Up[mu, t, z, 0, 1] = sla.expm(h * Q) @ U[mu, t, z, 0, 1]
            Um[mu, t, z, 0, 1] = sla.expm(-h * Q) @ U[mu, t, z, 0, 1]
            fd = (_loss_solve(Up, eta, chi, m0) - _loss_solve(Um, eta, chi, m0)) / (2 * h)
            an = np.real(np.trace(np.conj(F[mu, t, z, 0, 1]).T @ Q))
            assert abs(fd - an) < 1e-7 * max(1.0, abs(an))
