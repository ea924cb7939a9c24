"""Differentiation on the GPU: link force, batched dot, adjoint solve and the
autograd Functions, against the oracle's gradients and finite differences of
the oracle's dense-LU loss."""
import numpy as np
import pytest

import lqcd_synth as syn
import paper_2601_05816_amd as lq
from oracle import dirac, gradients

from helpers import rel_err_per_rhs

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch

    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _l2(block):
    return np.ascontiguousarray(np.moveaxis(block, 0, -1))


def _from_l2(t):
    return np.moveaxis(t.detach().cpu().numpy(), -1, 0)


@pytest.mark.parametrize("layout", [lq.RHS_OUTER, lq.LAYOUT1, lq.LAYOUT2])
@pytest.mark.parametrize("project", [False, True])
def test_link_force_matches_oracle(gpu_lib, layout, project):
    from helpers import to_layout_np

    dims = (4, 4, 2, 6)
    U = syn.gauge_field(dims, "near_identity", config=41)
    g = syn.spinor_block(dims, 3, config=41, role=syn.ROLE_CHI)
    psi = syn.spinor_block(dims, 3, config=41)
    want = gradients.apply_link_grad(U, g, psi)
    if project:
        want = gradients.su3_force(U, want)
    got = lq.link_force(_dev(U), _dev(to_layout_np(g, layout)), _dev(to_layout_np(psi, layout)), -0.5,
                        layout=layout, project=project).cpu().numpy()
    assert np.linalg.norm(got - want) <= 1e-13 * np.linalg.norm(want)


def test_block_dot(gpu_lib):
    dims = (4, 2, 2, 4)
    a = syn.spinor_block(dims, 5, config=42)
    b = syn.spinor_block(dims, 5, config=42, role=syn.ROLE_CHI)
    got = lq.block_dot(_dev(_l2(a)), _dev(_l2(b)), dims).cpu().numpy()
    want = np.array([np.vdot(a[i], b[i]) for i in range(5)])
    assert np.allclose(got, want, rtol=1e-13, atol=0)


def test_apply_gradients_vs_oracle_and_gradcheck(gpu_lib):
    import torch

    from paper_2601_05816_amd.autograd import wilson_apply

    dims = (4, 4, 2, 2)
    m0 = 0.1
    U = syn.gauge_field(dims, "haar", config=43)
    psi = syn.spinor_block(dims, 2, config=43)
    chi = syn.spinor_block(dims, 2, config=43, role=syn.ROLE_CHI)
    Ut = _dev(U).requires_grad_()
    pt = _dev(_l2(psi)).requires_grad_()
    mt = torch.tensor(m0, dtype=torch.float64, device="cuda", requires_grad=True)
    y = wilson_apply(Ut, pt, mt)
    loss = torch.real(torch.sum(torch.conj(_dev(_l2(chi))) * y))
    loss.backward()
    want = gradients.apply_link_grad(U, chi, psi)
    assert np.linalg.norm(Ut.grad.cpu().numpy() - want) <= 1e-12 * np.linalg.norm(want)
    assert np.all(rel_err_per_rhs(_from_l2(pt.grad), dirac.apply_dw_dagger(U, chi, m0)) < 1e-12)
    assert abs(float(mt.grad) - np.real(np.vdot(chi, psi))) < 1e-10 * abs(np.vdot(chi, psi))
    # torch's own finite-difference check on a tiny lattice
    small = (2, 2, 2, 4)
    Us = _dev(syn.gauge_field(small, "haar", config=44)).requires_grad_()
    ps = _dev(_l2(syn.spinor_block(small, 1, config=44))).requires_grad_()
    assert torch.autograd.gradcheck(lambda u, p: wilson_apply(u, p, 0.3), (Us, ps), eps=1e-6, atol=1e-7)


class _DenseLoss:
    """L = Re <chi, A^-1 eta> with A = D_W(U, m0) or its adjoint, from the
    oracle's dense matrix, for central differences.  One LU of A serves all
    evaluations: a perturbed link entry U_mu(x)[a][b] changes only the
    columns of D at x and at its neighbours along mu, so the perturbed A is
    A plus a low-rank term and is solved exactly with the Woodbury identity
    (checked on a random vector that no other column changed); a perturbed
    mass is A + dm I, factorised afresh."""

    def __init__(self, U, eta, chi, m0, dagger):
        import scipy.linalg as sla

        self.sla, self.U, self.m0, self.dagger = sla, U, m0, dagger
        self.dims = U.shape[1:5]
        n = eta.shape[0]
        D = dirac.dense(U, m0)
        self.A = D.conj().T.copy() if dagger else D
        self.lu = sla.lu_factor(self.A)
        self.B = eta.reshape(n, -1).T
        self.chi = chi.reshape(n, -1).T
        self.Y = sla.lu_solve(self.lu, self.B)

    def _loss(self, X):
        return float(np.real(np.vdot(self.chi, X)))

    def mass(self, dm):
        n = self.A.shape[0]
        return self._loss(self.sla.lu_solve(self.sla.lu_factor(self.A + dm * np.eye(n)), self.B))

    def link(self, k, delta):
        """L with U.flat[k] += delta."""
        sla, dims, n = self.sla, self.dims, self.A.shape[0]
        mu, t, z, y, x, _, _ = np.unravel_index(k, self.U.shape)
        sites = set()
        for step in (0, 1, -1):
            c = [t, z, y, x]
            c[mu] = (c[mu] + step) % dims[mu]
            sites.add(int(np.ravel_multi_index(tuple(c), dims)))
        cols = np.array(sorted(12 * st + j for st in sites for j in range(12)))
        m = len(cols)
        Up = self.U.copy()
        Up.reshape(-1)[k] += delta
        E = np.zeros((m, n), dtype=np.complex128)
        E[np.arange(m), cols] = 1.0
        E = E.reshape((m,) + tuple(dims) + (4, 3))
        dC = (dirac.apply_dw(Up, E, self.m0) - dirac.apply_dw(self.U, E, self.m0)).reshape(m, n).T
        v = np.random.default_rng(k).standard_normal(n) + 0j
        vb = v.reshape((1,) + tuple(dims) + (4, 3))
        dv = (dirac.apply_dw(Up, vb, self.m0) - dirac.apply_dw(self.U, vb, self.m0)).reshape(n)
        assert np.allclose(dv, dC @ v[cols], rtol=0, atol=1e-13 * max(1.0, np.abs(dv).max()))
        Y = self.Y
        if self.dagger:  # A' = A + E_C dC^H
            P = np.zeros((n, m), dtype=np.complex128)
            P[cols, np.arange(m)] = 1.0
            Z = sla.lu_solve(self.lu, P)
            QH = dC.conj().T
            X = Y - Z @ np.linalg.solve(np.eye(m) + QH @ Z, QH @ Y)
        else:  # A' = A + dC E_C^T
            Z = sla.lu_solve(self.lu, dC)
            X = Y - Z @ np.linalg.solve(np.eye(m) + Z[cols], Y[cols])
        return self._loss(X)


@pytest.mark.parametrize("dagger", [False, True])
def test_solve_gradients_fd_4x4x4x4(gpu_lib, dagger):
    """x = A^-1 eta with A = D or D^dagger: the gradients of L = Re <chi, x>
    against central differences of the dense-LU loss."""
    import torch

    from paper_2601_05816_amd.autograd import wilson_solve

    dims = (4, 4, 4, 4)
    m0 = 0.05
    U = syn.gauge_field(dims, "near_identity", config=45, eps=0.3)
    eta = syn.spinor_block(dims, 2, config=45)
    chi = syn.spinor_block(dims, 2, config=45, role=syn.ROLE_CHI)
    Ut = _dev(U).requires_grad_()
    et = _dev(_l2(eta)).requires_grad_()
    mt = torch.tensor(m0, dtype=torch.float64, device="cuda", requires_grad=True)
    x = wilson_solve(Ut, et, mt, tol=1e-13, eo=True, dagger=dagger)
    loss = torch.real(torch.sum(torch.conj(_dev(_l2(chi))) * x))
    loss.backward()
    gU = Ut.grad.cpu().numpy()
    h = 1e-6
    rng = np.random.default_rng(3)
    L = _DenseLoss(U, eta, chi, m0, dagger)
    for k in rng.choice(U.size, size=8, replace=False):
        for unit in (1.0, 1j):
            fd = (L.link(k, h * unit) - L.link(k, -h * unit)) / (2 * h)
            an = gU.reshape(-1)[k].real if unit == 1.0 else gU.reshape(-1)[k].imag
            assert abs(fd - an) < 1e-6 * max(1.0, abs(an)), (k, unit, fd, an)
    fd = (L.mass(h) - L.mass(-h)) / (2 * h)
    assert abs(fd - float(mt.grad)) < 1e-6 * max(1.0, abs(fd))
    # grad_eta = lambda = A^-dagger chi
    lam = np.linalg.solve(L.A.conj().T, chi.reshape(2, -1).T).T.reshape(chi.shape)
    assert np.all(rel_err_per_rhs(_from_l2(et.grad), lam) < 1e-10)


def test_solve_gradient_16x16x16x32(gpu_lib):
    """Differentiation workload: 16^3 x 32, eps = 0.3, m0 = 0.05, 8 rhs,
    L = sum_i Re <chi_i, x_i>.  Checked without an oracle solve: the oracle
    confirms D x = eta and D^dagger lambda = chi on the GPU's x and lambda, and
    recomputes the link gradient from them."""
    import torch

    dims = (32, 16, 16, 16)
    m0 = 0.05
    U = syn.gauge_field(dims, "near_identity", config=5, eps=0.3)
    eta = syn.spinor_block(dims, 8, config=5)
    chi = syn.spinor_block(dims, 8, config=5, role=syn.ROLE_CHI)
    Ud, ed, cd = _dev(U), _dev(_l2(eta)), _dev(_l2(chi))
    x, st, rc = lq.gmres_solve(Ud, ed, m0, eo=True, tol=1e-12)
    assert rc == lq.OK
    lam, st2, rc2 = lq.gmres_solve(Ud, cd, m0, eo=True, tol=1e-12, dagger=True)
    assert rc2 == lq.OK
    G = lq.link_force(Ud, lam, x, 0.5).cpu().numpy()
    xs, ls = _from_l2(x), _from_l2(lam)
    assert np.all(rel_err_per_rhs(dirac.apply_dw(U, xs, m0), eta) <= 1e-12)
    assert np.all(rel_err_per_rhs(dirac.apply_dw_dagger(U, ls, m0), chi) <= 1e-12)
    want = -gradients.apply_link_grad(U, ls, xs)
    assert np.linalg.norm(G - want) <= 1e-12 * np.linalg.norm(want)
