"""Pins for the oracle's batched GMRES (Algorithm 2): dense LU, scipy's
restarted GMRES, the Arnoldi relation, Givens rotations, breakdown and the
zero right-hand side, and iterative refinement reaching the FP64 residual."""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import lqcd_synth as syn
from oracle import closed_forms as cf
from oracle import dirac, gmres, solve


def test_givens_zeroes_second_entry():
    rng = np.random.default_rng(1)
    for _ in range(20):
        a, b = rng.standard_normal(2) + 1j * rng.standard_normal(2)
        c, s = gmres.givens(a, b)
        G = np.array([[c, s], [-np.conj(s), c]])
        out = G @ np.array([a, b])
        assert abs(out[1]) < 1e-15 * abs(a)
        assert np.allclose(G.conj().T @ G, np.eye(2), atol=1e-15)
        assert abs(abs(out[0]) - np.hypot(abs(a), abs(b))) < 1e-14
    c, s = gmres.givens(0.0, 2.0 + 1j)
    G = np.array([[c, s], [-np.conj(s), c]])
    assert abs((G @ np.array([0, 2 + 1j]))[1]) == 0


def test_arnoldi_relation():
    dims = (4, 4, 2, 2)
    U = syn.gauge_field(dims, "haar", config=21)
    v0 = syn.spinor_block(dims, 1, config=21)[0]
    op = lambda v: dirac.apply_dw(U, v, 0.1)
    m = 12
    V, H = gmres.arnoldi(op, v0, m)
    AV = op(V[:m])
    Vm1 = V.reshape(m + 1, -1)
    lhs = AV.reshape(m, -1).T
    rhs = Vm1.T @ H
    assert np.linalg.norm(lhs - rhs) <= 1e-13 * np.linalg.norm(lhs)
    gram = Vm1.conj() @ Vm1.T
    # modified Gram-Schmidt keeps orthogonality to O(kappa * eps)
    assert np.max(np.abs(gram - np.eye(m + 1))) < 1e-10
    assert np.allclose(np.tril(H, -2), 0)


def test_gmres_matches_dense_lu():
    dims = (4, 4, 4, 4)
    m0 = 0.1
    U = syn.gauge_field(dims, "haar", config=22)
    b = syn.spinor_block(dims, 3, config=22)
    D = dirac.dense(U, m0)
    x_lu = np.linalg.solve(D, b.reshape(3, -1).T).T.reshape(b.shape)
    x, st = solve.solve(U, b, m0, tol=1e-10, restart=30)
    assert np.all(st.converged)
    assert np.all(st.true_relres <= 1e-10)
    kappa = np.linalg.cond(D)
    for i in range(3):
        err = np.linalg.norm(x[i] - x_lu[i]) / np.linalg.norm(x_lu[i])
        assert err <= kappa * 1e-10
    # the estimate |gamma_{j+1}| / ||b|| is below tol at exit
    assert np.all(st.est_relres < 1e-10)


def test_gmres_vs_scipy():
    dims = (4, 4, 4, 4)
    m0 = 0.1
    U = syn.gauge_field(dims, "haar", config=23)
    b = syn.spinor_block(dims, 1, config=23)
    n = b[0].size
    A = spla.LinearOperator((n, n), matvec=lambda v: dirac.apply_dw(U, v.reshape((1,) + b.shape[1:]), m0).reshape(-1),
                            dtype=np.complex128)
    xs, info = spla.gmres(A, b.reshape(-1), rtol=1e-10, atol=0, restart=30, maxiter=200)
    assert info == 0
    x, st = gmres.gmres(lambda v: dirac.apply_dw(U, v, m0), b, 1e-10, restart=30)
    assert np.linalg.norm(x.reshape(-1) - xs) <= 1e-8 * np.linalg.norm(xs)


def test_batched_equals_single():
    """Each rhs of a batch runs its own GMRES: solving rhs one at a time gives
    the same iterates (up to rounding)."""
    dims = (4, 2, 2, 4)
    U = syn.gauge_field(dims, "haar", config=24)
    b = syn.spinor_block(dims, 3, config=24)
    op = lambda v: dirac.apply_dw(U, v, 0.1)
    xb, sb = gmres.gmres(op, b, 1e-10, restart=10)
    for i in range(3):
        xi, si = gmres.gmres(op, b[i:i + 1], 1e-10, restart=10)
        assert np.allclose(xi[0], xb[i], atol=1e-12)
        assert si.iters[0] == sb.iters[i]


def test_zero_rhs_and_breakdown():
    dims = (4, 4, 4, 4)
    U = syn.gauge_field(dims, "unit", config=0)
    m0 = 0.1
    # a plane wave times an eigenvector of M(p) spans a 1-dimensional Krylov space
    n, _ = syn.plane_wave_modes(dims, config=25, count=1)[0]
    p = cf.momenta(n, dims)
    w, vecs = np.linalg.eig(cf.free_symbol(p, m0))
    u = np.outer(vecs[:, 0], [1.0, 0.5j, -0.25])
    b = np.stack([cf.plane_wave(dims, p, u), np.zeros(dims + (4, 3), dtype=np.complex128)])
    x, st = gmres.gmres(lambda v: dirac.apply_dw(U, v, m0), b, 1e-12, restart=30)
    assert st.iters[0] == 1            # happy breakdown after one step
    assert np.allclose(x[0], b[0] / w[0], atol=1e-13)
    assert np.all(x[1] == 0) and st.converged[1] and st.iters[1] == 0


def test_not_converged_reported():
    dims = (4, 4, 4, 4)
    U = syn.gauge_field(dims, "haar", config=26)
    b = syn.spinor_block(dims, 2, config=26)
    x, st = gmres.gmres(lambda v: dirac.apply_dw(U, v, -0.05), b, 1e-10, restart=5, max_restarts=1)
    assert not np.any(st.converged)
    assert np.all(st.true_relres > 1e-10) and np.all(st.iters == 5)


def test_eo_solve_full_residual():
    dims = (4, 4, 4, 4)
    m0 = 0.1
    U = syn.gauge_field(dims, "near_identity", config=27)
    b = syn.spinor_block(dims, 2, config=27)
    x, st = solve.solve(U, b, m0, tol=1e-10, eo=True)
    assert np.all(st.true_relres <= 1e-10)
    xf, sf = solve.solve(U, b, m0, tol=1e-10, eo=False)
    assert np.linalg.norm(x - xf) <= 1e-8 * np.linalg.norm(xf)


@pytest.mark.parametrize("mode", ["f32", "f16"])
def test_iterative_refinement_reaches_fp64(mode):
    dims = (4, 4, 4, 4)
    m0 = 0.1
    U = syn.gauge_field(dims, "near_identity", config=28)
    b = syn.spinor_block(dims, 2, config=28)
    x, st = solve.solve(U, b, m0, tol=1e-10, eo=True, mode=mode)
    assert np.all(st.true_relres <= 1e-10)
    D = dirac.dense(U, m0)
    x_lu = np.linalg.solve(D, b.reshape(2, -1).T).T.reshape(b.shape)
    kappa = np.linalg.cond(D)
    for i in range(2):
        assert np.linalg.norm(x[i] - x_lu[i]) / np.linalg.norm(x_lu[i]) <= kappa * 1e-10


def test_f16_rounding_per_rhs_scale():
    a = np.array([[1e-4 + 2e-5j, -3e-4 + 0j], [100 + 1j, -5 - 7j]])
    r = solve.round_f16(a)
    rel = np.abs(r - a) / np.abs(a).max(axis=1, keepdims=True)
    assert np.all(rel < 2 ** -11)
