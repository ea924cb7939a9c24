"""Pins of the oracle's block GMRES (one block Krylov subspace shared by all
rhs, Sec. II) against facts that do not go through its own iteration: the
explicit power-basis definition of the minimiser, single-rhs GMRES for b = 1,
the subspace inclusion K_k(A, y_q) in K_k(A, Y), dense LU solutions, the
block Arnoldi relation, exact termination on a small dense matrix, and
converged or zero columns."""
import numpy as np
import pytest

import lqcd_synth as syn
from oracle import block_gmres as bg
from oracle import dirac, evenodd, gmres


def _schur_problem(dims, nrhs, config, m0=0.1):
    U = syn.gauge_field(dims, "haar", config=config)
    b = syn.spinor_block(dims, nrhs, config=config)
    rhs = evenodd.prepare_source(U, b, m0)
    return U, rhs, (lambda v: evenodd.apply_schur(U, v, m0))


@pytest.mark.parametrize("k", [1, 2, 3])
def test_one_cycle_is_the_power_basis_minimiser(k):
    """k steps of block GMRES = argmin over K_k(A, R0) built from
    [R0, A R0, ..., A^{k-1} R0] (thin QR + least squares per column)."""
    U, B, op = _schur_problem((2, 2, 2, 4), 3, config=31)
    X0 = 0.1 * syn.spinor_block((2, 2, 2, 4), 3, config=32)
    X0 = X0.reshape(3, -1)[:, : B.reshape(3, -1).shape[1]].reshape(B.shape)
    x, st = bg.block_gmres(op, B, np.zeros(3), restart=k, max_restarts=1, x0=X0)
    want = bg.block_krylov_min(op, B, X0, k)
    assert st.steps == k and st.breakdowns == 0
    assert np.abs(x - want).max() <= 1e-10 * np.abs(want).max()


def test_one_rhs_reduces_to_gmres():
    """b = 1: the block iteration is plain GMRES (Algorithm 2 for one rhs)."""
    U, B, op = _schur_problem((4, 2, 2, 2), 1, config=33)
    for k in (1, 4, 9):
        x, _ = bg.block_gmres(op, B, np.zeros(1), restart=k, max_restarts=1)
        y, _ = gmres.gmres(op, B, 1e-300, restart=k, max_restarts=1)
        assert np.abs(x - y).max() <= 1e-12 * np.abs(y).max()


def test_subspace_inclusion_bounds_each_rhs():
    """K_k(A, y_q) is a subspace of K_k(A, Y): after one cycle of k block
    steps every column's residual is at most that of k steps of GMRES on that
    column alone."""
    dims = (4, 2, 2, 4)
    U, B, op = _schur_problem(dims, 4, config=34)
    k = 5
    x, _ = bg.block_gmres(op, B, np.zeros(4), restart=k, max_restarts=1)
    rb = np.linalg.norm((B - op(x)).reshape(4, -1), axis=1)
    rs = np.zeros(4)
    for q in range(4):
        y, _ = gmres.gmres(op, B[q:q + 1], 1e-300, restart=k, max_restarts=1)
        rs[q] = np.linalg.norm((B[q:q + 1] - op(y)).reshape(-1))
    assert np.all(rb <= rs * (1 + 1e-10))
    # the shared space is larger than each column's own: strictly smaller residuals here
    assert np.all(rb < 0.99 * rs)


@pytest.mark.parametrize("eo", [False, True])
def test_solution_matches_dense_lu(eo):
    dims = (2, 2, 2, 4)
    m0 = 0.1
    U = syn.gauge_field(dims, "haar", config=35)
    b = syn.spinor_block(dims, 3, config=36)
    x, st = bg.block_solve(U, b, m0, tol=1e-11, restart=6, max_restarts=50, eo=eo)
    D = dirac.dense(U, m0)
    want = np.linalg.solve(D, b.reshape(3, -1).T).T.reshape(b.shape)
    assert np.all(st.converged)
    assert np.all(np.linalg.norm((x - want).reshape(3, -1), axis=1)
                  <= 1e-8 * np.linalg.norm(want.reshape(3, -1), axis=1))
    rel = st.true_res / np.linalg.norm(b.reshape(3, -1), axis=1)
    assert np.all(rel <= 1e-11)


def test_block_arnoldi_relation():
    dims = (4, 2, 2, 2)
    U, B, op = _schur_problem(dims, 3, config=37)
    R0 = B.reshape(3, -1).T
    m = 4
    V, Hbar, S = bg.block_arnoldi(op, R0, m, B.shape[1:])
    n = V.shape[0]
    assert np.linalg.norm(V.conj().T @ V - np.eye(V.shape[1])) <= 1e-11  # one MGS pass: O(kappa eps)
    AV = op(np.ascontiguousarray(V[:, : m * 3].T).reshape((m * 3,) + B.shape[1:])).reshape(m * 3, n).T
    assert np.linalg.norm(AV - V @ Hbar) <= 1e-13 * np.linalg.norm(AV)
    assert np.linalg.norm(V[:, :3] @ S - R0) <= 1e-13 * np.linalg.norm(R0)
    # H_{j+1,j} blocks are upper triangular
    for j in range(m):
        blk = Hbar[(j + 1) * 3:(j + 2) * 3, j * 3:(j + 1) * 3]
        assert np.abs(np.tril(blk, -1)).max() == 0.0


def test_exact_after_n_over_b_steps():
    """n = 12, b = 3: K_4(A, R0) is the whole space, so four block steps solve
    exactly (the fourth step finds the rank-deficient remainder)."""
    rng = np.random.default_rng(5)
    n, b = 12, 3
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 4 * np.eye(n)
    op = lambda v: (A @ v.reshape(v.shape[0], n).T).T.reshape(v.shape)
    B = rng.standard_normal((b, n)) + 1j * rng.standard_normal((b, n))
    x, st = bg.block_gmres(op, B, np.full(b, 1e-9), restart=4, max_restarts=1)
    want = np.linalg.solve(A, B.T).T
    assert st.steps == 4
    assert np.abs(x - want).max() <= 1e-9 * np.abs(want).max()


def test_zero_and_converged_columns():
    dims = (2, 2, 2, 4)
    U, B, op = _schur_problem(dims, 3, config=38)
    B = B.copy()
    B[1] = 0
    thr = 1e-10 * np.linalg.norm(B.reshape(3, -1), axis=1)
    x, st = bg.block_gmres(op, B, thr, restart=8, max_restarts=40)
    assert np.all(st.converged)
    assert np.abs(x[1]).max() == 0.0
    # restarting from the solution: nothing left to do
    x2, st2 = bg.block_gmres(op, B, thr, restart=8, max_restarts=40, x0=x)
    assert st2.steps == 0 and np.array_equal(x2, x)


def test_rank_deficient_right_hand_sides():
    """Two equal right-hand sides make the residual block rank deficient: the
    dependent column sits out the first cycle and both converge to the same
    solution (dense LU)."""
    dims = (2, 2, 2, 4)
    m0 = 0.1
    U = syn.gauge_field(dims, "haar", config=39)
    b = syn.spinor_block(dims, 3, config=39)
    b[2] = b[0]
    x, st = bg.block_solve(U, b, m0, tol=1e-11, restart=6, max_restarts=60, eo=False)
    assert np.all(st.converged)
    D = dirac.dense(U, m0)
    want = np.linalg.solve(D, b.reshape(3, -1).T).T.reshape(b.shape)
    assert np.all(np.linalg.norm((x - want).reshape(3, -1), axis=1) <= 1e-8 * np.linalg.norm(want.reshape(3, -1), axis=1))
