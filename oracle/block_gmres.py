"""Block GMRES: all right-hand sides expand one common block Krylov subspace.

TEST INFRASTRUCTURE ONLY: imported by tests/, the smoke check and the
benchmark's CPU baseline, never by the library path.

Sec. II (multiple right-hand sides) defines the block Krylov subspace of the
rhs matrix Y = [y_1 | ... | y_b],

    K_k(A, Y) = span{Y, A Y, ..., A^{k-1} Y},

which contains every individual Krylov subspace K_k(A, y_i); block solvers
minimise over it, and the paper contrasts them with the batched solver it
uses (Sec. III-A.2).  It does not spell out the block iteration.  The oracle
takes it from its definition:

* `block_krylov_min` is the definition itself for one cycle of k steps:
  X = X0 + Q Z with Q an orthonormal basis of K_k(A, R0), R0 = B - A X0, and
  each column of Z minimising its own residual ||r0_q - A Q z_q||.  It builds
  Q from the explicit power basis (thin QR), so it is for small k only.
* `block_gmres` is the restarted iteration (block GMRES(m)) that reaches the
  same minimiser step by step: thin QR R0 = V_0 S; per step W = A V_j, block
  modified Gram-Schmidt H_ij = V_i^H W, W -= V_i H_ij (i = 0..j), thin QR
  W = V_{j+1} H_{j+1,j}; Y_j = argmin ||E_1 S - Hbar_j Y|| column by column
  (library least squares); the column norms of E_1 S - Hbar_j Y_j are the
  per-rhs residual estimates.  At the end of a cycle X += [V_0 .. V_j] Y_j.

Readings taken where the definition leaves choices:
* inner product <a, b> = sum conj(a) b, as everywhere in the oracle;
* a cycle ends after m steps, when every active column's estimate is at or
  below its threshold ("max over rhs" exit, as Algorithm 2), or at a
  breakdown: the new block is numerically rank deficient, i.e. its columns
  are linearly dependent and K_k(A, R0) stops growing in that direction (a
  diagonal entry of the Householder triangular factor at or below
  BREAKDOWN = 1e-12 of the block's largest column norm; Householder QR in
  complex128 resolves dependence to about 1e-16 of that norm, and 1e-12
  keeps four orders of magnitude above that floor); the step that found it
  still enters the least-squares problem (its Hessenberg columns are
  complete), later steps are not taken;
* each cycle restarts from the true residual B - A X with only the columns
  that have not converged (converged columns keep their x); if that residual
  block is itself numerically rank deficient (a diagonal entry of its
  triangular factor at or below the breakdown threshold, e.g. two equal
  right-hand sides), the columns at those diagonal entries sit out the cycle
  (their x is not updated, they are active again at the next restart), one
  factorisation at a time until the remaining block has full rank;
* the thresholds are absolute residual norms per column (the caller turns a
  relative tolerance into them), so the full-system reading of the odd-even
  solve carries over unchanged.
Vectors are complex128; a block is held as an n x b matrix (one column per
rhs) inside, and as the rhs-first arrays of the other oracle modules at the
interface.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import dirac, evenodd
from .gmres import _norms

BREAKDOWN = 1e-12


@dataclass
class BlockStats:
    steps: int                 # block Arnoldi steps taken (all cycles)
    cycles: int                # cycles started
    converged: np.ndarray      # bool per rhs
    true_res: np.ndarray       # ||b_q - A x_q|| at exit, per rhs
    est_res: np.ndarray        # last least-squares residual estimate per rhs
    breakdowns: int            # cycles ended by a rank-deficient block
    iters: np.ndarray = None   # block steps during which each rhs was active


def _to_mat(blk: np.ndarray) -> np.ndarray:
    return blk.reshape(blk.shape[0], -1).T.astype(np.complex128)


def _to_blk(mat: np.ndarray, shape) -> np.ndarray:
    return np.ascontiguousarray(mat.T).reshape((mat.shape[1],) + tuple(shape))


def _apply_mat(apply, M: np.ndarray, shape) -> np.ndarray:
    return _to_mat(apply(_to_blk(M, shape)))


def _thin_qr(W: np.ndarray):
    """W = Q R with Q orthonormal columns; returns (Q, R, rank_deficient)."""
    Q, R = np.linalg.qr(W, mode="reduced")
    scale = float(np.max(np.linalg.norm(W, axis=0))) if W.size else 0.0
    deficient = scale == 0.0 or bool(np.any(np.abs(np.diag(R)) <= BREAKDOWN * scale))
    return Q, R, deficient


def block_krylov_min(apply, B: np.ndarray, X0: np.ndarray, k: int) -> np.ndarray:
    """The definition: X0 + argmin over K_k(A, R0), column by column, with an
    orthonormal basis of the explicit power basis [R0, A R0, ..., A^{k-1} R0]."""
    shape = B.shape[1:]
    R0 = _to_mat(B) - _apply_mat(apply, _to_mat(X0), shape)
    blocks = [R0]
    for _ in range(1, k):
        blocks.append(_apply_mat(apply, blocks[-1], shape))
    Q, _ = np.linalg.qr(np.concatenate(blocks, axis=1), mode="reduced")
    AQ = _apply_mat(apply, Q, shape)
    Z = np.linalg.lstsq(AQ, R0, rcond=None)[0]
    return _to_blk(_to_mat(X0) + Q @ Z, shape)


def block_arnoldi(apply, R0: np.ndarray, m: int, shape):
    """m steps of block Arnoldi (block MGS, thin QR) from the n x b matrix R0.
    Returns (V, Hbar, S): V n x (m+1) b, Hbar (m+1) b x m b, R0 = V_0 S."""
    b = R0.shape[1]
    V0, S, _ = _thin_qr(R0)
    V = [V0]
    Hbar = np.zeros(((m + 1) * b, m * b), dtype=np.complex128)
    for j in range(m):
        W = _apply_mat(apply, V[j], shape)
        for i in range(j + 1):
            Hij = V[i].conj().T @ W
            Hbar[i * b:(i + 1) * b, j * b:(j + 1) * b] = Hij
            W = W - V[i] @ Hij
        Q, R, _ = _thin_qr(W)
        Hbar[(j + 1) * b:(j + 2) * b, j * b:(j + 1) * b] = R
        V.append(Q)
    return np.concatenate(V, axis=1), Hbar, S


def block_gmres(apply, B: np.ndarray, thresholds: np.ndarray, restart: int = 30, max_restarts: int = 200,
                x0: np.ndarray | None = None, max_steps: int | None = None):
    """Restarted block GMRES(m).  `apply` maps a block (k, ...) to A times it;
    column q is converged when ||b_q - A x_q|| <= thresholds[q].  max_steps
    caps the total number of block steps (for fixed-work comparisons).
    Returns (x, BlockStats)."""
    shape = B.shape[1:]
    nrhs = B.shape[0]
    m = int(restart)
    Bm = _to_mat(B)
    X = np.zeros_like(Bm) if x0 is None else _to_mat(x0)
    thr = np.asarray(thresholds, dtype=np.float64).reshape(nrhs)
    est = np.full(nrhs, np.inf)
    iters = np.zeros(nrhs, dtype=np.int64)
    steps_total, cycles, breakdowns = 0, 0, 0
    for _cycle in range(max_restarts):
        if max_steps is not None and steps_total >= max_steps:
            break
        Rm = Bm - _apply_mat(apply, X, shape)
        rn = np.linalg.norm(Rm, axis=0)
        act = np.nonzero(rn > thr)[0]
        est[rn <= thr] = rn[rn <= thr]
        if act.size == 0:
            break
        cycles += 1
        while True:
            V0, S, deficient = _thin_qr(Rm[:, act])
            if not deficient:
                break
            scale = float(np.max(np.linalg.norm(Rm[:, act], axis=0)))
            drop = np.abs(np.diag(S)) <= BREAKDOWN * scale
            act = act[~drop]
        b = act.size
        V = [V0]
        Hbar = np.zeros(((m + 1) * b, m * b), dtype=np.complex128)
        G = np.zeros(((m + 1) * b, b), dtype=np.complex128)
        G[:b] = S
        Y, done_steps = None, 0
        for j in range(m):
            if max_steps is not None and steps_total >= max_steps:
                break
            W = _apply_mat(apply, V[j], shape)
            for i in range(j + 1):
                Hij = V[i].conj().T @ W
                Hbar[i * b:(i + 1) * b, j * b:(j + 1) * b] = Hij
                W = W - V[i] @ Hij
            Q, Rj, deficient = _thin_qr(W)
            Hbar[(j + 1) * b:(j + 2) * b, j * b:(j + 1) * b] = Rj
            V.append(Q)
            steps_total += 1
            done_steps = j + 1
            Hj = Hbar[:(j + 2) * b, :(j + 1) * b]
            Gj = G[:(j + 2) * b]
            Y = np.linalg.lstsq(Hj, Gj, rcond=None)[0]
            e = np.linalg.norm(Gj - Hj @ Y, axis=0)
            est[act] = e
            if deficient:
                # the step's columns of Hbar are complete (A V_j lies in the
                # current space up to the tiny remainder), so the step counts;
                # the space cannot grow further in this cycle
                breakdowns += 1
                break
            if np.all(e <= thr[act]):
                break
        if done_steps == 0:
            break
        Vm = np.concatenate(V[:done_steps], axis=1)
        X[:, act] = X[:, act] + Vm @ Y
        iters[act] += done_steps
    true = np.linalg.norm(Bm - _apply_mat(apply, X, shape), axis=0)
    return _to_blk(X, shape), BlockStats(steps_total, cycles, true <= thr, true, est, breakdowns, iters)


def block_solve(U, b, m0, tol=1e-10, restart=30, max_restarts=200, eo=False, max_steps=None):
    """x = D_W^{-1} b for the rhs block b with block GMRES, on the full system
    or on the odd-even Schur complement (prepare, solve S x_e = b'_e,
    reconstruct).  Column q stops at a residual of tol ||b_q|| of the reduced
    system, which after reconstruction is the full system's residual."""
    b = np.asarray(b, dtype=np.complex128)
    thr = tol * _norms(b)
    if eo:
        rhs = evenodd.prepare_source(U, b, m0)
        y, st = block_gmres(lambda v: evenodd.apply_schur(U, v, m0), rhs, thr, restart, max_restarts,
                            max_steps=max_steps)
        x = evenodd.reconstruct(U, b, y, m0)
    else:
        x, st = block_gmres(lambda v: dirac.apply_dw(U, v, m0), b, thr, restart, max_restarts, max_steps=max_steps)
    true = _norms(b - dirac.apply_dw(U, x, m0))
    st.true_res = true
    st.converged = true <= thr
    return x, st
