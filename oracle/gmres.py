"""Batched restarted GMRES (Algorithm 2, Sec. III-A.2) and its iterative
refinement variant with a lower working precision.

Every right-hand side i runs its own restarted GMRES(m) in lock-step with the
others (batched, not block Krylov).  One restart cycle:

  r_i = b_i - A x_i, beta_i = ||r_i||, v_0 = r_i / beta_i, gamma = beta_i e_1
  for j = 0 .. m-1:
      w = A v_j                                   (one block apply for all i)
      modified Gram-Schmidt: h_kj = <v_k, w>, w -= h_kj v_k   (k = 0..j)
      h_{j+1,j} = ||w||, v_{j+1} = w / h_{j+1,j}
      apply the previous Givens rotations to column j, build the rotation
      that zeroes h_{j+1,j}, rotate gamma
      relnorm_i = |gamma_{j+1}| / ||b_i||
  x_i += V_i y_i with y_i the least-squares minimiser of ||gamma - H y||
  (back substitution on the rotated upper triangle).

Readings where the paper is silent (Algorithm 2 fixes the loop structure and
the stopping quantity only):
  * the orthogonalisation is modified Gram-Schmidt; <a, b> = sum conj(a) b;
  * x_0 = 0 unless a guess is given; a zero right-hand side returns x = 0;
  * a rhs whose relnorm falls below tol (or whose Krylov space closes,
    h_{j+1,j} = 0) stops taking Arnoldi steps for the rest of the cycle; the
    cycle ends when none is left, which is the "max over rhs" exit;
  * the next cycle starts from the true residual b - A x, so convergence is
    confirmed on the true residual, and the solve ends when every rhs has
    ||b_i - A x_i|| <= tol ||b_i|| or the restart cap is reached.
The Hessenberg matrix, the rotations and gamma are complex128 regardless of
the precision the vectors are held in.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np


@dataclass
class GmresStats:
    iters: np.ndarray          # Arnoldi steps taken per rhs (all cycles)
    restarts: np.ndarray       # cycles started per rhs
    converged: np.ndarray      # bool per rhs
    true_relres: np.ndarray    # ||b - A x|| / ||b|| at exit, per rhs
    est_relres: np.ndarray     # last |gamma_{j+1}| / ||b|| per rhs
    history: list = field(default_factory=list)


def _norms(a: np.ndarray) -> np.ndarray:
    flat = a.reshape(a.shape[0], -1)
    return np.sqrt(np.sum((flat.real.astype(np.float64) ** 2 + flat.imag.astype(np.float64) ** 2), axis=1))


def _dot(a: np.ndarray, b: np.ndarray) -> complex:
    return complex(np.vdot(a.reshape(-1), b.reshape(-1)))


def givens(a: complex, b: complex):
    """Complex rotation G = [[c, s], [-conj(s), c]] (c real) with G [a; b] = [rho; 0]."""
    if a == 0:
        return 0.0, 1.0 + 0j
    r = np.hypot(abs(a), abs(b))
    c = abs(a) / r
    s = (a / abs(a)) * np.conj(b) / r
    return c, s


def back_substitute(R: np.ndarray, g: np.ndarray) -> np.ndarray:
    """Solve the upper-triangular system R y = g."""
    n = R.shape[0]
    y = np.zeros(n, dtype=np.complex128)
    for i in range(n - 1, -1, -1):
        y[i] = (g[i] - R[i, i + 1:n] @ y[i + 1:n]) / R[i, i]
    return y


def arnoldi(apply, v0: np.ndarray, m: int):
    """m steps of Arnoldi with modified Gram-Schmidt for one vector v0
    (shape of one rhs).  Returns V (m+1, ...) and H (m+1, m) without
    rotations, for checking A V_m = V_{m+1} H_m."""
    V = np.zeros((m + 1,) + v0.shape, dtype=v0.dtype)
    H = np.zeros((m + 1, m), dtype=np.complex128)
    V[0] = v0 / np.linalg.norm(v0)
    for j in range(m):
        w = apply(V[j][None])[0]
        for k in range(j + 1):
            H[k, j] = _dot(V[k], w)
            w = w - H[k, j] * V[k]
        H[j + 1, j] = np.linalg.norm(w)
        V[j + 1] = w / H[j + 1, j]
    return V, H


def gmres(apply, b: np.ndarray, tol: float, restart: int = 30, max_restarts: int = 200,
          x0: np.ndarray | None = None, vec_dtype=None, record: bool = False):
    """Batched restarted GMRES.  `apply` maps a block (k, ...) to A times it.

    Returns (x, GmresStats).  x has b's shape, in vec_dtype (default b.dtype)."""
    vec_dtype = np.dtype(vec_dtype or b.dtype)
    nrhs = b.shape[0]
    m = int(restart)
    b = b.astype(vec_dtype)
    x = np.zeros_like(b) if x0 is None else x0.astype(vec_dtype).copy()
    bnorm = _norms(b)
    iters = np.zeros(nrhs, dtype=np.int64)
    restarts = np.zeros(nrhs, dtype=np.int64)
    est = np.zeros(nrhs)
    done = bnorm == 0
    x[done] = 0
    history = []
    for _cycle in range(max_restarts):
        act = np.nonzero(~done)[0]
        if act.size == 0:
            break
        r = b[act] - apply(x[act]).astype(vec_dtype)
        rn = _norms(r)
        ok = rn <= tol * bnorm[act]
        done[act[ok]] = True
        est[act[ok]] = rn[ok] / bnorm[act[ok]]
        act, r, rn = act[~ok], r[~ok], rn[~ok]
        if act.size == 0:
            break
        k = act.size
        restarts[act] += 1
        V = np.zeros((m + 1,) + r.shape, dtype=vec_dtype)
        H = np.zeros((k, m + 1, m), dtype=np.complex128)
        cs = np.zeros((k, m))
        sn = np.zeros((k, m), dtype=np.complex128)
        g = np.zeros((k, m + 1), dtype=np.complex128)
        V[0] = (r / rn.reshape((k,) + (1,) * (r.ndim - 1))).astype(vec_dtype)
        g[:, 0] = rn
        live = np.ones(k, dtype=bool)
        steps = np.zeros(k, dtype=np.int64)
        for j in range(m):
            idx = np.nonzero(live)[0]
            if idx.size == 0:
                break
            w = apply(V[j, idx]).astype(vec_dtype)
            for q, i in enumerate(idx):
                wi = w[q]
                for kk in range(j + 1):
                    h = _dot(V[kk, i], wi)
                    H[i, kk, j] = h
                    wi = wi - np.asarray(h, dtype=vec_dtype) * V[kk, i]
                hn = float(np.sqrt(np.sum(np.abs(wi.astype(np.complex128)) ** 2)))
                H[i, j + 1, j] = hn
                for kk in range(j):
                    t1 = cs[i, kk] * H[i, kk, j] + sn[i, kk] * H[i, kk + 1, j]
                    t2 = -np.conj(sn[i, kk]) * H[i, kk, j] + cs[i, kk] * H[i, kk + 1, j]
                    H[i, kk, j], H[i, kk + 1, j] = t1, t2
                c, s = givens(H[i, j, j], H[i, j + 1, j])
                cs[i, j], sn[i, j] = c, s
                H[i, j, j] = c * H[i, j, j] + s * H[i, j + 1, j]
                H[i, j + 1, j] = 0
                g[i, j + 1] = -np.conj(s) * g[i, j]
                g[i, j] = c * g[i, j]
                steps[i] = j + 1
                rel = abs(g[i, j + 1]) / bnorm[act[i]]
                est[act[i]] = rel
                if hn > 0:
                    V[j + 1, i] = (wi / hn).astype(vec_dtype)
                if rel < tol or hn == 0:
                    live[i] = False
            if record:
                history.append(est[act].copy())
        for i in range(k):
            n = steps[i]
            if n == 0:
                continue
            y = back_substitute(H[i, :n, :n], g[i, :n])
            upd = np.tensordot(y.astype(np.complex128), V[:n, i].astype(np.complex128), axes=(0, 0))
            x[act[i]] = (x[act[i]].astype(np.complex128) + upd).astype(vec_dtype)
            iters[act[i]] += n
    true = np.zeros(nrhs)
    nz = bnorm > 0
    if np.any(nz):
        rr = b[nz].astype(np.complex128) - apply(x[nz]).astype(np.complex128)
        true[nz] = _norms(rr) / bnorm[nz]
    conv = (true <= tol) | ~nz
    return x, GmresStats(iters, restarts, conv, true, est, history)


def gmres_ir(apply_hi, apply_lo, b: np.ndarray, tol: float, inner_tol: float,
             restart: int = 30, max_outer: int = 50, inner_max_restarts: int = 1, lo_dtype=np.complex64):
    """GMRES with iterative refinement: the residual r = b - A x and the
    update x += d are in complex128, the correction A d = r is solved to
    relative accuracy inner_tol by `gmres` with vectors held in lo_dtype and
    the operator `apply_lo` (which applies A in the working precision).

    Returns (x, stats) with stats.iters the total inner Arnoldi steps and
    stats.restarts the outer iterations, per rhs."""
    nrhs = b.shape[0]
    x = np.zeros_like(b, dtype=np.complex128)
    bnorm = _norms(b)
    iters = np.zeros(nrhs, dtype=np.int64)
    outer = np.zeros(nrhs, dtype=np.int64)
    done = bnorm == 0
    for _ in range(max_outer):
        act = np.nonzero(~done)[0]
        if act.size == 0:
            break
        r = b[act] - apply_hi(x[act])
        rel = _norms(r) / bnorm[act]
        ok = rel <= tol
        done[act[ok]] = True
        act, r = act[~ok], r[~ok]
        if act.size == 0:
            break
        d, st = gmres(apply_lo, r.astype(lo_dtype), inner_tol, restart=restart,
                      max_restarts=inner_max_restarts, vec_dtype=lo_dtype)
        x[act] += d.astype(np.complex128)
        iters[act] += st.iters
        outer[act] += 1
    true = np.zeros(nrhs)
    nz = bnorm > 0
    if np.any(nz):
        true[nz] = _norms(b[nz] - apply_hi(x[nz])) / bnorm[nz]
    return x, GmresStats(iters, outer, (true <= tol) | ~nz, true, true.copy())
