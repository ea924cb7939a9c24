"""Solving D_W x = b for a block of right-hand sides with the batched GMRES of
Algorithm 2, on the full system or on the odd-even Schur complement, in
complex128 or as iterative refinement around a lower working precision.

Tolerance reading: the target is the normwise relative true residual of the
FULL system per rhs, ||b_i - D_W x_i|| <= tol ||b_i||.  The Schur solve stops
at ||b'_e - S x_e|| <= tol ||b_i|| (so its own relative tolerance is
tol ||b_i|| / ||b'_e,i||); after reconstruction the odd rows of the full
residual vanish and its even rows equal the Schur residual.
"""
from __future__ import annotations

import numpy as np

from . import dirac, evenodd
from .gmres import GmresStats, _norms, gmres, gmres_ir


def round_f16(a: np.ndarray) -> np.ndarray:
    """Round a block to half-precision storage with one scale per rhs (the
    largest |re| or |im| of that rhs maps to 1), returned as complex64."""
    flat = a.reshape(a.shape[0], -1)
    s = np.maximum(np.max(np.abs(flat.real), axis=1), np.max(np.abs(flat.imag), axis=1))
    s = np.where(s > 0, s, 1.0).astype(np.float32)
    sh = (a.shape[0],) + (1,) * (a.ndim - 1)
    sc = (a / s.reshape(sh)).astype(np.complex64)
    re = sc.real.astype(np.float16).astype(np.float32)
    im = sc.imag.astype(np.float16).astype(np.float32)
    return ((re + 1j * im).astype(np.complex64) * s.reshape(sh)).astype(np.complex64)


def round_links_f16(U: np.ndarray) -> np.ndarray:
    re = U.real.astype(np.float16).astype(np.float32)
    im = U.imag.astype(np.float16).astype(np.float32)
    return (re + 1j * im).astype(np.complex64)


def _operators(U, m0, eo):
    if eo:
        return lambda v: evenodd.apply_schur(U, v, m0)
    return lambda v: dirac.apply_dw(U, v, m0)


def _lo_operator(U, m0, eo, mode):
    if mode == "f32":
        U32 = U.astype(np.complex64)
        op = _operators(U32, np.float32(m0), eo)
        return lambda v: op(v.astype(np.complex64)).astype(np.complex64)
    if mode == "f16":
        U16 = round_links_f16(U)
        op = _operators(U16, np.float32(m0), eo)
        return lambda v: round_f16(op(round_f16(v)))
    raise ValueError(mode)


def solve(U, b, m0, tol=1e-10, restart=30, max_restarts=200, eo=False, mode="f64",
          inner_tol=None, max_outer=60):
    """x = D_W^{-1} b per rhs.  mode "f64" runs complex128 GMRES; "f32"/"f16"
    run iterative refinement (complex128 residual and update, inner GMRES in
    the working precision).  Returns (x, stats) with stats.true_relres the
    full-system relative residual."""
    b = np.asarray(b, dtype=np.complex128)
    bnorm = _norms(b)
    if eo:
        rhs = evenodd.prepare_source(U, b, m0)
        rn = _norms(rhs)
        scale = np.where(rn > 0, bnorm / np.where(rn > 0, rn, 1), 1.0)
    else:
        rhs = b
        scale = np.ones(b.shape[0])
    # Per-rhs tolerance for the reduced system: tol * ||b|| / ||rhs||; the
    # batched solve takes one tolerance, so use the strictest one.
    t = tol * float(np.min(scale))
    op = _operators(U, m0, eo)
    if mode == "f64":
        y, st = gmres(op, rhs, t, restart=restart, max_restarts=max_restarts)
    else:
        lo = _lo_operator(U, m0, eo, mode)
        it = inner_tol if inner_tol is not None else (1e-4 if mode == "f32" else 1e-2)
        y, st = gmres_ir(op, lo, rhs, t, it, restart=restart, max_outer=max_outer)
    x = evenodd.reconstruct(U, b, y, m0) if eo else y
    nz = bnorm > 0
    true = np.zeros(b.shape[0])
    if np.any(nz):
        true[nz] = _norms(b[nz] - dirac.apply_dw(U, x[nz], m0)) / bnorm[nz]
    return x, GmresStats(st.iters, st.restarts, (true <= tol) | ~nz, true, st.est_relres)
