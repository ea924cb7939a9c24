"""GPU gmres_solve against the oracle.

A solve is accepted when the oracle, applied to the GPU's x in complex128,
finds ||b - D x|| <= tol ||b|| for every rhs (one oracle apply checks a
solution without an oracle solve); small cases also compare x with dense LU
within kappa * tol and iteration counts with the oracle's GMRES."""
import numpy as np
import pytest

import lqcd_synth as syn
import paper_2601_05816_amd as lq
from oracle import closed_forms as cf
from oracle import dirac, gmres as ogmres

from helpers import from_layout_np, rel_err_per_rhs, to_layout_np

pytestmark = pytest.mark.gpu


def _solve(U, b, m0, layout=lq.LAYOUT2, x0=None, **kw):
    import torch

    Ud = torch.from_numpy(U).to("cuda")
    bd = torch.from_numpy(to_layout_np(b, layout)).to("cuda")
    x0d = None if x0 is None else torch.from_numpy(to_layout_np(x0, layout)).to("cuda")
    x, st, rc = lq.gmres_solve(Ud, bd, m0, layout=layout, x0=x0d, **kw)
    return from_layout_np(x.cpu().numpy(), layout, 4), st, rc


def _true_relres(U, b, x, m0):
    return rel_err_per_rhs(dirac.apply_dw(U, x, m0), b)


@pytest.mark.parametrize("eo", [False, True])
def test_4x4x4x4_haar_dense_lu(gpu_lib, eo):
    dims = (4, 4, 4, 4)
    m0 = 0.1
    U = syn.gauge_field(dims, "haar", config=1)
    b = syn.spinor_block(dims, 1, config=1)
    x, st, rc = _solve(U, b, m0, restart=30, eo=eo, tol=1e-10)
    assert rc == lq.OK and st["converged"].all()
    rr = _true_relres(U, b, x, m0)
    assert np.all(rr <= 1e-10)
    assert np.allclose(rr, st["true_relres"], rtol=1e-2, atol=1e-15)
    D = dirac.dense(U, m0)
    x_lu = np.linalg.solve(D, b.reshape(1, -1).T).T.reshape(b.shape)
    assert rel_err_per_rhs(x, x_lu)[0] <= np.linalg.cond(D) * 1e-10
    if not eo:
        # iteration count of the oracle's GMRES (MGS) on the same system: the
        # GPU (CGS) may differ by rounding only
        _, ost = ogmres.gmres(lambda v: dirac.apply_dw(U, v, m0), b, 1e-10, restart=30)
        assert abs(int(st["iters"][0]) - int(ost.iters[0])) <= 2


@pytest.mark.parametrize("layout", [lq.RHS_OUTER, lq.LAYOUT1, lq.LAYOUT2])
@pytest.mark.parametrize("mode", ["f64", "ir-f32", "ir-f16"])
def test_ragged_shapes_all_modes(gpu_lib, layout, mode):
    dims = (4, 6, 2, 8)
    m0 = 0.05
    U = syn.gauge_field(dims, "near_identity", config=2, eps=0.3)
    b = syn.spinor_block(dims, 5, config=2)
    x, st, rc = _solve(U, b, m0, layout=layout, restart=12, eo=True, mode=mode, tol=1e-10)
    assert rc == lq.OK, st
    assert np.all(_true_relres(U, b, x, m0) <= 1e-10)
    if mode != "f64":
        assert np.all(st["outer_iters"] >= 2)


@pytest.mark.parametrize("nrhs", [1, 4, 12])
def test_16x16x16x32_eo_modes(gpu_lib, nrhs):
    dims = (32, 16, 16, 16)
    m0 = -0.05
    U = syn.gauge_field(dims, "near_identity", config=2, eps=0.3)
    b = syn.spinor_block(dims, nrhs, config=2)
    xs = {}
    for mode in ("f64", "ir-f32"):
        x, st, rc = _solve(U, b, m0, restart=30, eo=True, mode=mode, tol=1e-10)
        assert rc == lq.OK and st["converged"].all(), (mode, st)
        assert np.all(_true_relres(U, b, x, m0) <= 1e-10), mode
        xs[mode] = x
    # both modes reach the same solution to the accuracy the residual allows
    assert np.all(rel_err_per_rhs(xs["ir-f32"], xs["f64"]) <= 1e-7)


def test_full_vs_eo_same_solution(gpu_lib):
    dims = (8, 4, 4, 4)
    m0 = 0.1
    U = syn.gauge_field(dims, "near_identity", config=3)
    b = syn.spinor_block(dims, 3, config=3)
    xf, sf, _ = _solve(U, b, m0, eo=False)
    xe, se, _ = _solve(U, b, m0, eo=True)
    assert np.all(rel_err_per_rhs(xe, xf) <= 1e-8)
    assert np.all(se["iters"] < sf["iters"])      # the Schur system needs fewer steps


def test_zero_rhs_and_breakdown(gpu_lib):
    dims = (4, 4, 4, 4)
    m0 = 0.1
    U = syn.gauge_field(dims, "unit", config=0)
    n, _ = syn.plane_wave_modes(dims, config=25, count=1)[0]
    p = cf.momenta(n, dims)
    w, vecs = np.linalg.eig(cf.free_symbol(p, m0))
    u = np.outer(vecs[:, 0], [1.0, 0.5j, -0.25])
    b = np.stack([cf.plane_wave(dims, p, u), np.zeros(dims + (4, 3), dtype=np.complex128),
                  syn.spinor_block(dims, 1, config=4)[0]])
    x, st, rc = _solve(U, b, m0, eo=False, tol=1e-12)
    assert rc == lq.OK
    assert st["iters"][0] == 1 and np.allclose(x[0], b[0] / w[0], atol=1e-13)
    assert np.all(x[1] == 0) and st["iters"][1] == 0 and st["converged"][1]
    assert st["iters"][2] > 1


def test_not_converged_and_guess(gpu_lib):
    dims = (4, 4, 4, 4)
    m0 = -0.05
    U = syn.gauge_field(dims, "haar", config=5)
    b = syn.spinor_block(dims, 2, config=5)
    x, st, rc = _solve(U, b, m0, eo=False, restart=5, max_restarts=1)
    assert rc == lq.NOT_CONVERGED
    assert not st["converged"].any() and np.all(st["iters"] == 5) and np.all(st["true_relres"] > 1e-10)
    # resuming from the last iterate is the restart checkpoint
    x2, st2, rc2 = _solve(U, b, m0, x0=x, eo=False, restart=30)
    assert rc2 == lq.OK and np.all(_true_relres(U, b, x2, m0) <= 1e-10)
    # an exact guess needs no iterations
    x3, st3, rc3 = _solve(U, b, m0, x0=x2, eo=False, tol=1e-9)
    assert rc3 == lq.OK and np.all(st3["iters"] == 0)


def test_fixed_iterations_match_oracle(gpu_lib):
    """The paper's solver protocol: exactly 10 restarts of length 10."""
    dims = (4, 4, 4, 8)
    m0 = 0.1
    U = syn.gauge_field(dims, "near_identity", config=6)
    b = syn.spinor_block(dims, 2, config=6)
    x, st, rc = _solve(U, b, m0, eo=False, restart=10, max_restarts=10, fixed_iters=True)
    assert rc == lq.OK and np.all(st["iters"] == 100)
    xo, ost = ogmres.gmres(lambda v: dirac.apply_dw(U, v, m0), b, 0.0, restart=10, max_restarts=10)
    assert np.all(ost.iters == 100)
    assert np.all(rel_err_per_rhs(x, xo) <= 1e-9)


def test_errors(gpu_lib):
    import torch

    dims = (4, 4, 4, 4)
    U = torch.from_numpy(syn.gauge_field(dims, "haar", config=7)).to("cuda")
    b = torch.from_numpy(to_layout_np(syn.spinor_block(dims, 2, config=7), lq.LAYOUT2)).to("cuda")
    with pytest.raises(lq.LqcdError) as e:
        lq.gmres_solve(U, b, -4.0, eo=True)
    assert e.value.code == -7
    bad = b.clone()
    bad[0, 0, 0, 0, 0, 0, 1] = float("nan")
    with pytest.raises(lq.LqcdError) as e:
        lq.gmres_solve(U, bad, 0.1, eo=True)
    assert e.value.code == -8
    small = torch.empty(16, dtype=torch.uint8, device="cuda")
    p = lq.solver_params()
    import ctypes
    rc = lq.load().gmres_solve(ctypes.byref(lq._lattice(dims)), U.data_ptr(), b.data_ptr(), b.data_ptr(), 2, 0.1,
                               lq.LAYOUT2, ctypes.byref(p), small.data_ptr(), 16, None, None)
    assert rc == -6


@pytest.mark.parametrize("eo", [False, True])
@pytest.mark.parametrize("mode", ["f64", "ir-f32"])
def test_adjoint_solve(gpu_lib, eo, mode):
    """dagger = 1 solves D^dagger x = b (the adjoint solve of a gradient)."""
    dims = (4, 4, 6, 4)
    m0 = 0.1
    U = syn.gauge_field(dims, "near_identity", config=8, eps=0.3)
    b = syn.spinor_block(dims, 3, config=8)
    x, st, rc = _solve(U, b, m0, eo=eo, mode=mode, tol=1e-10, dagger=True)
    assert rc == lq.OK
    assert np.all(rel_err_per_rhs(dirac.apply_dw_dagger(U, x, m0), b) <= 1e-10)


@pytest.mark.parametrize("mode", ["ir-f32", "ir-f16"])
@pytest.mark.parametrize("variant", [0, 4])
def test_refinement_vector_paths(gpu_lib, mode, variant):
    """nrhs divisible by four: the 16-byte-per-lane BLAS kernels of the FP32 /
    FP16 bases and (variant 4) the two-rhs-per-lane Schur kernels."""
    gpu_lib.set_kernel_variant(variant)
    dims = (8, 8, 4, 8)
    m0 = 0.05
    U = syn.gauge_field(dims, "near_identity", config=9, eps=0.3)
    b = syn.spinor_block(dims, 8, config=9)
    x, st, rc = _solve(U, b, m0, restart=16, eo=True, mode=mode, tol=1e-10)
    gpu_lib.set_kernel_variant(0)
    assert rc == lq.OK
    assert np.all(_true_relres(U, b, x, m0) <= 1e-10)


@pytest.mark.parametrize("gs", ["cgs2", "mgs"])
def test_orthogonalisation_options(gpu_lib, gs):
    """CGS2 and MGS (Algorithm 2 leaves the orthogonalisation open): the fixed
    10 x 10 protocol gives the oracle's (MGS) iterate, a converged solve
    matches dense LU within kappa * tol with the oracle's iteration count, and
    the FP32 refinement and the lock-step batch run with them."""
    dims = (4, 4, 4, 8)
    m0 = 0.1
    U = syn.gauge_field(dims, "near_identity", config=6)
    b = syn.spinor_block(dims, 2, config=6)
    x, st, rc = _solve(U, b, m0, eo=False, restart=10, max_restarts=10, fixed_iters=True, gs=gs)
    assert rc == lq.OK and np.all(st["iters"] == 100)
    xo, ost = ogmres.gmres(lambda v: dirac.apply_dw(U, v, m0), b, 0.0, restart=10, max_restarts=10)
    assert np.all(rel_err_per_rhs(x, xo) <= 1e-9)
    dims = (4, 4, 4, 4)
    U = syn.gauge_field(dims, "haar", config=1)
    b = syn.spinor_block(dims, 3, config=1)
    x, st, rc = _solve(U, b, m0, restart=30, eo=False, tol=1e-10, gs=gs)
    assert rc == lq.OK and np.all(_true_relres(U, b, x, m0) <= 1e-10)
    D = dirac.dense(U, m0)
    x_lu = np.linalg.solve(D, b.reshape(3, -1).T).T.reshape(b.shape)
    assert np.all(rel_err_per_rhs(x, x_lu) <= np.linalg.cond(D) * 1e-10)
    _, ost = ogmres.gmres(lambda v: dirac.apply_dw(U, v, m0), b, 1e-10, restart=30)
    assert np.all(np.abs(st["iters"] - ost.iters) <= 2)
    x, st, rc = _solve(U, b, m0, restart=30, eo=True, mode="ir-f32", tol=1e-10, gs=gs)
    assert rc == lq.OK and np.all(_true_relres(U, b, x, m0) <= 1e-10)


@pytest.mark.parametrize("layout", [lq.RHS_OUTER, lq.LAYOUT1, lq.LAYOUT2])
def test_rhs_chunked_solves(gpu_lib, layout):
    """rhs_block: a solve in chunks of consecutive rhs gives every rhs the
    result of the unchunked solve (the same arithmetic per rhs up to the
    order of partial sums): the fixed 10 x 10 protocol to 1e-12, converged
    solves to the residual bound with the same step counts (+-1), in FP64
    and FP32 refinement, with and without an initial guess; with
    rhs_block = 0 and a workspace that holds only two rhs the library picks
    width 2."""
    import torch

    dims = (4, 4, 4, 8)
    m0 = 0.1
    U = syn.gauge_field(dims, "near_identity", config=7, eps=0.3)
    b = syn.spinor_block(dims, 6, config=7)
    xa, sa, _ = _solve(U, b, m0, layout=layout, eo=True, restart=10, max_restarts=10, fixed_iters=True)
    xc, sc, rc = _solve(U, b, m0, layout=layout, eo=True, restart=10, max_restarts=10, fixed_iters=True, rhs_block=4)
    assert rc == lq.OK and np.all(sc["iters"] == sa["iters"])
    assert np.all(rel_err_per_rhs(xc, xa) <= 1e-12)
    for mode in ("f64", "ir-f32"):
        xa, sa, _ = _solve(U, b, m0, layout=layout, eo=True, mode=mode, tol=1e-10)
        xc, sc, rc = _solve(U, b, m0, layout=layout, eo=True, mode=mode, tol=1e-10, rhs_block=4)
        assert rc == lq.OK and np.all(_true_relres(U, b, xc, m0) <= 1e-10), mode
        assert np.all(np.abs(sc["iters"] - sa["iters"]) <= 1), mode
        assert np.all(rel_err_per_rhs(xc, xa) <= 1e-8), mode
    # an initial guess: chunks read their columns of x0
    xg, sg, rc = _solve(U, b, m0, layout=layout, x0=xa, eo=True, tol=1e-9, rhs_block=5)
    assert rc == lq.OK and np.all(sg["iters"] == 0)
    # automatic width from the workspace
    p = lq.solver_params(eo=True, tol=1e-10, rhs_block=2)
    work = torch.empty(lq.gmres_workspace_bytes(dims, 6, p), dtype=torch.uint8, device="cuda")
    p0 = lq.solver_params(eo=True, tol=1e-10)
    assert lq.gmres_rhs_block(dims, 6, p0, work.numel()) == 2
    xw, sw, rc = _solve(U, b, m0, layout=layout, work=work, eo=True, tol=1e-10)
    assert rc == lq.OK and np.all(_true_relres(U, b, xw, m0) <= 1e-10)


def test_solution_buffer(gpu_lib):
    """out= receives x (the same tensor comes back), with and without an
    initial guess copied into it; the results equal those of a new tensor
    and of x0= alone bit for bit; a buffer of the wrong shape is rejected."""
    import torch

    dims = (8, 4, 4, 4)
    m0 = -0.05
    U = torch.from_numpy(syn.gauge_field(dims, "near_identity", config=5, eps=0.3)).to("cuda")
    b = torch.from_numpy(to_layout_np(syn.spinor_block(dims, 3, config=5), lq.LAYOUT2)).to("cuda")
    kw = dict(restart=10, eo=True, tol=1e-10)
    x_new, _, rc = lq.gmres_solve(U, b, m0, **kw)
    out = torch.full_like(b, float("nan"))
    x_out, _, rc2 = lq.gmres_solve(U, b, m0, out=out, **kw)
    assert rc == rc2 == lq.OK and x_out is out and torch.equal(x_out, x_new)
    x0 = 0.5 * x_new
    x_g, _, _ = lq.gmres_solve(U, b, m0, x0=x0, **kw)
    out2 = torch.empty_like(b)
    x_g2, _, _ = lq.gmres_solve(U, b, m0, x0=x0, out=out2, **kw)
    assert x_g2 is out2 and torch.equal(x_g2, x_g) and torch.equal(x0, 0.5 * x_new)
    with pytest.raises(ValueError):
        lq.gmres_solve(U, b, m0, out=torch.empty_like(b[..., :2]), **kw)
