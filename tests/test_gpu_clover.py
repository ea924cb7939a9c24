"""The clover-improved operator D = D_W - C on the GPU against the oracle:
full apply (three precisions, three layouts, D and D^dagger), the site-local
inverse of D_oo, and the odd-even Schur complement with a site-dependent
D_oo; a full-size case checked on sampled sites.  The apply tests run with
both kernel kinds configured (one work item per site and rhs; time-streaming
pencils)."""
import numpy as np
import pytest

import lqcd_synth as syn
import paper_2601_05816_amd as lq
from oracle import clover, dirac, geometry

from helpers import from_dev, from_layout_np, rel_err_per_rhs, rounded, to_dev, to_layout_np

pytestmark = pytest.mark.gpu
TOL = {lq.F64: 1e-12, lq.F32: 1e-5, lq.F16: 1e-3}
LAYOUTS = [lq.RHS_OUTER, lq.LAYOUT1, lq.LAYOUT2]


def _g5h(x):
    return dirac.apply_gamma5(x.reshape(x.shape[0], -1, 1, 1, 1, 4, 3)).reshape(x.shape)


@pytest.fixture(params=[1, 3], ids=["site", "pencil"])
def clover_kernel(request, gpu_lib):
    """The apply tests run with the plain operator configured for the
    one-(site, rhs) kernels and for the time-streaming pencils: the full
    clover apply follows that choice (the odd-even clover passes always take
    the one-(site, rhs) kernels).  The solves run with the tuned default."""
    gpu_lib.set_kernel_variant(request.param)
    yield request.param
    gpu_lib.set_kernel_variant(0)


@pytest.mark.parametrize("prec", [lq.F64, lq.F32, lq.F16])
@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("dagger", [False, True])
def test_clover_apply_vs_oracle(gpu_lib, clover_kernel, prec, layout, dagger):
    dims = (4, 4, 6, 4)
    U = rounded(syn.gauge_field(dims, "haar", config=21), prec)
    cp = rounded(syn.clover_field(dims, config=21, scale=0.4), prec)
    psi = rounded(syn.spinor_block(dims, 3, config=21), prec)
    want = (clover.apply_dwc_dagger if dagger else clover.apply_dwc)(U, cp, psi, 0.1)
    out = lq.dirac_apply_clover(to_dev(U, prec), to_dev(cp, prec), to_dev(to_layout_np(psi, layout), prec), 0.1,
                                layout=layout, dagger=dagger)
    got = from_layout_np(from_dev(out, prec), layout, 4)
    assert np.all(rel_err_per_rhs(got, want) <= TOL[prec])


@pytest.mark.parametrize("prec", [lq.F64, lq.F32])
def test_clover_inverse_vs_oracle(gpu_lib, prec):
    dims = (4, 2, 4, 2)
    cp = rounded(syn.clover_field(dims, config=22, scale=0.5), prec)
    got = lq.clover_inverse(to_dev(cp, prec), -0.3, dims)
    g = got.cpu().numpy().astype(np.complex128)
    want = clover.diagonal_inverse(cp, -0.3)
    assert np.abs(g - want).max() <= (1e-13 if prec == lq.F64 else 1e-6) * np.abs(want).max()


def test_clover_inverse_singular(gpu_lib):
    dims = (2, 2, 2, 2)
    cp = np.zeros(dims + (42,), dtype=np.complex128)
    cp[0, 1, 0, 1, 21 + 3] = 3.9  # (4 + m0) - C singular on one site (m0 = -0.1)
    with pytest.raises(lq.LqcdError) as e:
        lq.clover_inverse(to_dev(cp, lq.F64), -0.1, dims)
    assert e.value.code == -7


@pytest.mark.parametrize("prec", [lq.F64, lq.F32])
@pytest.mark.parametrize("layout", [lq.LAYOUT1, lq.LAYOUT2])
def test_clover_schur_vs_oracle(gpu_lib, clover_kernel, prec, layout):
    """S and S^dagger = gamma5 S gamma5 with the clover term."""
    dims = (4, 4, 2, 6)
    m0 = -0.2
    U = rounded(syn.gauge_field(dims, "near_identity", config=23, eps=0.4), prec)
    cp = rounded(syn.clover_field(dims, config=23, scale=0.3), prec)
    psi = rounded(syn.spinor_block(dims, 4, config=23), prec)
    pe = geometry.to_half(psi, dims, 0)
    Cd = to_dev(cp, prec)
    Ci = lq.clover_inverse(Cd, m0, dims)
    want = clover.apply_schur(U, cp, pe, m0)
    for dagger in (False, True):
        out = lq.dirac_apply_eo_clover(to_dev(U, prec), Cd, Ci, to_dev(to_layout_np(pe, layout), prec), m0,
                                       layout=layout, dagger=dagger)
        got = from_layout_np(from_dev(out, prec), layout, 1)
        w = _g5h(clover.apply_schur(U, cp, _g5h(pe), m0)) if dagger else want
        assert np.all(rel_err_per_rhs(got, w) <= TOL[prec] * 4)


def test_clover_full_size_sampled(gpu_lib, clover_kernel):
    """32^3 x 64, 16 rhs, FP64: sampled sites against the oracle's site-by-site
    Wilson apply minus C(x) psi(x)."""
    import torch

    dims = (64, 32, 32, 32)
    m0 = -0.05
    U = syn.gauge_field(dims, "near_identity", config=3, eps=0.3)
    cp = syn.clover_field(dims, config=3, scale=0.2)
    psi = syn.spinor_block(dims, 16, config=3)
    out = lq.dirac_apply_clover(torch.from_numpy(U).to("cuda"), torch.from_numpy(cp).to("cuda"),
                                torch.from_numpy(np.ascontiguousarray(np.moveaxis(psi, 0, -1))).to("cuda"), m0)
    sites = np.random.default_rng(5).choice(int(np.prod(dims)), size=48, replace=False)
    got = np.moveaxis(out.reshape(-1, 4, 3, 16)[torch.from_numpy(sites).to("cuda")].cpu().numpy(), -1, 0)
    w = dirac.apply_dw_sites(U, psi, m0, sites)
    flat = psi.reshape(16, -1, 12)[:, sites]
    cm = clover.site_matrix(cp.reshape(-1, 42)[sites])
    w = w - np.einsum("sij,nsj->nsi", cm, flat).reshape(w.shape)
    assert np.all(rel_err_per_rhs(got, w) <= 1e-12)


@pytest.mark.parametrize("eo", [True, False])
@pytest.mark.parametrize("mode", ["f64", "ir-f32", "ir-f16"])
@pytest.mark.parametrize("dagger", [False, True])
def test_clover_solve_vs_dense_lu(gpu_lib, eo, mode, dagger):
    """gmres_solve_clover on 4^4 against numpy's dense LU of D = D_W - C (or D^dagger)."""
    import torch

    dims = (4, 4, 4, 4)
    m0 = 0.1
    U = syn.gauge_field(dims, "near_identity", config=24, eps=0.3)
    cp = syn.clover_field(dims, config=24, scale=0.3)
    b = syn.spinor_block(dims, 2, config=24)
    D = clover.dense(U, cp, m0)
    A = D.conj().T if dagger else D
    want = np.linalg.solve(A, b.reshape(2, -1).T).T.reshape(b.shape)
    x, st, rc = lq.gmres_solve_clover(torch.from_numpy(U).to("cuda"), torch.from_numpy(cp).to("cuda"),
                                      torch.from_numpy(np.ascontiguousarray(np.moveaxis(b, 0, -1))).to("cuda"), m0,
                                      eo=eo, mode=mode, tol=1e-11, dagger=dagger, restart=20)
    assert rc == lq.OK and np.all(st["converged"] == 1)
    got = np.moveaxis(x.cpu().numpy(), -1, 0)
    kappa = np.linalg.cond(D)
    assert np.all(rel_err_per_rhs(got, want) <= 1e-11 * kappa)


def test_clover_solve_16x16x16x32_residual(gpu_lib):
    """16^3 x 32, 4 rhs, odd-even, FP32 refinement: the oracle's clover apply on
    the GPU's solution reproduces b to 1e-10."""
    import torch

    dims = (32, 16, 16, 16)
    m0 = -0.05
    U = syn.gauge_field(dims, "near_identity", config=25, eps=0.3)
    cp = syn.clover_field(dims, config=25, scale=0.2)
    b = syn.spinor_block(dims, 4, config=25)
    x, st, rc = lq.gmres_solve_clover(torch.from_numpy(U).to("cuda"), torch.from_numpy(cp).to("cuda"),
                                      torch.from_numpy(np.ascontiguousarray(np.moveaxis(b, 0, -1))).to("cuda"), m0,
                                      eo=True, mode="ir-f32", tol=1e-10, use_graph=True)
    assert rc == lq.OK
    xs = np.moveaxis(x.cpu().numpy(), -1, 0)
    assert np.all(rel_err_per_rhs(clover.apply_dwc(U, cp, xs, m0), b) <= 1e-10)
    assert np.all(st["true_relres"] <= 1e-10)


def test_clover_singular_site_rejected(gpu_lib):
    import torch

    dims = (4, 4, 4, 4)
    U = syn.gauge_field(dims, "near_identity", config=26)
    cp = np.zeros(dims + (42,), dtype=np.complex128)
    cp[1, 0, 0, 0, 2] = 4.1  # (4 + m0) - C singular at an odd site for m0 = 0.1
    b = syn.spinor_block(dims, 1, config=26)
    with pytest.raises(lq.LqcdError) as e:
        lq.gmres_solve_clover(torch.from_numpy(U).to("cuda"), torch.from_numpy(cp).to("cuda"),
                              torch.from_numpy(np.ascontiguousarray(np.moveaxis(b, 0, -1))).to("cuda"), 0.1, eo=True)
    assert e.value.code == -7
