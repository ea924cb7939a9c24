"""GPU parity of dirac_apply and dirac_apply_eo against the oracle.

Tolerances (per rhs, normwise relative): FP64 1e-12, FP32 1e-5 (against the
oracle evaluated in complex128 on the FP32-rounded inputs).  FP16 storage
rounds the output to half precision, whose unit roundoff is 2^-11 = 4.9e-4;
FP32 arithmetic error is far below that, so the bound is 1e-3 against the
oracle on the FP16-rounded inputs."""
import numpy as np
import pytest

import lqcd_synth as syn
import paper_2601_05816_amd as lq
from oracle import closed_forms as cf
from oracle import dirac, evenodd, geometry

from helpers import apply_eo_gpu, apply_gpu, rel_err_per_rhs, rounded

pytestmark = pytest.mark.gpu


@pytest.fixture(params=[1, 2, 3], ids=["site", "pencil_lds", "pencil"], autouse=True)
def kernel_variant(request, gpu_lib):
    """Run every apply test with both Wilson kernel variants."""
    gpu_lib.set_kernel_variant(request.param)
    yield request.param
    gpu_lib.set_kernel_variant(0)
TOL = {lq.F64: 1e-12, lq.F32: 1e-5, lq.F16: 1e-3}
LAYOUTS = [lq.RHS_OUTER, lq.LAYOUT1, lq.LAYOUT2]


def _g5h(x):
    """gamma5 on a half-lattice block (nrhs, V/2, 4, 3)."""
    return dirac.apply_gamma5(x.reshape(x.shape[0], -1, 1, 1, 1, 4, 3)).reshape(x.shape)


_apply_gpu = apply_gpu
_apply_eo_gpu = apply_eo_gpu


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("dagger", [False, True])
def test_apply_4x4x4x4_haar(gpu_lib, layout, dagger):
    dims = (4, 4, 4, 4)
    U = syn.gauge_field(dims, "haar", config=1)
    psi = syn.spinor_block(dims, 1, config=1)
    want = (dirac.apply_dw_dagger if dagger else dirac.apply_dw)(U, psi, 0.1)
    got = _apply_gpu(U, psi, 0.1, layout, lq.F64, dagger)
    assert np.all(rel_err_per_rhs(got, want) <= TOL[lq.F64])


@pytest.mark.parametrize("dims,nrhs", [((2, 2, 2, 6), 3), ((4, 6, 2, 8), 5), ((6, 4, 4, 2), 7), ((2, 2, 2, 2), 1),
                                       ((4, 4, 8, 4), 70)])
@pytest.mark.parametrize("prec", [lq.F64, lq.F32, lq.F16])
def test_apply_ragged_shapes(gpu_lib, dims, nrhs, prec):
    """Extents that differ per direction and work counts that leave a ragged
    last workgroup, in every layout."""
    U = rounded(syn.gauge_field(dims, "haar", config=2), prec)
    psi = rounded(syn.spinor_block(dims, nrhs, config=2), prec)
    want = dirac.apply_dw(U, psi, -0.05)
    for layout in LAYOUTS:
        got = _apply_gpu(U, psi, -0.05, layout, prec)
        assert np.all(rel_err_per_rhs(got, want) <= TOL[prec]), (layout, rel_err_per_rhs(got, want).max())


@pytest.mark.parametrize("nrhs", [1, 4, 12])
@pytest.mark.parametrize("prec", [lq.F64, lq.F32])
def test_apply_16x16x16x32(gpu_lib, nrhs, prec):
    dims = (32, 16, 16, 16)
    U = rounded(syn.gauge_field(dims, "near_identity", config=2, eps=0.3), prec)
    psi = rounded(syn.spinor_block(dims, nrhs, config=2), prec)
    want = dirac.apply_dw(U, psi, -0.05)
    got = _apply_gpu(U, psi, -0.05, lq.LAYOUT2, prec)
    assert np.all(rel_err_per_rhs(got, want) <= TOL[prec])


def test_layouts_bitwise_identical_and_deterministic(gpu_lib):
    dims = (4, 4, 4, 8)
    U = syn.gauge_field(dims, "near_identity", config=3)
    psi = syn.spinor_block(dims, 6, config=3)
    outs = [_apply_gpu(U, psi, 0.05, layout, lq.F64) for layout in LAYOUTS]
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])
    assert np.array_equal(outs[2], _apply_gpu(U, psi, 0.05, lq.LAYOUT2, lq.F64))


@pytest.mark.parametrize("layout", LAYOUTS)
@pytest.mark.parametrize("prec", [lq.F64, lq.F32, lq.F16])
@pytest.mark.parametrize("dagger", [False, True])
def test_schur_apply(gpu_lib, layout, prec, dagger):
    dims = (4, 4, 6, 4)
    U = rounded(syn.gauge_field(dims, "haar", config=4), prec)
    psi = rounded(syn.spinor_block(dims, 3, config=4), prec)
    psi_e = geometry.to_half(psi, dims, 0)
    if dagger:
        # S^dagger = gamma5 S gamma5
        want = _g5h(evenodd.apply_schur(U, _g5h(psi_e), 0.1))
    else:
        want = evenodd.apply_schur(U, psi_e, 0.1)
    got = _apply_eo_gpu(U, psi_e, 0.1, layout, prec, dagger)
    assert np.all(rel_err_per_rhs(got, want) <= TOL[prec])


@pytest.mark.parametrize("nrhs", [1, 12])
def test_schur_apply_16x16x16x32(gpu_lib, nrhs):
    dims = (32, 16, 16, 16)
    U = syn.gauge_field(dims, "near_identity", config=2, eps=0.3)
    psi = syn.spinor_block(dims, nrhs, config=2)
    psi_e = geometry.to_half(psi, dims, 0)
    want = evenodd.apply_schur(U, psi_e, -0.05)
    got = _apply_eo_gpu(U, psi_e, -0.05, lq.LAYOUT2, lq.F64)
    assert np.all(rel_err_per_rhs(got, want) <= TOL[lq.F64])


def test_full_size_pure_gauge_plane_waves(gpu_lib):
    """32^3 x 64, 16 rhs, the launch configuration of the benchmark: with
    U_mu(x) = G(x) G(x+mu)^dag and psi = G(x) e^{ip.x} u the exact result is
    G(x) e^{ip.x} M(p) u (checked on a sample of sites); plus the oracle's
    site-by-site apply on a random field at sampled sites."""
    import torch

    dims = (64, 32, 32, 32)
    nrhs = 16
    m0 = -0.05
    G = syn.gauge_transform(dims, config=3)
    U = cf.pure_gauge_links(G)
    modes = syn.plane_wave_modes(dims, config=3, count=nrhs)
    rng = np.random.default_rng(7)
    sites = np.sort(rng.choice(int(np.prod(dims)), size=4096, replace=False))
    coords = np.stack(np.unravel_index(sites, dims), axis=-1)
    Gs = G.reshape(-1, 3, 3)[sites]
    psi_dev = torch.empty(dims + (4, 3, nrhs), dtype=torch.complex128, device="cuda")
    want = np.empty((nrhs, sites.size, 4, 3), dtype=np.complex128)
    for i, (n, u) in enumerate(modes):
        p = cf.momenta(n, dims)
        wave = cf.colour_rotate(G, cf.plane_wave(dims, p, u))
        psi_dev[..., i] = torch.from_numpy(wave).to("cuda")
        ph = np.exp(1j * coords @ p)
        want[i] = ph[:, None, None] * np.einsum("kab,sb->ksa", Gs, cf.free_symbol(p, m0) @ u)
    Ud = torch.from_numpy(U).to("cuda")
    out = lq.dirac_apply(Ud, psi_dev, m0, layout=lq.LAYOUT2)
    got = out.reshape(-1, 4, 3, nrhs)[torch.from_numpy(sites).to("cuda")].cpu().numpy()
    got = np.moveaxis(got, -1, 0)
    assert np.all(rel_err_per_rhs(got, want) <= TOL[lq.F64])
    # Gaussian spinors on the same field, the oracle's site-by-site apply at sampled sites
    psi2 = syn.spinor_block(dims, nrhs, config=3)
    out2 = lq.dirac_apply(Ud, torch.from_numpy(np.ascontiguousarray(np.moveaxis(psi2, 0, -1))).to("cuda"), m0,
                          layout=lq.LAYOUT2)
    few = sites[::16]
    got2 = np.moveaxis(out2.reshape(-1, 4, 3, nrhs)[torch.from_numpy(few).to("cuda")].cpu().numpy(), -1, 0)
    want2 = dirac.apply_dw_sites(U, psi2, m0, few)
    assert np.all(rel_err_per_rhs(got2, want2) <= TOL[lq.F64])
