"""GPU parity of the fused Schur kernel (variant 8: the odd field H_oe psi_e
of a workgroup's tile and its y / z halo computed into LDS one time slice at
a time and H_eo applied there) against the oracle's Schur complement, in
three precisions, three layouts, D and D^dagger, several tiles, residency
shares, t segments and rhs counts (one to several rhs chunks), inside the
odd-even solvers, and through the workspace and allocation-free entry
points.  A NaN-filled workspace that the apply leaves untouched shows that
the fused kernel, not the two hop passes, produced the result."""
import numpy as np
import pytest

import lqcd_synth as syn
import paper_2601_05816_amd as lq
from oracle import dirac, evenodd, geometry

from helpers import from_dev, from_layout_np, rel_err_per_rhs, rounded, to_dev, to_layout_np

pytestmark = pytest.mark.gpu

TOL = {lq.F64: 1e-12, lq.F32: 1e-5, lq.F16: 1e-3}
LAYOUTS = [lq.RHS_OUTER, lq.LAYOUT1, lq.LAYOUT2]


def _g5h(x):
    """gamma5 on a half-lattice block (nrhs, V/2, 4, 3)."""
    return dirac.apply_gamma5(x.reshape(x.shape[0], -1, 1, 1, 1, 4, 3)).reshape(x.shape)


@pytest.fixture(autouse=True)
def automatic_selection_after(gpu_lib):
    yield
    gpu_lib.set_kernel_config(0)


def _schur_ws(U, psi_e, m0, layout, prec, dagger=False):
    """dirac_apply_eo_ws with a NaN-filled workspace; returns the result and
    whether the workspace was left untouched."""
    import torch

    dims = U.shape[1:5]
    Ud = to_dev(U, prec)
    pd = to_dev(to_layout_np(psi_e, layout), prec)
    nrhs = psi_e.shape[0]
    work = torch.full((lq.dirac_apply_eo_workspace_bytes(dims, nrhs, prec),), 0xFF, dtype=torch.uint8,
                      device=pd.device)
    out = lq.dirac_apply_eo_ws(Ud, pd, m0, work, layout=layout, dagger=dagger)
    torch.cuda.synchronize()
    untouched = bool((work == 0xFF).all().item())
    return from_layout_np(from_dev(out, prec), layout, 1), untouched


def _want(U, psi_e, m0, dagger):
    if dagger:  # S^dagger = gamma5 S gamma5
        return _g5h(evenodd.apply_schur(U, _g5h(psi_e), m0))
    return evenodd.apply_schur(U, psi_e, m0)


@pytest.mark.parametrize("prec", [lq.F64, lq.F32, lq.F16])
@pytest.mark.parametrize("dims,nrhs", [((8, 4, 4, 4), 5), ((6, 4, 6, 8), 4), ((4, 6, 2, 4), 3),
                                       ((4, 4, 4, 8), 16)])
@pytest.mark.parametrize("cfg", [(0, 0, 0, 0, 1), (2, 2, 0, 1, 2), (1, 2, 2, 0, 1), (2, 1, 0, 0, 2)])
def test_fused_schur_matches_oracle(gpu_lib, prec, dims, nrhs, cfg):
    """cfg = (tile_y, tile_z, segments, nontemporal, wg_per_cu).  Lattices
    include a y extent of 2 (the y halo rows wrap onto the interior rows),
    rhs counts that give one rhs per workgroup and several chunks."""
    ty, tz, seg, nt, occ = cfg
    gpu_lib.set_kernel_config(8, ty, tz, seg, nt, occ)
    U = rounded(syn.gauge_field(dims, "haar", config=21), prec)
    psi = rounded(syn.spinor_block(dims, nrhs, config=21), prec)
    psi_e = geometry.to_half(psi, dims, 0)
    for layout in LAYOUTS:
        for dagger in (False, True):
            got, untouched = _schur_ws(U, psi_e, -0.2, layout, prec, dagger)
            if dims[2] % max(ty, 1) == 0 and dims[1] % max(tz, 1) == 0:
                assert untouched, (layout, dagger)
            assert np.all(rel_err_per_rhs(got, _want(U, psi_e, -0.2, dagger)) <= TOL[prec] * 2), (layout, dagger)


@pytest.mark.parametrize("prec", [lq.F64, lq.F32])
def test_fused_schur_allocating_and_noalloc_entries(gpu_lib, prec):
    """dirac_apply_eo and dirac_apply_eo_noalloc run the same fused kernel."""
    import torch

    gpu_lib.set_kernel_config(8)
    dims = (6, 4, 4, 8)
    U = rounded(syn.gauge_field(dims, "haar", config=22), prec)
    psi_e = geometry.to_half(rounded(syn.spinor_block(dims, 6, config=22), prec), dims, 0)
    want = evenodd.apply_schur(U, psi_e, 0.1)
    Ud = to_dev(U, prec)
    pd = to_dev(to_layout_np(psi_e, lq.LAYOUT2), prec)
    got = from_layout_np(from_dev(lq.dirac_apply_eo(Ud, pd, 0.1), prec), lq.LAYOUT2, 1)
    assert np.all(rel_err_per_rhs(got, want) <= TOL[prec] * 2)
    out = torch.empty_like(pd)
    lq.dirac_apply_eo_noalloc(Ud, pd, 0.1, out)
    got = from_layout_np(from_dev(out, prec), lq.LAYOUT2, 1)
    assert np.all(rel_err_per_rhs(got, want) <= TOL[prec] * 2)


def test_fused_schur_larger_lattice(gpu_lib):
    """16^3 x 32 (four x-rows of 8 compact columns per tile row, 64 tiles of
    2 x 2, 16 rhs in chunks): every rhs against the oracle."""
    gpu_lib.set_kernel_config(8, 2, 2, 0, 1, 1)
    dims = (32, 16, 16, 16)
    U = syn.gauge_field(dims, "near_identity", config=23, eps=0.3)
    psi_e = geometry.to_half(syn.spinor_block(dims, 16, config=23), dims, 0)
    got, untouched = _schur_ws(U, psi_e, -0.05, lq.LAYOUT2, lq.F64)
    assert untouched
    assert np.all(rel_err_per_rhs(got, evenodd.apply_schur(U, psi_e, -0.05)) <= TOL[lq.F64])


def test_fused_schur_in_solves(gpu_lib):
    """The fused kernel as the odd-even operator of GMRES (converged rhs are
    masked: their stores are skipped): FP64 and both refinement modes reach
    a true 1e-10 on every rhs, checked with the oracle's D_W."""
    gpu_lib.set_kernel_config(8)
    dims = (8, 4, 4, 8)
    m0 = -0.05
    U = syn.gauge_field(dims, "near_identity", config=24, eps=0.3)
    b = syn.spinor_block(dims, 6, config=24)
    b[2] *= 1e-3
    Ud = to_dev(U, lq.F64)
    bd = to_dev(to_layout_np(b, lq.LAYOUT2), lq.F64)
    for mode in ("f64", "ir-f32", "ir-f16"):
        x, st, rc = lq.gmres_solve(Ud, bd, m0, layout=lq.LAYOUT2, eo=True, mode=mode, tol=1e-10)
        assert rc == lq.OK, mode
        xs = from_layout_np(from_dev(x, lq.F64), lq.LAYOUT2, 4)
        res = dirac.apply_dw(U, xs, m0) - b
        rel = np.linalg.norm(res.reshape(6, -1), axis=1) / np.linalg.norm(b.reshape(6, -1), axis=1)
        assert np.all(rel <= 1e-10), (mode, rel)
