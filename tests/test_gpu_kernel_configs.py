"""GPU parity of the Wilson kernels in forced launch configurations: pencil
tiles and t segments, non-temporal stores, the autotuner's choice, the
LDS-fed FP64 kernel, residency caps, the two-rhs-per-lane FP32 / FP16
kernels and the row-broadcast-link kernels, each against the oracle
(tolerances as in test_gpu_apply.py)."""
import numpy as np
import pytest

import lqcd_synth as syn
import paper_2601_05816_amd as lq
from oracle import dirac, evenodd, geometry

from helpers import apply_eo_gpu as _apply_eo_gpu
from helpers import apply_gpu as _apply_gpu
from helpers import from_dev, from_layout_np, rel_err_per_rhs, rounded, to_dev, to_layout_np

pytestmark = pytest.mark.gpu

TOL = {lq.F64: 1e-12, lq.F32: 1e-5, lq.F16: 1e-3}
LAYOUTS = [lq.RHS_OUTER, lq.LAYOUT1, lq.LAYOUT2]


def _g5h(x):
    """gamma5 on a half-lattice block (nrhs, V/2, 4, 3)."""
    return dirac.apply_gamma5(x.reshape(x.shape[0], -1, 1, 1, 1, 4, 3)).reshape(x.shape)


@pytest.fixture(autouse=True)
def automatic_selection_after(gpu_lib):
    """Every test forces its own configuration; restore automatic selection."""
    yield
    gpu_lib.set_kernel_config(0)


@pytest.mark.parametrize("kernel_variant", [2, 3])
@pytest.mark.parametrize("pencil", [(1, 1, 1), (2, 1, 3), (1, 2, 6), (3, 2, 2), (0, 0, 12)])
def test_pencil_tilings(gpu_lib, kernel_variant, pencil):
    """Every tile shape and segment count gives the same result (the mapping
    of work items to columns, rhs and t segments is a bijection)."""
    gpu_lib.set_kernel_variant(kernel_variant, pencil)
    dims = (12, 4, 6, 4)
    U = syn.gauge_field(dims, "haar", config=9)
    psi = syn.spinor_block(dims, 5, config=9)
    for layout in LAYOUTS:
        got = _apply_gpu(U, psi, 0.2, layout, lq.F64)
        assert np.all(rel_err_per_rhs(got, dirac.apply_dw(U, psi, 0.2)) <= TOL[lq.F64])
        psi_e = geometry.to_half(psi, dims, 0)
        got = _apply_eo_gpu(U, psi_e, 0.2, layout, lq.F64)
        assert np.all(rel_err_per_rhs(got, evenodd.apply_schur(U, psi_e, 0.2)) <= TOL[lq.F64])


@pytest.mark.parametrize("kernel_variant", [2, 3])
@pytest.mark.parametrize("nt", [0, 1])
def test_nontemporal_stores_and_autotuned_choice(gpu_lib, kernel_variant, nt):
    """Non-temporal output stores, and whatever configuration the autotuner
    records, give the oracle's result."""
    import torch

    dims = (8, 4, 6, 4)
    U = syn.gauge_field(dims, "near_identity", config=10)
    psi = syn.spinor_block(dims, 16, config=10)
    want = dirac.apply_dw(U, psi, -0.05)
    gpu_lib.set_kernel_config(kernel_variant, 0, 0, 0, nt)
    got = _apply_gpu(U, psi, -0.05, lq.LAYOUT2, lq.F64)
    assert np.all(rel_err_per_rhs(got, want) <= TOL[lq.F64])
    psi_e = geometry.to_half(psi, dims, 0)
    got = _apply_eo_gpu(U, psi_e, -0.05, lq.LAYOUT2, lq.F64)
    assert np.all(rel_err_per_rhs(got, evenodd.apply_schur(U, psi_e, -0.05)) <= TOL[lq.F64])
    # automatic selection after tuning this exact problem
    gpu_lib.set_kernel_config(0)
    gpu_lib.tune_clear()
    Ud = to_dev(U, lq.F64)
    pd = to_dev(to_layout_np(psi, lq.LAYOUT2), lq.F64)
    best = gpu_lib.autotune(Ud, pd, torch.empty_like(pd), layout=lq.LAYOUT2, reps=1)
    assert best["variant"] in (1, 2, 3, 5, 6, 7) and best["ms"] > 0
    got = from_layout_np(from_dev(lq.dirac_apply(Ud, pd, -0.05, layout=lq.LAYOUT2), lq.F64), lq.LAYOUT2, 4)
    assert np.all(rel_err_per_rhs(got, want) <= TOL[lq.F64])
    # odd-even: the hop pass and the whole Schur apply (two passes or fused)
    pe = to_dev(to_layout_np(psi_e, lq.LAYOUT2), lq.F64)
    best = gpu_lib.autotune(Ud, pe, torch.empty_like(pe), layout=lq.LAYOUT2, eo=True, reps=1)
    assert best["variant"] in (1, 2, 3, 6) and best["ms"] > 0
    got = from_layout_np(from_dev(lq.dirac_apply_eo(Ud, pe, -0.05, layout=lq.LAYOUT2), lq.F64), lq.LAYOUT2, 1)
    assert np.all(rel_err_per_rhs(got, evenodd.apply_schur(U, psi_e, -0.05)) <= TOL[lq.F64])
    gpu_lib.tune_clear()


@pytest.mark.parametrize("nrhs", [10, 11, 12, 16, 24, 64])
@pytest.mark.parametrize("pencil", [(0, 0, 0), (2, 1, 3), (1, 2, 1), (3, 2, 2)])
def test_lds_fed_full_kernel(gpu_lib, nrhs, pencil):
    """Variant 5 (spinors and links arrive by global-to-LDS transfers, three
    hops in flight per wavefront): FP64, rhs-innermost, D and D^dagger, tiles
    and segment counts that leave wavefronts partly idle."""
    gpu_lib.set_kernel_config(5, pencil[0], pencil[1], pencil[2], 1)
    try:
        dims = (6, 4, 6, 4)
        U = syn.gauge_field(dims, "haar", config=13)
        psi = syn.spinor_block(dims, nrhs, config=13)
        for dagger in (False, True):
            want = (dirac.apply_dw_dagger if dagger else dirac.apply_dw)(U, psi, -0.3)
            got = _apply_gpu(U, psi, -0.3, lq.LAYOUT2, lq.F64, dagger)
            assert np.all(rel_err_per_rhs(got, want) <= TOL[lq.F64])
        # unsupported combinations fall back to the plain pencil kernel
        got = _apply_gpu(U, psi[:4], -0.3, lq.LAYOUT2, lq.F64)
        assert np.all(rel_err_per_rhs(got, dirac.apply_dw(U, psi[:4], -0.3)) <= TOL[lq.F64])
        got = _apply_gpu(U, psi, -0.3, lq.LAYOUT1, lq.F64)
        assert np.all(rel_err_per_rhs(got, dirac.apply_dw(U, psi, -0.3)) <= TOL[lq.F64])
    finally:
        gpu_lib.set_kernel_config(0)


@pytest.mark.parametrize("kernel_variant", [2, 3])
@pytest.mark.parametrize("occ", [1, 2, 4])
def test_residency_cap(gpu_lib, kernel_variant, occ):
    """Capping the workgroups per compute unit (through the LDS request) only
    changes which workgroups run together, never the result: full and Schur
    applies, FP64 and FP32 (variant 4 for FP32 in the variant-3 case)."""
    dims = (8, 4, 6, 4)
    U = syn.gauge_field(dims, "haar", config=12)
    psi = syn.spinor_block(dims, 16, config=12)
    for prec in (lq.F64, lq.F32):
        v = 4 if (kernel_variant == 3 and prec == lq.F32) else kernel_variant
        gpu_lib.set_kernel_config(v, 2, 2, 0, 1, occ)
        Up, pp = rounded(U, prec), rounded(psi, prec)
        got = _apply_gpu(Up, pp, 0.15, lq.LAYOUT2, prec)
        assert np.all(rel_err_per_rhs(got, dirac.apply_dw(Up, pp, 0.15)) <= TOL[prec])
        pe = geometry.to_half(pp, dims, 0)
        got = _apply_eo_gpu(Up, pe, 0.15, lq.LAYOUT2, prec)
        assert np.all(rel_err_per_rhs(got, evenodd.apply_schur(Up, pe, 0.15)) <= TOL[prec] * 2)
    gpu_lib.set_kernel_config(0)


@pytest.mark.parametrize("prec", [lq.F32, lq.F16])
@pytest.mark.parametrize("nrhs", [2, 6, 16])
@pytest.mark.parametrize("pencil", [(0, 0, 0), (2, 1, 3), (1, 2, 1)])
def test_two_rhs_per_lane_kernels(gpu_lib, prec, nrhs, pencil):
    """Variant 4 (two rhs per work item, vector loads) for FP32 and FP16, full
    and Schur applies, D and D^dagger, several tilings."""
    gpu_lib.set_kernel_variant(4, pencil)
    dims = (6, 4, 6, 4)
    U = rounded(syn.gauge_field(dims, "haar", config=11), prec)
    psi = rounded(syn.spinor_block(dims, nrhs, config=11), prec)
    for dagger in (False, True):
        want = (dirac.apply_dw_dagger if dagger else dirac.apply_dw)(U, psi, 0.1)
        got = _apply_gpu(U, psi, 0.1, lq.LAYOUT2, prec, dagger)
        assert np.all(rel_err_per_rhs(got, want) <= TOL[prec])
    psi_e = geometry.to_half(psi, dims, 0)
    got = _apply_eo_gpu(U, psi_e, 0.1, lq.LAYOUT2, prec)
    assert np.all(rel_err_per_rhs(got, evenodd.apply_schur(U, psi_e, 0.1)) <= TOL[prec] * 2)


@pytest.mark.parametrize("prec", [lq.F64, lq.F32, lq.F16])
@pytest.mark.parametrize("nrhs", [16, 32])
@pytest.mark.parametrize("pencil", [(0, 0, 0, 0), (2, 1, 3, 1), (1, 2, 1, 0), (3, 2, 2, 1)])
def test_row_broadcast_link_kernels(gpu_lib, prec, nrhs, pencil):
    """Variant 6 (each 16-lane row loads its column's links once and moves
    them to its lanes by row broadcasts): full apply D and D^dagger and the
    Schur apply in both rhs-fastest layouts, three precisions, tiles and
    segment counts; unsupported rhs counts fall back to variant 3."""
    gpu_lib.set_kernel_config(6, pencil[0], pencil[1], pencil[2], pencil[3])
    dims = (6, 4, 6, 4)
    U = rounded(syn.gauge_field(dims, "haar", config=14), prec)
    psi = rounded(syn.spinor_block(dims, nrhs, config=14), prec)
    psi_e = geometry.to_half(psi, dims, 0)
    for layout in (lq.LAYOUT1, lq.LAYOUT2):
        for dagger in (False, True):
            want = (dirac.apply_dw_dagger if dagger else dirac.apply_dw)(U, psi, -0.2)
            got = _apply_gpu(U, psi, -0.2, layout, prec, dagger)
            assert np.all(rel_err_per_rhs(got, want) <= TOL[prec])
            if dagger:  # S^dagger = gamma5 S gamma5
                want = _g5h(evenodd.apply_schur(U, _g5h(psi_e), -0.2))
            else:
                want = evenodd.apply_schur(U, psi_e, -0.2)
            got = _apply_eo_gpu(U, psi_e, -0.2, layout, prec, dagger)
            assert np.all(rel_err_per_rhs(got, want) <= TOL[prec] * 2)
    got = _apply_gpu(U, psi[:5], -0.2, lq.LAYOUT2, prec)
    assert np.all(rel_err_per_rhs(got, dirac.apply_dw(U, psi[:5], -0.2)) <= TOL[prec])


def test_row_broadcast_link_kernels_in_solves(gpu_lib):
    """The odd-even row-broadcast kernel inside GMRES (its lanes of converged
    rhs keep loading and broadcasting links and skip only their stores):
    FP64 and FP32 refinement reach the tolerance on every rhs."""
    gpu_lib.set_kernel_config(6, 0, 0, 0, 1)
    dims = (8, 4, 4, 4)
    m0 = -0.05
    U = syn.gauge_field(dims, "near_identity", config=15, eps=0.3)
    b = syn.spinor_block(dims, 16, config=15)
    b[3] *= 1e-3  # rhs with different iteration counts
    Ud = to_dev(U, lq.F64)
    bd = to_dev(to_layout_np(b, lq.LAYOUT2), lq.F64)
    for mode in ("f64", "ir-f32"):
        x, st, rc = lq.gmres_solve(Ud, bd, m0, layout=lq.LAYOUT2, eo=True, mode=mode, tol=1e-10)
        assert rc == lq.OK
        xs = from_layout_np(from_dev(x, lq.F64), lq.LAYOUT2, 4)
        res = dirac.apply_dw(U, xs, m0) - b
        rel = np.linalg.norm(res.reshape(16, -1), axis=1) / np.linalg.norm(b.reshape(16, -1), axis=1)
        assert np.all(rel <= 1e-10), (mode, rel)


@pytest.mark.parametrize("prec", [lq.F64, lq.F32, lq.F16])
@pytest.mark.parametrize("dims,nrhs", [((4, 4, 2, 16), 16), ((4, 2, 2, 16), 32), ((2, 2, 2, 16), 64),
                                       ((6, 4, 2, 4), 64)])
@pytest.mark.parametrize("pencil", [(0, 0, 0, 1), (1, 2, 2, 0), (2, 1, 4, 1)])
def test_x_neighbours_through_lds(gpu_lib, prec, dims, nrhs, pencil):
    """Variant 7 (row-broadcast links and the +-x neighbours of the inner
    columns of a workgroup read from LDS, 256 / nrhs consecutive columns per
    workgroup, end columns from memory; FP64 blocks of 32 and 64 rhs run in
    chunks of 16, 16 columns per workgroup): full apply D and D^dagger in
    both rhs-fastest layouts on lattices whose x extent holds whole
    workgroups; the odd-even apply (compact x rows of half the length) and
    the FP64 64-rhs apply on the last lattice (x = 4) fall back to
    variant 6."""
    gpu_lib.set_kernel_config(7, pencil[0], pencil[1], pencil[2], pencil[3])
    U = rounded(syn.gauge_field(dims, "haar", config=16), prec)
    psi = rounded(syn.spinor_block(dims, nrhs, config=16), prec)
    for layout in (lq.LAYOUT1, lq.LAYOUT2):
        for dagger in (False, True):
            want = (dirac.apply_dw_dagger if dagger else dirac.apply_dw)(U, psi, 0.3)
            got = _apply_gpu(U, psi, 0.3, layout, prec, dagger)
            assert np.all(rel_err_per_rhs(got, want) <= TOL[prec])
    psi_e = geometry.to_half(psi, dims, 0)
    got = _apply_eo_gpu(U, psi_e, 0.3, lq.LAYOUT2, prec)
    assert np.all(rel_err_per_rhs(got, evenodd.apply_schur(U, psi_e, 0.3)) <= TOL[prec] * 2)


@pytest.mark.parametrize("prec", [lq.F64, lq.F32, lq.F16])
@pytest.mark.parametrize("dims,nrhs", [((4, 2, 2, 32), 16), ((4, 2, 4, 16), 32), ((2, 2, 2, 8), 64)])
@pytest.mark.parametrize("pencil", [(0, 0, 0, 1), (1, 2, 2, 0), (2, 1, 1, 1)])
def test_x_neighbours_through_lds_odd_even(gpu_lib, prec, dims, nrhs, pencil):
    """Variant 7 in the odd-even hop passes (the workgroup's 256 / nrhs
    consecutive compact columns put their streamed +t spinor into LDS, the
    next step's x neighbours of the inner columns are read there): the
    Schur apply S and S^dagger in both rhs-fastest layouts against the
    oracle, on lattices whose compact x rows hold whole workgroups."""
    gpu_lib.set_kernel_config(7, pencil[0], pencil[1], pencil[2], pencil[3])
    U = rounded(syn.gauge_field(dims, "haar", config=17), prec)
    psi_e = geometry.to_half(rounded(syn.spinor_block(dims, nrhs, config=17), prec), dims, 0)
    for layout in (lq.LAYOUT1, lq.LAYOUT2):
        for dagger in (False, True):
            if dagger:  # S^dagger = gamma5 S gamma5
                want = _g5h(evenodd.apply_schur(U, _g5h(psi_e), -0.15))
            else:
                want = evenodd.apply_schur(U, psi_e, -0.15)
            got = _apply_eo_gpu(U, psi_e, -0.15, layout, prec, dagger)
            assert np.all(rel_err_per_rhs(got, want) <= TOL[prec] * 2), (layout, dagger)


def test_x_neighbours_through_lds_odd_even_in_solves(gpu_lib):
    """The odd-even variant 7 inside GMRES (converged rhs keep taking part in
    the loads, LDS exchange and barriers and skip their stores): all three
    modes reach a true 1e-10 on every rhs, checked with the oracle's D_W."""
    gpu_lib.set_kernel_config(7, 0, 0, 0, 1)
    dims = (8, 2, 2, 32)
    m0 = -0.05
    U = syn.gauge_field(dims, "near_identity", config=18, eps=0.3)
    b = syn.spinor_block(dims, 16, config=18)
    b[5] *= 1e-3  # rhs with different iteration counts
    Ud = to_dev(U, lq.F64)
    bd = to_dev(to_layout_np(b, lq.LAYOUT2), lq.F64)
    for mode in ("f64", "ir-f32", "ir-f16"):
        x, st, rc = lq.gmres_solve(Ud, bd, m0, layout=lq.LAYOUT2, eo=True, mode=mode, tol=1e-10)
        assert rc == lq.OK, mode
        xs = from_layout_np(from_dev(x, lq.F64), lq.LAYOUT2, 4)
        res = dirac.apply_dw(U, xs, m0) - b
        rel = np.linalg.norm(res.reshape(16, -1), axis=1) / np.linalg.norm(b.reshape(16, -1), axis=1)
        assert np.all(rel <= 1e-10), (mode, rel)
