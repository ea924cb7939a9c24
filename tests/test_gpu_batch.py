"""Uneven multi-lattice batches in one persistent launch, against the oracle
and against one dirac_apply per lattice."""
import numpy as np
import pytest

import lqcd_synth as syn
import paper_2601_05816_amd as lq
from oracle import dirac

from helpers import rel_err_per_rhs, rounded, to_dev

pytestmark = pytest.mark.gpu
TOL = {lq.F64: 1e-12, lq.F32: 1e-5, lq.F16: 1e-3}


def _l2(block):
    return np.ascontiguousarray(np.moveaxis(block, 0, -1))


@pytest.mark.parametrize("prec", [lq.F64, lq.F32, lq.F16])
@pytest.mark.parametrize("grid", [0, 1, 7])
@pytest.mark.parametrize("kind", [1, 2])
@pytest.mark.parametrize("dagger", [False, True])
def test_uneven_batch_small(gpu_lib, prec, grid, kind, dagger):
    """Small lattices of different shapes and rhs counts (odd and even, so the
    pencil kernel mixes one and two rhs per work item); neither the kernel nor
    the persistent grid size (including a single workgroup, or the eight the
    pencil kernel rounds up to) changes the result."""
    gpu_lib.set_batch_kernel(kind)
    gpu_lib.set_batch_grid(grid)
    cases = [((4, 4, 4, 4), 1, 0.1), ((8, 4, 4, 4), 5, -0.05), ((4, 6, 2, 8), 3, 0.3), ((2, 2, 2, 2), 2, 0.0),
             ((6, 4, 4, 2), 7, -0.2)]
    probs, wants = [], []
    for k, (dims, n, m0) in enumerate(cases):
        U = rounded(syn.gauge_field(dims, "near_identity", config=50 + k, eps=0.2 + 0.3 * k / 7), prec)
        psi = rounded(syn.spinor_block(dims, n, config=50 + k), prec)
        probs.append((to_dev(U, prec), to_dev(_l2(psi), prec), m0))
        wants.append((dirac.apply_dw_dagger if dagger else dirac.apply_dw)(U, psi, m0))
    outs = lq.dirac_apply_batch(probs, dagger=dagger)
    gpu_lib.set_batch_grid(0)
    gpu_lib.set_batch_kernel(0)
    from helpers import from_dev
    for out, want in zip(outs, wants):
        got = np.moveaxis(from_dev(out, prec), -1, 0)
        assert np.all(rel_err_per_rhs(got, want) <= TOL[prec])


def test_batch_composition_matches_single_applies(gpu_lib):
    """The eight-lattice composition (L = 8..24, T = 2L, 1..32 rhs), FP32:
    one persistent launch equals eight separate applies bit for bit."""
    import torch

    comp = syn.batch_composition()
    probs = []
    gen = torch.Generator(device="cuda").manual_seed(4)
    for c in comp:
        dims = c["dims"]
        U = torch.randn((4,) + dims + (3, 3), dtype=torch.complex64, device="cuda", generator=gen)
        psi = torch.randn(dims + (4, 3, c["nrhs"]), dtype=torch.complex64, device="cuda", generator=gen)
        probs.append((U, psi, -0.05))
    gpu_lib.set_kernel_variant(1)
    singles = [lq.dirac_apply(U, psi, m0) for U, psi, m0 in probs]
    gpu_lib.set_kernel_variant(0)
    gpu_lib.set_batch_kernel(1)
    outs = lq.dirac_apply_batch(probs)
    for a, b in zip(outs, singles):
        assert torch.equal(a, b)
    # the pencil kernel sums the same terms in the pencil order
    gpu_lib.set_batch_kernel(2)
    outs = lq.dirac_apply_batch(probs)
    gpu_lib.set_batch_kernel(0)
    for a, b in zip(outs, singles):
        d = torch.linalg.vector_norm((a - b).reshape(-1, a.shape[-1]), dim=0)
        assert torch.all(d <= 1e-6 * torch.linalg.vector_norm(b.reshape(-1, b.shape[-1]), dim=0))


@pytest.mark.parametrize("prec", [lq.F32, lq.F16])
@pytest.mark.parametrize("cfg", [(2, 0, 0, 0, 0, 0), (2, 2, 2, 2, 1, 1)])
@pytest.mark.parametrize("grid", [0, 8])
def test_batch_links_through_lds(gpu_lib, prec, cfg, grid):
    """Lattices whose kernel configuration is variant 2 (the links of each
    step staged in LDS) run that body inside the persistent pencil launch
    when they have 8 or more rhs (LDS slices for 5 or 9 columns per
    wavefront), the others the plain pencil body: every lattice against the
    oracle, and those with 8 or more rhs bit for bit equal to their own
    variant-2 launch."""
    import torch

    from helpers import from_dev

    gpu_lib.set_kernel_config(*cfg)
    gpu_lib.set_batch_kernel(2)
    gpu_lib.set_batch_grid(grid)
    cases = [((4, 4, 4, 4), 8, 0.1), ((8, 4, 4, 4), 12, -0.05), ((4, 4, 2, 8), 16, 0.3), ((2, 2, 2, 2), 5, 0.0),
             ((6, 4, 4, 2), 20, -0.2)]
    try:
        probs, wants = [], []
        for k, (dims, n, m0) in enumerate(cases):
            U = rounded(syn.gauge_field(dims, "near_identity", config=90 + k, eps=0.3), prec)
            psi = rounded(syn.spinor_block(dims, n, config=90 + k), prec)
            probs.append((to_dev(U, prec), to_dev(_l2(psi), prec), m0))
            wants.append(dirac.apply_dw(U, psi, m0))
        outs = lq.dirac_apply_batch(probs)
        singles = [lq.dirac_apply(U, psi, m0) for U, psi, m0 in probs]
        torch.cuda.synchronize()
    finally:
        gpu_lib.set_batch_grid(0)
        gpu_lib.set_batch_kernel(0)
        gpu_lib.set_kernel_config(0)
    for out, single, want, (dims, n, m0) in zip(outs, singles, wants, cases):
        if n >= 8:  # the same body as the lattice's own launch
            assert torch.equal(out, single), (dims, n)
        got = np.moveaxis(from_dev(out, prec), -1, 0)
        assert np.all(rel_err_per_rhs(got, want) <= TOL[prec])


@pytest.mark.parametrize("kind", [1, 2])
def test_batch_composition_matches_oracle(gpu_lib, kind):
    """The eight-lattice composition (L = 8..24, T = 2L, 1..32 rhs, FP32) in
    one persistent launch against the oracle: at sampled sites of every
    lattice, D_W evaluated by the oracle on the 3^4 neighbourhood gathered
    around the site (D_W reads only nearest neighbours) from the FP32 values
    the GPU read."""
    import torch

    from helpers import neighbourhood

    comp = syn.batch_composition()
    probs = []
    gen = torch.Generator(device="cuda").manual_seed(41)
    for c in comp:
        dims = c["dims"]
        U = torch.randn((4,) + dims + (3, 3), dtype=torch.complex64, device="cuda", generator=gen)
        psi = torch.randn(dims + (4, 3, c["nrhs"]), dtype=torch.complex64, device="cuda", generator=gen)
        probs.append((U, psi, -0.05))
    gpu_lib.set_batch_kernel(kind)
    outs = lq.dirac_apply_batch(probs)
    gpu_lib.set_batch_kernel(0)
    torch.cuda.synchronize()
    rng = np.random.default_rng(42)
    for (U, psi, m0), out, c in zip(probs, outs, comp):
        dims, n = c["dims"], c["nrhs"]
        v = int(np.prod(dims))
        Uf, pf, of = U.reshape(4, v, 3, 3), psi.reshape(v, 4, 3, n), out.reshape(v, 4, 3, n)
        for s in rng.integers(0, v, 4):
            coord = np.unravel_index(int(s), dims)
            nb = torch.from_numpy(neighbourhood(coord, dims)).to("cuda")
            Ub = Uf[:, nb].cpu().numpy().astype(np.complex128).reshape((4,) + (3,) * 4 + (3, 3))
            pb = np.moveaxis(pf[nb].cpu().numpy().astype(np.complex128), -1, 0).reshape((n,) + (3,) * 4 + (4, 3))
            want = dirac.apply_dw_sites(Ub, pb, m0, [40])
            got = np.moveaxis(of[int(s)].cpu().numpy().astype(np.complex128), -1, 0)[:, None]
            assert np.all(rel_err_per_rhs(got, want) <= TOL[lq.F32]), (dims, int(s))


@pytest.mark.parametrize("mode", ["f64", "ir-f32"])
@pytest.mark.parametrize("graph", [False, True])
@pytest.mark.parametrize("kind", [1, 2])
def test_batched_solve_uneven(gpu_lib, mode, graph, kind):
    """Four lattices of different shapes, masses and rhs counts solved in one
    lock-step GMRES (persistent batched applies); every solution passes the
    oracle's residual check."""
    import torch

    cases = [((4, 4, 4, 4), 1, 0.1), ((8, 4, 4, 4), 5, -0.05), ((4, 6, 2, 8), 3, 0.3), ((6, 4, 4, 2), 7, 0.05)]
    probs, host = [], []
    for k, (dims, n, m0) in enumerate(cases):
        U = syn.gauge_field(dims, "near_identity", config=60 + k, eps=0.2 + 0.3 * k / 7)
        b = syn.spinor_block(dims, n, config=60 + k)
        probs.append((torch.from_numpy(U).to("cuda"), torch.from_numpy(_l2(b)).to("cuda"), m0))
        host.append((U, b, m0))
    gpu_lib.set_batch_kernel(kind)
    try:
        xs, stats, rc = lq.gmres_solve_batch(probs, restart=12, eo=True, mode=mode, tol=1e-10, use_graph=graph)
    finally:
        gpu_lib.set_batch_kernel(0)
    assert rc == lq.OK
    for x, st, (U, b, m0) in zip(xs, stats, host):
        xh = np.moveaxis(x.cpu().numpy(), -1, 0)
        assert np.all(rel_err_per_rhs(dirac.apply_dw(U, xh, m0), b) <= 1e-10)
        assert np.all(st["converged"] == 1)


def test_graph_replays_match_eager(gpu_lib):
    """The captured Arnoldi steps, replayed over many cycles, give bit for bit
    the result of launching the same kernels one by one."""
    import torch

    dims = (8, 4, 4, 8)
    U = torch.from_numpy(syn.gauge_field(dims, "near_identity", config=70)).to("cuda")
    b = torch.from_numpy(_l2(syn.spinor_block(dims, 6, config=70))).to("cuda")
    outs = []
    for graph in (False, True, True):
        x, st, rc = lq.gmres_solve(U, b, -0.05, restart=8, eo=True, tol=1e-11, use_graph=graph)
        assert rc == lq.OK and st["restarts"].max() > 3
        outs.append((x.clone(), st["iters"].copy()))
    assert torch.equal(outs[0][0], outs[1][0]) and torch.equal(outs[0][0], outs[2][0])
    assert np.array_equal(outs[0][1], outs[1][1])


def test_batched_solve_fp16_needs_one_volume(gpu_lib):
    """FP16 refinement of a batch needs lattices of one volume (documented
    argument error, raised before any launch)."""
    import torch

    probs = []
    for k, dims in enumerate([(4, 4, 4, 4), (8, 4, 4, 4)]):
        U = torch.from_numpy(syn.gauge_field(dims, "near_identity", config=80 + k)).to("cuda")
        b = torch.from_numpy(_l2(syn.spinor_block(dims, 2, config=80 + k))).to("cuda")
        probs.append((U, b, 0.1))
    with pytest.raises(lq.LqcdError, match="one volume"):
        lq.gmres_solve_batch(probs, restart=8, eo=True, mode="ir-f16")
    # equal volumes (different shapes) are accepted
    probs2 = []
    for k, dims in enumerate([(8, 4, 4, 4), (4, 8, 4, 4)]):
        U = syn.gauge_field(dims, "near_identity", config=82 + k)
        b = syn.spinor_block(dims, 2, config=82 + k)
        probs2.append((torch.from_numpy(U).to("cuda"), torch.from_numpy(_l2(b)).to("cuda"), 0.1, U, b))
    xs, stats, rc = lq.gmres_solve_batch([p[:3] for p in probs2], restart=8, eo=True, mode="ir-f16", tol=1e-10)
    assert rc == lq.OK
    for x, (_, _, m0, U, b) in zip(xs, probs2):
        xh = np.moveaxis(x.cpu().numpy(), -1, 0)
        assert np.all(rel_err_per_rhs(dirac.apply_dw(U, xh, m0), b) <= 1e-10)
