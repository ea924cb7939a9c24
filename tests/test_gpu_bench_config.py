"""Parity at the benchmark's lattice (32^3 x 64) in the benchmark's launch
configuration: the MI355X tune table that bench.py loads picks the kernel,
tile, t segments, store kind and residency of every apply here.  Inputs are
drawn on the GPU; sampled outputs are checked against the oracle evaluated
on a neighbourhood gathered around each sampled site.  D_W at a site reads
only its nearest neighbours (a 3^4 block suffices); the Schur complement
reaches two hops (a 6^4 block with the site at offset (2, 2, 2, 2), even
extents as the odd-even oracle needs, and the block's parity equal to the
lattice's because the centre is an even site), so the centre of the
gathered block is exact."""
import os

import numpy as np
import pytest

import paper_2601_05816_amd as lq
from oracle import dirac, evenodd, geometry

from helpers import neighbourhood, rel_err_per_rhs

pytestmark = pytest.mark.gpu

DIMS = (64, 32, 32, 32)
V = int(np.prod(DIMS))
M0 = -0.05
TUNE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2601_05816_amd",
                    "tune_mi355x.txt")
TOL = {lq.F64: 1e-12, lq.F32: 1e-5, lq.F16: 1e-3}
NSAMPLE = 8


@pytest.fixture(scope="module")
def tuned(gpu_lib):
    n = gpu_lib.tune_load(TUNE)
    assert n > 0
    gpu_lib.set_kernel_config(0)  # automatic selection: the table's entries
    yield gpu_lib
    gpu_lib.tune_clear()


def _draw(shape, prec, gen):
    """Gaussian complex field on the GPU in the storage of prec."""
    import torch

    if prec == lq.F64:
        return torch.randn(shape, dtype=torch.complex128, device="cuda", generator=gen)
    z = torch.randn(shape, dtype=torch.complex64, device="cuda", generator=gen)
    if prec == lq.F32:
        return z
    return torch.view_as_real(z).to(torch.float16).contiguous()


def _host(t, prec):
    """Device values (any storage) as complex128 on the host."""
    a = t.cpu().numpy()
    if prec == lq.F16:
        a = a.astype(np.float64)
        return a[..., 0] + 1j * a[..., 1]
    return a.astype(np.complex128)


def _sites_of_parity(rng, p, n):
    out = []
    while len(out) < n:
        s = int(rng.integers(0, V))
        if sum(np.unravel_index(s, DIMS)) % 2 == p:
            out.append(s)
    return out


@pytest.mark.parametrize("prec,nrhs", [(lq.F64, 1), (lq.F64, 4), (lq.F64, 16), (lq.F64, 64), (lq.F32, 16),
                                       (lq.F16, 16)])
def test_full_apply_benchmark_config(tuned, prec, nrhs):
    import torch

    g = torch.Generator(device="cuda").manual_seed(100 + 10 * prec + nrhs)
    U = _draw((4,) + DIMS + (3, 3), prec, g)
    psi = _draw(DIMS + (4, 3, nrhs), prec, g)
    out = lq.dirac_apply(U, psi, M0, layout=lq.LAYOUT2)
    torch.cuda.synchronize()
    tail = (2,) if prec == lq.F16 else ()
    Uf = U.reshape((4, V, 3, 3) + tail)
    pf = psi.reshape((V, 4, 3, nrhs) + tail)
    of = out.reshape((V, 4, 3, nrhs) + tail)
    rng = np.random.default_rng(200 + nrhs)
    for s in rng.integers(0, V, NSAMPLE):
        coord = np.unravel_index(int(s), DIMS)
        nb = torch.from_numpy(neighbourhood(coord, DIMS)).to("cuda")
        Ub = _host(Uf[:, nb], prec).reshape((4,) + (3,) * 4 + (3, 3))
        pb = np.moveaxis(_host(pf[nb], prec), -1, 0).reshape((nrhs,) + (3,) * 4 + (4, 3))
        want = dirac.apply_dw_sites(Ub, pb, M0, [40])  # centre (1, 1, 1, 1) of the 3^4 block
        got = np.moveaxis(_host(of[int(s)], prec), -1, 0)[:, None]
        assert np.all(rel_err_per_rhs(got, want) <= TOL[prec]), (int(s), coord)
    del U, psi, out
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", [lq.F64, lq.F32, lq.F16])
def test_schur_apply_benchmark_config(tuned, prec):
    """Schur apply at 16 rhs in the tuned configuration (FP16: the kernel the
    timed FP16-storage refinement solve runs), FP16 against the oracle on the
    FP16 values the GPU reads."""
    import torch

    nrhs = 16
    g = torch.Generator(device="cuda").manual_seed(300 + prec)
    U = _draw((4,) + DIMS + (3, 3), prec, g)
    psi_e = _draw((V // 2, 4, 3, nrhs), prec, g)
    out = lq.dirac_apply_eo(U, psi_e, M0, layout=lq.LAYOUT2)
    torch.cuda.synchronize()
    bd = (6, 6, 6, 6)
    centre = int(geometry.site_index(np.array([2, 2, 2, 2]), bd))
    rng = np.random.default_rng(400 + prec)
    Uf = U.reshape((4, V, 3, 3) + ((2,) if prec == lq.F16 else ()))
    for s in _sites_of_parity(rng, 0, NSAMPLE):
        coord = np.unravel_index(s, DIMS)
        nb = neighbourhood(coord, DIMS, -2, 3)
        even = np.asarray(np.unravel_index(nb, DIMS)).sum(axis=0) % 2 == 0
        Ub = _host(Uf[:, torch.from_numpy(nb).to("cuda")], prec).reshape((4,) + bd + (3, 3))
        pb = np.zeros((nrhs, nb.size, 4, 3), dtype=np.complex128)
        he = torch.from_numpy(nb[even] >> 1).to("cuda")  # compact index of an even site
        pb[:, even] = np.moveaxis(_host(psi_e[he], prec), -1, 0)
        pe = geometry.to_half(pb.reshape((nrhs,) + bd + (4, 3)), bd, 0)
        want = evenodd.apply_schur(Ub, pe, M0)[:, centre >> 1][:, None]
        got = np.moveaxis(_host(out[s >> 1], prec), -1, 0)[:, None]
        assert np.all(rel_err_per_rhs(got, want) <= TOL[prec]), (s, coord)
    del U, psi_e, out
    torch.cuda.empty_cache()


@pytest.fixture(scope="module")
def bench_system(tuned):
    """The benchmark's solver inputs: near-identity links (eps = 0.3, config 3)
    and 16 Gaussian sources on 32^3 x 64, resident on the GPU."""
    import torch

    import lqcd_synth as syn

    U = torch.from_numpy(syn.gauge_field(DIMS, "near_identity", config=3, eps=0.3)).to("cuda")
    b = torch.from_numpy(np.ascontiguousarray(np.moveaxis(syn.spinor_block(DIMS, 16, config=3), 0, -1))).to("cuda")
    yield U, b
    del U, b
    torch.cuda.empty_cache()


@pytest.mark.parametrize("mode", ["f64", "ir-f32", "ir-f16"])
def test_gmres_benchmark_config(bench_system, mode):
    """Odd-even GMRES(30) to a true relative residual of 1e-10, as timed by
    the benchmark; the oracle's D_W at sampled sites of x reproduces b there
    to within the global residual bound 1e-10 ||b|| (per rhs)."""
    import torch

    U, b = bench_system
    nrhs = b.shape[-1]
    x, st, rc = lq.gmres_solve(U, b, M0, layout=lq.LAYOUT2, restart=30, eo=True, mode=mode, tol=1e-10,
                               max_restarts=400, max_outer=60)
    assert rc == lq.OK and st["converged"].all() and np.all(st["true_relres"] <= 1e-10)
    bnorm = torch.linalg.vector_norm(b.reshape(-1, nrhs), dim=0).cpu().numpy()
    Uf = U.reshape(4, V, 3, 3)
    xf = x.reshape(V, 4, 3, nrhs)
    bf = b.reshape(V, 4, 3, nrhs)
    rng = np.random.default_rng(500)
    for s in rng.integers(0, V, NSAMPLE):
        coord = np.unravel_index(int(s), DIMS)
        nb = torch.from_numpy(neighbourhood(coord, DIMS)).to("cuda")
        Ub = _host(Uf[:, nb], lq.F64).reshape((4,) + (3,) * 4 + (3, 3))
        xb = np.moveaxis(_host(xf[nb], lq.F64), -1, 0).reshape((nrhs,) + (3,) * 4 + (4, 3))
        Dx = dirac.apply_dw_sites(Ub, xb, M0, [40])[:, 0]
        bs = np.moveaxis(_host(bf[int(s)], lq.F64), -1, 0)
        r = np.linalg.norm((Dx - bs).reshape(nrhs, -1), axis=1)
        assert np.all(r <= 1e-10 * bnorm * (1 + 1e-6)), (int(s), r / bnorm)
    del x
    torch.cuda.empty_cache()
