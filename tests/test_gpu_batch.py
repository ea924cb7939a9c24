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
def test_uneven_batch_small(gpu_lib, prec, grid):
    """Small lattices of different shapes and rhs counts; the persistent grid
    size (including a single workgroup) does not change the result."""
    gpu_lib.set_batch_grid(grid)
    cases = [((4, 4, 4, 4), 1, 0.1), ((8, 4, 4, 4), 5, -0.05), ((4, 6, 2, 8), 3, 0.3), ((2, 2, 2, 2), 2, 0.0),
             ((6, 4, 4, 2), 7, -0.2)]
    probs, wants = [], []
    for k, (dims, n, m0) in enumerate(cases):
        U = rounded(syn.gauge_field(dims, "near_identity", config=50 + k, eps=0.2 + 0.3 * k / 7), prec)
        psi = rounded(syn.spinor_block(dims, n, config=50 + k), prec)
        probs.append((to_dev(U, prec), to_dev(_l2(psi), prec), m0))
        wants.append(dirac.apply_dw(U, psi, m0))
    outs = lq.dirac_apply_batch(probs)
    gpu_lib.set_batch_grid(0)
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
    outs = lq.dirac_apply_batch(probs)
    for a, b in zip(outs, singles):
        assert torch.equal(a, b)
