"""The allocation-free Schur apply (dirac_apply_eo_noalloc) through the C-ABI:
two calls in a row, the second on a smaller problem, each equal to
dirac_apply_eo on the same inputs (the same kernels, so bit for bit) and to
the oracle within the FP64 / FP32 bar; sizes beyond the fixed scratch are
rejected."""
import ctypes

import numpy as np
import pytest

import lqcd_synth as syn
import paper_2601_05816_amd as lq
from oracle import evenodd, geometry

from helpers import from_dev, from_layout_np, rel_err_per_rhs, rounded, to_dev, to_layout_np

pytestmark = pytest.mark.gpu

TOL = {lq.F64: 1e-12, lq.F32: 1e-5}


def _abi_call(U, pe, out, dims, nrhs, m0, prec, dagger=False):
    lib = lq.load()
    return lib.dirac_apply_eo_noalloc(ctypes.byref(lq._lattice(dims)), U.data_ptr(), pe.data_ptr(), out.data_ptr(),
                                      nrhs, m0, lq.LAYOUT2, prec, lq.DAGGER if dagger else 0, lq._stream())


@pytest.mark.parametrize("prec", [lq.F64, lq.F32])
def test_noalloc_matches_dirac_apply_eo(gpu_lib, prec):
    import torch

    cases = [((8, 4, 6, 4), 12, -0.05, False), ((4, 4, 2, 4), 3, 0.2, True)]  # second call smaller
    for k, (dims, nrhs, m0, dagger) in enumerate(cases):
        U = rounded(syn.gauge_field(dims, "haar", config=60 + k), prec)
        psi = rounded(syn.spinor_block(dims, nrhs, config=60 + k), prec)
        pe = geometry.to_half(psi, dims, 0)
        Ud = to_dev(U, prec)
        ped = to_dev(to_layout_np(pe, lq.LAYOUT2), prec)
        out = torch.full_like(ped, float("nan"))
        rc = _abi_call(Ud, ped, out, dims, nrhs, m0, prec, dagger)
        assert rc == lq.OK, lq.load().lqcd_last_error()
        torch.cuda.synchronize()
        ref = lq.dirac_apply_eo(Ud, ped, m0, layout=lq.LAYOUT2, dagger=dagger)
        torch.cuda.synchronize()
        assert torch.equal(out, ref)
        if not dagger:
            got = from_layout_np(from_dev(out, prec), lq.LAYOUT2, 1)
            assert np.all(rel_err_per_rhs(got, evenodd.apply_schur(U, pe, m0)) <= TOL[prec])


def test_noalloc_rejects_blocks_beyond_scratch(gpu_lib):
    import torch

    dims = (64, 32, 32, 32)  # V/2 x 12 x 2 x 16 bytes = 402 MB > 256 MiB
    U = torch.empty(1, dtype=torch.complex128, device="cuda")
    rc = _abi_call(U, U, U, dims, 2, 0.1, lq.F64)
    assert rc == -6 and b"scratch" in lq.load().lqcd_last_error()
    assert lq.NOALLOC_SCRATCH_BYTES == 256 << 20
