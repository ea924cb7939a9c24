"""The HBM probe computes what it claims (copy and triad)."""
import pytest

import paper_2601_05816_amd as lq

pytestmark = pytest.mark.gpu


def test_probe_copy_and_triad(gpu_lib):
    import torch

    n = (1 << 20) + 6  # not a multiple of the unrolled stride: exercises the tail loop
    src = torch.arange(n, dtype=torch.float64, device="cuda")
    dst = torch.zeros(n, dtype=torch.float64, device="cuda")
    t = lq.hbm_probe(src, dst, kind="copy", reps=2)          # dst = src
    assert t > 0 and torch.equal(dst, src)
    a = torch.zeros(n, dtype=torch.float64, device="cuda")
    c = torch.full((n,), 2.0, dtype=torch.float64, device="cuda")
    t = lq.hbm_probe(a, src, c, kind="triad", reps=2)        # a = src + 3 c
    assert t > 0 and torch.equal(a, src + 6.0)
