"""Pins for the oracle's geometry (Sec. III-A.1 site numbering): hand-worked
sites, brute-force loops, and the structural invariants."""
import itertools
import os

import numpy as np
import pytest

from oracle import geometry as geo

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "geometry_4x4x4x4.txt")


def _golden_rows():
    rows = []
    with open(GOLDEN) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            c, i, n, p = line.split("|")
            rows.append(([int(t) for t in c.split()], int(i), [int(t) for t in n.split()], int(p)))
    return rows


def test_hand_worked_sites():
    dims = (4, 4, 4, 4)
    nbr = geo.neighbour_table(dims)
    par = geo.parity(dims)
    for c, idx, n, p in _golden_rows():
        assert int(geo.site_index(c, dims)) == idx
        assert list(nbr[idx]) == n
        assert par[idx] == p


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4), (8, 4, 4, 4), (6, 2, 4, 2)])
def test_brute_force_loops(dims):
    """Neighbours and parity from plain nested loops over coordinates."""
    n0, n1, n2, n3 = dims
    nbr = geo.neighbour_table(dims)
    par = geo.parity(dims)
    idx = 0
    for x0, x1, x2, x3 in itertools.product(range(n0), range(n1), range(n2), range(n3)):
        x = [x0, x1, x2, x3]
        for mu in range(4):
            up = list(x)
            up[mu] = (up[mu] + 1) % dims[mu]
            dn = list(x)
            dn[mu] = (dn[mu] - 1) % dims[mu]
            # numbering written out as a sum of coordinate times stride
            s_up = up[0] * n1 * n2 * n3 + up[1] * n2 * n3 + up[2] * n3 + up[3]
            s_dn = dn[0] * n1 * n2 * n3 + dn[1] * n2 * n3 + dn[2] * n3 + dn[3]
            assert nbr[idx, mu] == s_up
            assert nbr[idx, 4 + mu] == s_dn
        assert par[idx] == (x0 + x1 + x2 + x3) % 2
        idx += 1


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4), (8, 4, 4, 4), (16, 8, 8, 8)])
def test_invariants(dims):
    v = int(np.prod(dims))
    nbr = geo.neighbour_table(dims)
    par = geo.parity(dims)
    ar = np.arange(v)
    for mu in range(4):
        assert np.array_equal(nbr[nbr[:, mu], 4 + mu], ar)      # (x+mu)-mu = x
        assert np.array_equal(nbr[nbr[:, 4 + mu], mu], ar)
        assert np.all(par[nbr[:, mu]] != par)                   # every link flips parity
    eo = geo.eo_sites(dims)
    assert eo.shape == (2, v // 2)
    for p in range(2):
        assert np.all(par[eo[p]] == p)
        # compact index of a site of either parity is its number halved
        assert np.array_equal(eo[p] >> 1, np.arange(v // 2))
    assert np.array_equal(np.sort(np.concatenate([eo[0], eo[1]])), ar)


def test_half_roundtrip():
    dims = (4, 2, 2, 4)
    rng = np.random.default_rng(0)
    a = rng.standard_normal((3,) + dims + (4, 3)) + 0j
    e = geo.to_half(a, dims, 0)
    o = geo.to_half(a, dims, 1)
    assert np.array_equal(geo.from_half(e, dims, 0) + geo.from_half(o, dims, 1), a)


def test_odd_extent_rejected():
    with pytest.raises(ValueError):
        geo.neighbour_table((4, 4, 4, 3))
