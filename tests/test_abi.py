"""The C-ABI library on the CPU: it loads, exports every function that
include/lqcd.h declares, computes the geometry tables bit-exactly, and rejects
invalid arguments before touching the device."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2601_05816_amd as lq
from oracle import geometry

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "lqcd.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", text, flags=re.M)
    return sorted(set(n for n in names if n not in ("if", "for", "while")))


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("dirac_apply", "dirac_apply_eo", "gmres_solve", "gmres_workspace_bytes", "lqcd_lattice_tables",
              "lqcd_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = lq.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, f"symbols declared in lqcd.h but not exported: {missing}"


@pytest.mark.parametrize("dims", [(2, 2, 2, 2), (4, 4, 4, 4), (8, 4, 6, 2), (4, 6, 2, 8)])
def test_lattice_tables_bit_exact(dims):
    nbr, eo = lq.lattice_tables(dims)
    assert np.array_equal(nbr, geometry.neighbour_table(dims))
    assert np.array_equal(eo, geometry.eo_sites(dims))


def test_invalid_arguments_rejected_on_host():
    lib = lq.load()
    bad = lq._lattice((4, 4, 4, 3))
    rc = lib.dirac_apply(ctypes.byref(bad), 1, 1, 1, 1, 0.1, lq.LAYOUT2, lq.F64, 0, None)
    assert rc == -2 and b"even" in lib.lqcd_last_error()
    good = lq._lattice((4, 4, 4, 4))
    assert lib.dirac_apply(ctypes.byref(good), 1, 1, 1, 0, 0.1, lq.LAYOUT2, lq.F64, 0, None) == -1
    assert lib.dirac_apply(ctypes.byref(good), 1, 1, 1, 2, 0.1, 7, lq.F64, 0, None) == -3
    assert lib.dirac_apply(ctypes.byref(good), 1, 1, 1, 2, 0.1, lq.LAYOUT2, 5, 0, None) == -4
    assert lib.dirac_apply(ctypes.byref(good), None, 1, 1, 2, 0.1, lq.LAYOUT2, lq.F64, 0, None) == -1
    assert lib.dirac_apply_eo(ctypes.byref(good), 1, 1, 1, 2, -4.0, lq.LAYOUT2, lq.F64, 0, None) == -7
    nbr = np.empty((1, 8), dtype=np.int32)
    assert lib.lqcd_lattice_tables(ctypes.byref(bad), nbr.ctypes.data, None) == -2


def test_tune_table_roundtrip(tmp_path):
    """The autotuner's table is plain text; loading skips malformed lines."""
    lib = lq.load()
    lq.tune_clear()
    p = tmp_path / "tune.txt"
    p.write_text("# header\n0 64 32 32 32 16 0 2 : 2 4 4 1 1 4.8\nnot a line\n1 8 8 8 8 4 1 2 : 9 0 0 0 0 1.0\n"
                 "1 64 32 32 32 16 0 2 : 3 4 4 1 1 2 2.5\n1 8 8 8 8 4 1 2 : 2 0 0 0 0 11 1.0\n")
    assert lq.tune_load(p) == 2
    q = tmp_path / "out.txt"
    lq.tune_save(q)
    lines = [l for l in q.read_text().splitlines() if not l.startswith("#")]
    assert lines == ["0 64 32 32 32 16 0 2 : 2 4 4 1 1 0 4.800000", "1 64 32 32 32 16 0 2 : 3 4 4 1 1 2 2.500000"]
    lq.tune_clear()
    lq.set_kernel_config(0)
    with pytest.raises(lq.LqcdError):
        lq.set_kernel_config(9)
    with pytest.raises(lq.LqcdError):
        lq.set_kernel_config(2, wg_per_cu=9)
    with pytest.raises(lq.LqcdError):
        lq.set_batch_kernel(3)
    lq.set_batch_kernel(0)
    with pytest.raises(lq.LqcdError):
        lq.set_batch_grid(-1)


def test_block_gmres_rejects_bad_arguments_on_host():
    """Argument checks of the block solver run before any device work."""
    lib = lq.load()
    good = lq._lattice((4, 4, 4, 4))
    p = lq.solver_params()
    assert lib.block_gmres_workspace_bytes(ctypes.byref(good), 16, ctypes.byref(p)) > 0
    assert lib.block_gmres_workspace_bytes(ctypes.byref(good), 17, ctypes.byref(p)) == 0
    p1 = lq.solver_params(mode="ir-f32")
    assert lib.block_gmres_workspace_bytes(ctypes.byref(good), 4, ctypes.byref(p1)) == 0
    assert lib.block_gmres_solve(ctypes.byref(good), 1, 1, 1, 17, 0.1, lq.LAYOUT2, ctypes.byref(p), 1, 1 << 40,
                                 None, None) == -1
    assert lib.block_gmres_solve(ctypes.byref(good), 1, 1, 1, 4, 0.1, lq.LAYOUT2, ctypes.byref(p1), 1, 1 << 40,
                                 None, None) == -1
    pg = lq.solver_params(use_graph=True)
    assert lib.block_gmres_solve(ctypes.byref(good), 1, 1, 1, 4, 0.1, lq.LAYOUT2, ctypes.byref(pg), 1, 1 << 40,
                                 None, None) == -1
    assert lib.block_gmres_solve(ctypes.byref(good), None, 1, 1, 4, 0.1, lq.LAYOUT2, ctypes.byref(p), 1, 1 << 40,
                                 None, None) == -1
    assert lib.block_gmres_solve(ctypes.byref(good), 1, 1, 1, 4, 0.1, lq.LAYOUT2, ctypes.byref(p), 1, 16,
                                 None, None) == -6


def test_shipped_tune_table_loads_completely():
    """Every entry of the MI355X tune table the benchmark loads is accepted
    by the parser (a malformed line would be skipped silently and its
    problem would fall back to the default kernel)."""
    import os

    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2601_05816_amd",
                        "tune_mi355x.txt")
    entries = [l for l in open(path).read().splitlines() if l.strip() and not l.startswith("#")]
    lq.load()
    lq.tune_clear()
    try:
        assert lq.tune_load(path) == len(entries)
        for l in entries:
            cfg = l.split(":")[1].split()
            assert 1 <= int(cfg[0]) <= 7 and 0 <= int(cfg[5]) <= 8 and float(cfg[6]) > 0
    finally:
        lq.tune_clear()


def test_rhs_block_choice_on_host(tmp_path):
    """Chunk width of a solve (host logic, no device): the caller's width;
    else the full width if the workspace holds it, else the width with the
    least tuned time per rhs among those the workspace holds (the MI355X
    table for 32^3 x 64), or without table entries the largest; a workspace
    that holds no chunk is an error."""
    import ctypes

    lib = lq.load()
    dims = (64, 32, 32, 32)
    lat = lq._lattice(dims)
    p = lq.solver_params(eo=True, mode="f64")
    full = lq.gmres_workspace_bytes(dims, 64, p)
    ws = {w: lq.gmres_workspace_bytes(dims, 64, lq.solver_params(eo=True, mode="f64", rhs_block=w))
          for w in (1, 8, 16, 32)}
    assert ws[1] < ws[8] < ws[16] < ws[32] < full
    lq.tune_clear()
    assert lq.gmres_rhs_block(dims, 64, p, full) == 64
    assert lq.gmres_rhs_block(dims, 64, p, ws[16]) == 16
    assert lq.gmres_rhs_block(dims, 64, lq.solver_params(eo=True, rhs_block=8), full) == 8
    assert lib.gmres_rhs_block(ctypes.byref(lat), 64, ctypes.byref(p), ctypes.c_size_t(ws[1] - 1024)) == -6
    tune = os.path.join(os.path.dirname(HEADER), "..", "paper_2601_05816_amd", "tune_mi355x.txt")
    assert lq.tune_load(tune) > 0
    try:
        # the width with the least table time per rhs among those the
        # workspace holds (FP64 odd-even hop pass entries of the table)
        times = {}
        for line in open(tune):
            if line.startswith("#") or ":" not in line:
                continue
            k, v = line.split(":")
            k = [int(f) for f in k.split()]
            if k[0] == 1 and tuple(k[1:5]) == dims and k[6] == lq.F64 and k[7] == lq.LAYOUT2:
                times[k[5]] = float(v.split()[-1])
        cand = [w for w in (48, 32, 24, 16, 12, 8, 4, 2, 1) if w in times and ws.get(w, 0) <= ws[32]]
        want = min(cand, key=lambda w: (times[w] * ((64 + w - 1) // w), -w))
        assert lq.gmres_rhs_block(dims, 64, p, ws[32]) == want
    finally:
        lq.tune_clear()
    # a smaller chunk shrinks the workspace in proportion to its rhs
    assert abs(ws[32] / ws[16] - 2.0) < 0.01
