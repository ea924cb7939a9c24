#!/usr/bin/env python3
"""Benchmark: multi-rhs Wilson-Dirac apply on one MI355X.

Timed step: one application of the full Wilson-Dirac operator D_W to a block
of nrhs = 16 FP64 spinor fields on a 32^3 x 64 lattice (near-identity SU(3)
links U = exp(i 0.3 H), m0 = -0.05, rhs-innermost layout), inputs resident in
HBM.  Reported value: nominal GFLOP/s (1392 flop per site and rhs).  The JSON
line also carries the roofline of the kernel (algorithmic HBM bytes
(36 + 24 nrhs) x 16 per site over the measured launch time), an nrhs sweep in
FP64/FP32/FP16 for the full and the Schur (odd-even) apply, the solvers
(FP64 GMRES against FP32 / FP16 refinement to a true residual of 1e-10, the
fixed 100-iteration protocol, block GMRES, the clover operator, the uneven
multi-lattice batch, differentiation, small lattices) and the oracle's CPU
throughput on a sample of the same apply (two of the 16 rhs).

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-sweep] [--no-cpu] [--no-counters]
    python bench.py --only {apply,sweep-f64,schur-f64,schur-sizes,clover-f64,gmres-fixed,block-fixed,block-hard,gmres-sweep,
                            gmres-ir}
                    [--prec f64|f32|f16] [--kind full|schur] [--nrhs N] [--calibrate]
                                    (one workload, for profilers)

The headline kernel's HBM traffic (roofline.traffic) is measured in the same
run: two child processes run `--only apply --calibrate` under
`rocprofv3 --pmc FETCH_SIZE` and `--pmc WRITE_SIZE` before this process
touches the GPU, and the counters are scaled by what they report for a plain
device copy of known size in the same child (`--no-counters` skips this).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

DIMS = (64, 32, 32, 32)
NRHS = 16
M0 = -0.05
EPS = 0.3
CONFIG = 3
FLOP_SITE_RHS = 1392          # 1320 projected hopping + 72 diagonal/combine
SCHUR_FLOP_SITE_RHS = 2712    # per even site: two hopping passes + axpy
HBM_PEAK_GBS = 8000.0
TUNE_FILE = os.path.join(ROOT, "paper_2601_05816_amd", "tune_mi355x.txt")
def bytes_full(v, nrhs, esz):
    """Algorithmic bytes of one full apply: every link, input and output element once."""
    return (36 + 24 * nrhs) * esz * v


def bytes_schur_two_pass(v, nrhs, esz):
    """Two hopping passes over half lattices.  Each pass reads every link once
    (8 links of 9 entries per output site = 72 per even site) and its input
    half spinor block and writes its output; the second also reads the axpy
    input: per even site 2 x 72 links + (12 + 12) + (12 + 12 + 12) nrhs."""
    return (2 * 72 + 60 * nrhs) * esz * (v // 2)


def table_entry(path, kind, dims, nrhs, prec, layout):
    """The autotuner table's configuration for (kind, dims, nrhs, prec, layout), or None."""
    want = [kind, *dims, nrhs, prec, layout]
    for line in open(path):
        if line.startswith("#") or ":" not in line:
            continue
        k, v = line.split(":", 1)
        try:
            if [int(a) for a in k.split()] != want:
                continue
            vals = v.split()
            c = [int(a) for a in vals[:-1]] + [0] * (6 - len(vals[:-1]))
            return {"variant": c[0], "tile_y": c[1], "tile_z": c[2], "segments": c[3], "nontemporal": c[4],
                    "wg_per_cu": c[5], "ms": float(vals[-1])}
        except ValueError:
            continue
    return None


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def timed(fn, steps, warmup):
    import torch

    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(steps):
        fn()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / steps  # ms per call


def tile_rhs(base, nrhs):
    """Block of nrhs rhs (LAYOUT2) built by repeating the generated rhs."""
    import torch

    reps = (nrhs + base.shape[-1] - 1) // base.shape[-1]
    return base.repeat(*([1] * (base.dim() - 1)), reps)[..., :nrhs].contiguous()


def to_f16(t):
    import torch

    return torch.view_as_real(t.to(torch.complex64)).to(torch.float16).contiguous()


def measure_traffic(steps=3):
    """HBM bytes per launch of the headline apply from rocprofv3 counters,
    each counter in a child process of its own (this process has not
    initialised the GPU yet).  Scale: true bytes of the probe's plain copy
    over what the counter reports for it.  Returns (traffic dict, None) or
    (None, reason)."""
    import csv
    import glob
    import shutil
    import subprocess
    import tempfile

    prof = shutil.which("rocprofv3") or "/opt/rocm/bin/rocprofv3"
    if not os.path.exists(prof):
        return None, "rocprofv3 not found"
    out = {}
    with tempfile.TemporaryDirectory(prefix="lqcd_pmc_") as tmp:
        env = dict(os.environ, TMPDIR=tmp)
        for counter in ("FETCH_SIZE", "WRITE_SIZE"):
            d = os.path.join(tmp, counter)
            cmd = [prof, "--pmc", counter, "-d", d, "-o", "run", "--output-format", "csv", "--",
                   sys.executable, os.path.abspath(__file__), "--only", "apply", "--calibrate",
                   "--steps", str(steps), "--warmup", "1"]
            try:
                r = subprocess.run(cmd, capture_output=True, text=True, timeout=240, env=env, cwd=ROOT)
            except subprocess.TimeoutExpired:
                return None, f"rocprofv3 {counter} run timed out"
            files = glob.glob(os.path.join(d, "**", "run_counter_collection.csv"), recursive=True)
            if r.returncode not in (0, 139) or not files:
                return None, f"rocprofv3 {counter} run failed (status {r.returncode}): {r.stderr[-300:]}"
            vals = {}
            for row in csv.DictReader(open(files[0])):
                vals.setdefault(row["Kernel_Name"], []).append(float(row["Counter_Value"]))
            info = json.loads([l for l in r.stdout.splitlines() if l.startswith("{")][-1])
            wk = [k for k in vals if "k_wilson_full" in k]
            ck = [k for k in vals if "k_copy<4, false>" in k]
            if len(wk) != 1 or not ck:
                return None, f"{counter}: kernels not found in the counter output ({list(vals)[:4]})"
            kib = float(np.mean(vals[wk[0]]))
            copy_kib = float(np.mean([v for k in ck for v in vals[k]]))
            true_copy = info["copy_bytes_per_array"]  # bytes read and bytes written by one copy launch
            out[counter] = {"kib_per_launch": kib, "copy_kib_per_launch": copy_kib, "scale": true_copy / (copy_kib * 1024),
                            "bytes_per_launch": kib * 1024 * true_copy / (copy_kib * 1024), "kernel": wk[0][:80],
                            "launches": len(vals[wk[0]])}
    read, write = out["FETCH_SIZE"]["bytes_per_launch"], out["WRITE_SIZE"]["bytes_per_launch"]
    return {"read_bytes": round(read), "write_bytes": round(write), "total_bytes": round(read + write),
            "fetch_scale": round(out["FETCH_SIZE"]["scale"], 4), "write_scale": round(out["WRITE_SIZE"]["scale"], 4),
            "kernel": out["FETCH_SIZE"]["kernel"], "launches_counted": out["FETCH_SIZE"]["launches"],
            "method": "rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE, one child process each (bench.py --only apply "
                      "--calibrate), scaled by the counters of a plain device copy of known size"}, None


def solve_times(lq, U64, b, mode, reps, warm, work, **kw):
    """Wall-clock seconds of `reps` solves after `warm` warm-up solves (all to
    the same tolerance, same workspace and solution buffer, both allocated
    before the timed region); returns (times, x, stats, status)."""
    import torch

    times, st, rc = [], None, None
    x = torch.empty_like(b)  # allocated outside the timed solves
    for i in range(warm + reps):
        torch.cuda.synchronize()
        t = time.time()
        x, st, rc = lq.gmres_solve(U64, b, M0, layout=lq.LAYOUT2, work=work, mode=mode, out=x, **kw)
        torch.cuda.synchronize()
        if i >= warm:
            times.append(time.time() - t)
    return times, x, st, rc


def time_stats(ts):
    ts = sorted(ts)
    return {"seconds": round(float(np.median(ts)), 3), "seconds_min": round(ts[0], 3),
            "seconds_max": round(ts[-1], 3), "solves_timed": len(ts)}


def gmres_section(lq, U64, psi64, nrhs, reps=3):
    """Time to a true relative residual of 1e-10 of the full system with odd-even
    GMRES(30): FP64 against FP64 refinement around FP32 and FP16-storage inner
    solves, each the median of `reps` solves after a warm-up solve; plus the
    fixed 100-iteration protocol (10 restarts of 10)."""
    import torch

    b = psi64[..., :nrhs].contiguous()
    out = {"lattice": list(DIMS), "nrhs": nrhs, "m0": M0, "restart": 30, "eo": True, "tol": 1e-10}
    sols = {}
    kw = dict(restart=30, eo=True, tol=1e-10, max_restarts=400, max_outer=60)
    for mode in ("f64", "ir-f32", "ir-f16"):
        p = lq.solver_params(mode=mode, **kw)
        work = torch.empty(lq.gmres_workspace_bytes(DIMS, nrhs, p), dtype=torch.uint8, device=b.device)
        ts, x, st, rc = solve_times(lq, U64, b, mode, reps, 1, work, **kw)
        sols[mode] = x
        rec = dict(time_stats(ts), converged=bool(st["converged"].all()), status=int(rc),
                   max_true_relres=float(st["true_relres"].max()),
                   true_relres_per_rhs=[float("%.3e" % v) for v in st["true_relres"]],
                   iters_max=int(st["iters"].max()), iters_mean=float(st["iters"].mean()),
                   outer_max=int(st["outer_iters"].max()), workspace_gb=round(work.numel() / 1e9, 2))
        if mode != "f64":
            # per rhs: ||x_mode - x_f64|| / ||x_f64|| (the FP64 GPU solve is checked against the oracle in tests)
            d = (x - sols["f64"]).reshape(-1, nrhs)
            rel = torch.linalg.vector_norm(d, dim=0) / torch.linalg.vector_norm(sols["f64"].reshape(-1, nrhs), dim=0)
            rec["max_rel_diff_vs_f64"] = float(rel.max())
            rec["rel_diff_vs_f64_per_rhs"] = [float("%.3e" % v) for v in rel.cpu().tolist()]
        log(f"GMRES {mode}: {json.dumps(rec)}")
        out[mode] = rec
        del work
        torch.cuda.empty_cache()
    out["speedup_ir_f32"] = round(out["f64"]["seconds"] / out["ir-f32"]["seconds"], 3)
    out["speedup_ir_f16"] = round(out["f64"]["seconds"] / out["ir-f16"]["seconds"], 3)
    # the paper's solver protocol: exactly 100 iterations (10 restarts x 10), FP64
    kwf = dict(restart=10, max_restarts=10, eo=True, fixed_iters=True)
    work = torch.empty(lq.gmres_workspace_bytes(DIMS, nrhs, lq.solver_params(**kwf)), dtype=torch.uint8,
                       device=b.device)
    ts, x, st, rc = solve_times(lq, U64, b, "f64", reps, 1, work, **kwf)
    out["fixed_100_iterations_f64"] = dict(time_stats(ts), ms_per_iteration=round(float(np.median(ts)) * 10, 3),
                                           true_relres_max=float(st["true_relres"].max()))
    log(f"GMRES fixed 100 iterations: {json.dumps(out['fixed_100_iterations_f64'])}")
    return out


def gmres_nrhs_sweep(lq, U64, psi64, result16=None):
    """Odd-even GMRES(30) to a true 1e-10 at nrhs 1, 4, 8, 16, 32 and 64 in the
    three modes (one timed solve per point after a warm-up solve per mode).
    Sources: the benchmark's 16 host-generated rhs, continued beyond 16 by
    Gaussian rhs drawn on the GPU from a seeded generator.  The workspace is
    the full width when it fits the free device memory (less a margin), else
    the largest that does; the library then solves in chunks of the width
    it picks (logged)."""
    import torch

    g = torch.Generator(device=psi64.device).manual_seed(1000 + CONFIG)
    extra = torch.randn(DIMS + (4, 3, 48), dtype=torch.complex128, device=psi64.device, generator=g)
    src = torch.cat([psi64, extra], dim=-1)
    del extra
    kw = dict(restart=30, eo=True, tol=1e-10, max_restarts=400, max_outer=60)
    pts = []
    for mode in ("f64", "ir-f32", "ir-f16"):
        warmed = False
        for n in (1, 4, 8, 16, 32, 64):
            if n == 16 and result16 is not None:
                r = result16[mode]
                pts.append({"nrhs": n, "mode": mode, "seconds": r["seconds"], "seconds_per_rhs":
                            round(r["seconds"] / n, 4), "rhs_block": n, "converged": r["converged"],
                            "max_true_relres": r["max_true_relres"], "iters_max": r["iters_max"],
                            "source": "gmres section (median of its solves)"})
                continue
            b = src[..., :n].contiguous()
            full = lq.gmres_workspace_bytes(DIMS, n, lq.solver_params(mode=mode, **kw))
            free, _ = torch.cuda.mem_get_info()
            nbytes = min(full, free - b.numel() * 16 - (8 << 30))
            p = lq.solver_params(mode=mode, **kw)
            width = lq.gmres_rhs_block(DIMS, n, p, nbytes)
            work = torch.empty(lq.gmres_workspace_bytes(DIMS, n, lq.solver_params(mode=mode, rhs_block=width, **kw)),
                               dtype=torch.uint8, device=b.device)
            ts, x, st, rc = solve_times(lq, U64, b, mode, 1, 0 if warmed else 1, work, **kw)
            warmed = True
            rec = {"nrhs": n, "mode": mode, "seconds": round(ts[0], 3), "seconds_per_rhs": round(ts[0] / n, 4),
                   "rhs_block": width, "converged": bool(st["converged"].all()), "status": int(rc),
                   "max_true_relres": float(st["true_relres"].max()), "iters_max": int(st["iters"].max()),
                   "workspace_gb": round(work.numel() / 1e9, 2)}
            log(f"GMRES sweep: {json.dumps(rec)}")
            pts.append(rec)
            del work, x, b
            torch.cuda.empty_cache()
    del src
    torch.cuda.empty_cache()
    return pts


def block_gmres_section(lq, U64, psi64, nrhs, batched=None):
    """Block GMRES (all rhs share one block Krylov space) on the headline
    system: time and block steps to a true 1e-10 with GMRES(30), odd-even,
    against the batched solver, and the fixed protocol of 100 steps (10
    restarts of 10) for the cost of one block step."""
    import torch

    b = psi64[..., :nrhs].contiguous()
    out = {"lattice": list(DIMS), "nrhs": nrhs, "restart": 30, "eo": True, "tol": 1e-10}
    p = lq.solver_params(restart=30, eo=True, tol=1e-10, max_restarts=400)
    work = torch.empty(lq.block_gmres_workspace_bytes(DIMS, nrhs, p), dtype=torch.uint8, device=b.device)
    torch.cuda.synchronize()
    t = time.time()
    x, st, rc = lq.block_gmres_solve(U64, b, M0, layout=lq.LAYOUT2, work=work, restart=30, eo=True, tol=1e-10,
                                     max_restarts=400)
    torch.cuda.synchronize()
    dt = time.time() - t
    out["to_1e-10"] = {"seconds": round(dt, 3), "status": int(rc), "converged": bool(st["converged"].all()),
                       "block_steps": int(st["iters"].max()), "max_true_relres": float(st["true_relres"].max()),
                       "workspace_gb": round(work.numel() / 1e9, 2)}
    if batched is not None:
        out["to_1e-10"]["batched_f64_seconds"] = batched["seconds"]
        out["to_1e-10"]["batched_f64_steps_max"] = batched["iters_max"]
        out["speedup_vs_batched"] = round(batched["seconds"] / dt, 3)
    log(f"block GMRES to 1e-10: {json.dumps(out['to_1e-10'])}")
    del work
    torch.cuda.empty_cache()
    p = lq.solver_params(restart=10, max_restarts=10, eo=True, fixed_iters=True)
    work = torch.empty(lq.block_gmres_workspace_bytes(DIMS, nrhs, p), dtype=torch.uint8, device=b.device)
    torch.cuda.synchronize()
    t = time.time()
    x, st, rc = lq.block_gmres_solve(U64, b, M0, layout=lq.LAYOUT2, work=work, restart=10, max_restarts=10, eo=True,
                                     fixed_iters=True)
    torch.cuda.synchronize()
    dt = time.time() - t
    out["fixed_100_steps"] = {"seconds": round(dt, 3), "ms_per_step": round(dt * 10, 3),
                              "true_relres_max": float(st["true_relres"].max())}
    log(f"block GMRES fixed 100 steps: {dt:.3f} s")
    del work
    torch.cuda.empty_cache()
    return out


def clover_section(lq, syn, U64, psi64, steps):
    """The clover-improved operator D = D_W - C on the headline workload
    (synthetic clover field, two Hermitian 6x6 blocks per site, scale 0.2):
    full and Schur applies in FP64 and odd-even GMRES(30) to a true 1e-10,
    FP64 against FP32 refinement."""
    import torch

    dev = U64.device
    v = int(np.prod(DIMS))
    t0 = time.time()
    C = torch.from_numpy(syn.clover_field(DIMS, config=CONFIG, scale=0.2)).to(dev)
    log(f"clover field generated ({time.time() - t0:.1f}s)")
    out = {"lattice": list(DIMS), "nrhs": NRHS, "m0": M0, "clover_scale": 0.2}
    eta = torch.empty_like(psi64)
    t_full = timed(lambda: lq.dirac_apply_clover(U64, C, psi64, M0, layout=lq.LAYOUT2, out=eta), steps, 2)
    nb = (36 + 42 + 24 * NRHS) * 16 * v  # links, clover field, in, out
    Ci = lq.clover_inverse(C, M0, DIMS)
    xe = psi64.reshape((v,) + tuple(psi64.shape[4:]))[: v // 2].contiguous()
    ye = torch.empty_like(xe)
    t_eo = timed(lambda: lq.dirac_apply_eo_clover(U64, C, Ci, xe, M0, layout=lq.LAYOUT2, out=ye), steps, 2)
    out["apply_f64"] = {"full_ms": round(t_full, 4), "full_gbs": round(nb / t_full / 1e6, 1),
                        # + 528 flop per site and rhs: two Hermitian 6x6 block products and the subtraction
                        "full_gflops": round((FLOP_SITE_RHS + 528) * v * NRHS / t_full / 1e6, 1),
                        "schur_ms": round(t_eo, 4),
                        "kernel": "full: time-streaming pencils; Schur: one (site, rhs) per work item"}
    log(f"clover apply FP64 nrhs={NRHS}: full {t_full:.3f} ms ({nb / t_full / 1e6:.0f} GB/s), Schur {t_eo:.3f} ms")
    del eta, ye, xe, Ci
    torch.cuda.empty_cache()
    b = psi64[..., :NRHS].contiguous()
    sol = {}
    for mode in ("f64", "ir-f32"):
        torch.cuda.synchronize()
        t = time.time()
        x, st, rc = lq.gmres_solve_clover(U64, C, b, M0, layout=lq.LAYOUT2, restart=30, eo=True, mode=mode,
                                          tol=1e-10, max_restarts=400, max_outer=60)
        torch.cuda.synchronize()
        dt = time.time() - t
        rec = {"seconds": round(dt, 3), "status": int(rc), "converged": bool(st["converged"].all()),
               "max_true_relres": float(st["true_relres"].max()), "iters_max": int(st["iters"].max())}
        if mode != "f64":
            d = (x - sol["f64"]).reshape(-1, NRHS)
            rel = torch.linalg.vector_norm(d, dim=0) / torch.linalg.vector_norm(sol["f64"].reshape(-1, NRHS), dim=0)
            rec["max_rel_diff_vs_f64"] = float(rel.max())
        sol[mode] = x
        out["gmres_" + mode.replace("-", "_")] = rec
        log(f"clover GMRES {mode}: {json.dumps(rec)}")
    out["speedup_ir_f32"] = round(out["gmres_f64"]["seconds"] / out["gmres_ir_f32"]["seconds"], 3)
    del sol, C
    torch.cuda.empty_cache()
    return out


def batch_section(lq, syn, steps):
    """The uneven eight-lattice batch (L = 8..24, T = 2L, eps_k = 0.2 + 0.3 k/7,
    1..32 rhs each, m0 = -0.05): the FP32 apply of all eight lattices in one
    persistent launch against eight separate launches, and the batched GMRES(30)
    to a true 1e-10 (FP32 operator inside FP64 refinement), eager and with
    hipGraph-captured Arnoldi steps, against solving the lattices one after
    the other the same way (each the median of three runs after a warm-up)."""
    import torch

    dev = torch.device("cuda:0")
    comp = syn.batch_composition()
    t0 = time.time()
    probs64 = []
    for c in comp:
        U = syn.gauge_field(c["dims"], "near_identity", config=40 + c["index"], eps=c["eps"])
        b = syn.spinor_block(c["dims"], c["nrhs"], config=40 + c["index"])
        probs64.append((torch.from_numpy(U).to(dev), torch.from_numpy(np.ascontiguousarray(np.moveaxis(b, 0, -1))).to(dev),
                        M0))
    log(f"batch inputs generated ({time.time() - t0:.1f}s)")
    out = {"lattices": [list(c["dims"]) for c in comp], "nrhs": [c["nrhs"] for c in comp],
           "eps": [round(c["eps"], 4) for c in comp], "m0": M0}
    # ------------------------------------------------ FP32 apply, one launch vs eight
    probs32 = [(U.to(torch.complex64), b.to(torch.complex64), m0) for U, b, m0 in probs64]
    outs = [torch.empty_like(b) for _, b, _ in probs32]
    # per-lattice kernel configurations first: the separate launches use them
    # directly, the persistent launch takes each lattice's pencil geometry
    for U, b, m0 in probs32:
        lq.autotune(U, b, torch.empty_like(b), m0, layout=lq.LAYOUT2, reps=2)
    batch_cfg = lq.autotune_batch(probs32, outs, reps=3)
    t_batch = timed(lambda: lq.dirac_apply_batch(probs32, outs=outs), steps, 2)
    t_seq = timed(lambda: [lq.dirac_apply(U, b, m0, layout=lq.LAYOUT2, out=o) for (U, b, m0), o in zip(probs32, outs)],
                  steps, 2)
    nbytes = sum(bytes_full(int(np.prod(c["dims"])), c["nrhs"], 8) for c in comp)
    out["apply_f32"] = {"one_launch_ms": round(t_batch, 4), "eight_launches_ms": round(t_seq, 4),
                        "persistent_config": batch_cfg, "gbs_one_launch": round(nbytes / t_batch / 1e6, 1),
                        "gbs_eight_launches": round(nbytes / t_seq / 1e6, 1)}
    log(f"batch apply FP32: one launch {t_batch:.3f} ms, eight launches {t_seq:.3f} ms")
    del probs32, outs
    torch.cuda.empty_cache()
    # ------------------------------------------------ batched GMRES vs one solve per lattice
    # (each the median of three after a warm-up run)
    kw = dict(restart=30, eo=True, mode="ir-f32", tol=1e-10, max_restarts=400, max_outer=60)

    def batched(graph):
        def f():
            xs, stats, rc = lq.gmres_solve_batch(probs64, use_graph=graph, **kw)
            return stats, rc
        return f

    def sequential(graph):
        def f():
            out = []
            for U, b, m0 in probs64:
                x, st, rc1 = lq.gmres_solve(U, b, m0, layout=lq.LAYOUT2, use_graph=graph, **kw)
                out.append(st)
                del x
            return out, None
        return f

    def run(fn):
        ts, res = [], None
        for i in range(4):
            torch.cuda.synchronize()
            t = time.time()
            res = fn()
            torch.cuda.synchronize()
            if i:
                ts.append(time.time() - t)
        return ts, res

    res = {}
    for graph in (False, True):
        ts_b, (stats, rc) = run(batched(graph))
        ts_s, (sstats, _) = run(sequential(graph))
        rec = dict(time_stats(ts_b), status=int(rc), converged=bool(all(st["converged"].all() for st in stats)),
                   max_true_relres=float(max(st["true_relres"].max() for st in stats)),
                   iters_max=[int(st["iters"].max()) for st in stats])
        seq = dict(time_stats(ts_s), converged=bool(all(st["converged"].all() for st in sstats)),
                   max_true_relres=float(max(st["true_relres"].max() for st in sstats)))
        tag = "graph" if graph else "eager"
        res[tag] = {"batched": rec, "one_lattice_at_a_time": seq,
                    "speedup_batched": round(seq["seconds"] / rec["seconds"], 3)}
        log(f"batch GMRES ir-f32 ({tag}): batched {rec['seconds']:.3f} s, one at a time {seq['seconds']:.3f} s")
    torch.cuda.empty_cache()
    out["gmres_ir_f32"] = dict(res, restart=30, tol=1e-10)
    return out


def small_section(lq, syn, with_oracle):
    """The small workloads beside the headline: a 4^4 Haar lattice (m0 = 0.1,
    one rhs: one apply and GMRES(30) on the full system; launch-latency
    bound, not a roofline point) and a 16^3 x 32 near-identity lattice
    (m0 = -0.05, nrhs 1 / 4 / 12: full and Schur applies in FP64 and FP32,
    labelled cache-resident because the working set is of the order of the
    256 MB Infinity Cache; odd-even GMRES(30) to 1e-10 at 12 rhs, FP64 against
    FP32 refinement), with the oracle timed on the same inputs (4^4 apply and
    GMRES; one rhs of the 16^3 x 32 apply)."""
    import torch

    dev = torch.device("cuda:0")
    out = {}
    dims = (4, 4, 4, 4)
    U = syn.gauge_field(dims, "haar", config=1)
    b = syn.spinor_block(dims, 1, config=1)
    Ud = torch.from_numpy(U).to(dev)
    bd = torch.from_numpy(np.ascontiguousarray(np.moveaxis(b, 0, -1))).to(dev)
    ms = timed(lambda: lq.dirac_apply(Ud, bd, 0.1, layout=lq.LAYOUT2), 20, 3)
    torch.cuda.synchronize()
    t = time.time()
    x, st, rc = lq.gmres_solve(Ud, bd, 0.1, layout=lq.LAYOUT2, eo=False, restart=30, tol=1e-10)
    torch.cuda.synchronize()
    w1 = {"lattice": list(dims), "nrhs": 1, "apply_ms": round(ms, 4), "gmres_seconds": round(time.time() - t, 4),
          "gmres_iters": int(st["iters"][0]), "converged": bool(st["converged"].all())}
    if with_oracle:
        from oracle import dirac, solve as osolve

        t = time.time()
        dirac.apply_dw(U, b, 0.1)
        w1["oracle_apply_s"] = round(time.time() - t, 4)
        t = time.time()
        _, ost = osolve.solve(U, b, 0.1, tol=1e-10, restart=30, eo=False)
        w1["oracle_gmres_s"] = round(time.time() - t, 3)
        w1["oracle_gmres_iters"] = int(ost.iters[0])
    out["haar_4x4x4x4"] = w1
    log(f"4^4: {json.dumps(w1)}")

    dims = (32, 16, 16, 16)
    v = int(np.prod(dims))
    U = syn.gauge_field(dims, "near_identity", config=2, eps=EPS)
    psi = syn.spinor_block(dims, 12, config=2)
    U64 = torch.from_numpy(U).to(dev)
    p64 = torch.from_numpy(np.ascontiguousarray(np.moveaxis(psi, 0, -1))).to(dev)
    pts = []
    for prec_name, prec, esz in (("f64", lq.F64, 16), ("f32", lq.F32, 8)):
        Up = U64 if prec == lq.F64 else U64.to(torch.complex64)
        for n in (1, 4, 12):
            x = p64[..., :n].contiguous()
            x = x if prec == lq.F64 else x.to(torch.complex64)
            y = torch.empty_like(x)
            tf = timed(lambda: lq.dirac_apply(Up, x, -0.05, layout=lq.LAYOUT2, out=y), 20, 3)
            xe = x.reshape((v,) + tuple(x.shape[4:]))[: v // 2].contiguous()
            ye = torch.empty_like(xe)
            te = timed(lambda: lq.dirac_apply_eo(Up, xe, -0.05, layout=lq.LAYOUT2, out=ye), 20, 3)
            pts.append({"prec": prec_name, "nrhs": n, "full_ms": round(tf, 4),
                        "full_gbs": round(bytes_full(v, n, esz) / tf / 1e6, 1), "schur_ms": round(te, 4),
                        "schur_gbs_two_pass": round(bytes_schur_two_pass(v, n, esz) / te / 1e6, 1),
                        "working_set_mb": round((bytes_full(v, n, esz)) / 1e6, 1), "cache_resident": True})
    w2 = {"lattice": list(dims), "applies": pts}
    b12 = p64.contiguous()
    for mode in ("f64", "ir-f32"):
        torch.cuda.synchronize()
        t = time.time()
        x, st, rc = lq.gmres_solve(U64, b12, -0.05, layout=lq.LAYOUT2, eo=True, restart=30, tol=1e-10, mode=mode)
        torch.cuda.synchronize()
        w2["gmres_" + mode.replace("-", "_")] = {"seconds": round(time.time() - t, 3), "status": int(rc),
                                                  "iters_max": int(st["iters"].max()),
                                                  "max_true_relres": float(st["true_relres"].max())}
    if with_oracle:
        from oracle import dirac

        t = time.time()
        dirac.apply_dw(U, psi[:1], -0.05)
        w2["oracle_apply_s_per_rhs"] = round(time.time() - t, 3)
    out["near_identity_16x16x16x32"] = w2
    log(f"16^3x32: GMRES f64 {w2['gmres_f64']['seconds']} s, ir-f32 {w2['gmres_ir_f32']['seconds']} s")
    return out


def autograd_section(lq, syn):
    """Differentiation at 16^3 x 32, nrhs = 8, m0 = 0.05: forward solve, then the
    backward of L = sum_i Re<chi_i, x_i> (adjoint solve, link force, dL/dm0)."""
    import torch

    from paper_2601_05816_amd.autograd import wilson_solve

    dev = torch.device("cuda:0")
    dims, nrhs, m0 = (32, 16, 16, 16), 8, 0.05
    U = torch.from_numpy(syn.gauge_field(dims, "near_identity", config=5, eps=EPS)).to(dev).requires_grad_(True)
    eta = torch.from_numpy(np.ascontiguousarray(np.moveaxis(syn.spinor_block(dims, nrhs, config=5), 0, -1))).to(dev)
    chi = torch.from_numpy(np.ascontiguousarray(np.moveaxis(syn.spinor_block(dims, nrhs, config=5, role=syn.ROLE_CHI), 0, -1))).to(dev)
    eta.requires_grad_(True)
    m = torch.tensor(m0, dtype=torch.float64, device=dev, requires_grad=True)
    res = {}
    for rep in range(2):  # the second repetition is reported (first-call set-up excluded)
        torch.cuda.synchronize()
        t = time.time()
        x = wilson_solve(U, eta, m, restart=30, eo=True, tol=1e-10)
        torch.cuda.synchronize()
        t_fwd = time.time() - t
        loss = (torch.conj(chi) * x).real.sum()
        t = time.time()
        loss.backward()
        torch.cuda.synchronize()
        t_bwd = time.time() - t
        res = {"lattice": list(dims), "nrhs": nrhs, "m0": m0, "forward_solve_s": round(t_fwd, 3),
               "backward_s": round(t_bwd, 3), "grad_U_norm": float(U.grad.norm()), "grad_m0": float(m.grad)}
        U.grad = None
        eta.grad = None
        m.grad = None
    log(f"autograd: forward {res['forward_solve_s']} s, backward {res['backward_s']} s")
    return res


def profile_only(args):
    """One workload under a profiler: GPU-drawn inputs (timing does not depend
    on the values; gmres-ir and gmres-sweep solve on the benchmark's
    near-identity links, whose iteration counts they reproduce), the kernel configurations of the
    tune file, `--steps` launches after `--warmup`; prints one JSON line of
    launch times."""
    import torch

    import paper_2601_05816_amd as lq

    lq.load()
    if os.path.exists(args.tune_file):
        lq.tune_load(args.tune_file)
    if args.variant or args.pencil:
        pv = [int(v) for v in args.pencil.split(",")] if args.pencil else [0, 0, 0, 0]
        pv += [0] * (5 - len(pv))
        lq.set_kernel_config(args.variant or 2, *pv)
    dev = torch.device("cuda:0")
    g = torch.Generator(device=dev).manual_seed(CONFIG)
    v = int(np.prod(DIMS))
    U = torch.randn((4,) + DIMS + (3, 3), dtype=torch.complex128, device=dev, generator=g)
    out = {"mode": args.only, "lattice": list(DIMS), "steps": args.steps, "warmup": args.warmup}
    if args.only == "apply":
        prec = {"f64": lq.F64, "f32": lq.F32, "f16": lq.F16}[args.prec]
        n = args.nrhs

        def conv(x):
            if prec == lq.F64:
                return x
            return x.to(torch.complex64) if prec == lq.F32 else to_f16(x)

        Up = conv(U)
        if args.kind == "full":
            x = conv(torch.randn(DIMS + (4, 3, n), dtype=torch.complex128, device=dev, generator=g))
            y = torch.empty_like(x)
            fn = lambda: lq.dirac_apply(Up, x, M0, layout=lq.LAYOUT2, out=y)
            alg = bytes_full(v, n, {lq.F64: 16, lq.F32: 8, lq.F16: 4}[prec])
        else:
            x = conv(torch.randn((v // 2, 4, 3, n), dtype=torch.complex128, device=dev, generator=g))
            y = torch.empty_like(x)
            wk = torch.empty(lq.dirac_apply_eo_workspace_bytes(DIMS, n, prec), dtype=torch.uint8, device=dev)
            fn = lambda: lq.dirac_apply_eo_ws(Up, x, M0, wk, layout=lq.LAYOUT2, out=y)
            alg = bytes_schur_two_pass(v, n, {lq.F64: 16, lq.F32: 8, lq.F16: 4}[prec])
            # one pass over links, input and output: what a fused apply must move
            out["fused_minimum_bytes"] = (72 + 24 * n) * {lq.F64: 16, lq.F32: 8, lq.F16: 4}[prec] * (v // 2)
        ms = timed(fn, args.steps, args.warmup)
        out.update(prec=args.prec, kind=args.kind, nrhs=n, ms=round(ms, 4), algorithmic_bytes=alg,
                   gbs_algorithmic=round(alg / ms / 1e6, 1))
        log(f"{args.kind} {args.prec} nrhs {n}: {ms:.4f} ms")
        if args.calibrate:
            del x, y, Up, U
            torch.cuda.empty_cache()
            na = 1 << 28  # doubles per array: 2 GiB read and 2 GiB written per copy launch
            a = torch.ones(na, dtype=torch.float64, device=dev)
            b = torch.empty_like(a)
            lq.hbm_probe(a, b, kind="copy", reps=1)
            out["copy_bytes_per_array"] = na * 8
    elif args.only == "sweep-f64":
        pts = []
        for n in (1, 4, 8, 16, 32, 64):  # dispatches: warmup + steps launches per point, in this order
            psi = torch.randn(DIMS + (4, 3, n), dtype=torch.complex128, device=dev, generator=g)
            eta = torch.empty_like(psi)
            ms = timed(lambda: lq.dirac_apply(U, psi, M0, layout=lq.LAYOUT2, out=eta), args.steps, args.warmup)
            pts.append({"nrhs": n, "ms": round(ms, 4)})
            log(f"nrhs {n}: {ms:.4f} ms")
            del psi, eta
        out["points"] = pts
    elif args.only == "schur-f64":
        xe = torch.randn((v // 2, 4, 3, NRHS), dtype=torch.complex128, device=dev, generator=g)
        ye = torch.empty_like(xe)
        wk = torch.empty(lq.dirac_apply_eo_workspace_bytes(DIMS, NRHS, lq.F64), dtype=torch.uint8, device=dev)
        ms = timed(lambda: lq.dirac_apply_eo_ws(U, xe, M0, wk, layout=lq.LAYOUT2, out=ye), args.steps, args.warmup)
        out.update(nrhs=NRHS, schur_ms=round(ms, 4))
    elif args.only == "schur-sizes":
        # the tuned Schur apply at 16 rhs on 2L x L^3 lattices whose working set
        # (links, input, output, odd temporary) fits the 256 MB Infinity Cache
        # or not: time per even site and rhs
        pts = []
        for L in (16, 20, 24, 32):
            dims = (2 * L, L, L, L)
            vol = 2 * L ** 4
            for pn, prec, esz in (("f16", lq.F16, 4), ("f32", lq.F32, 8), ("f64", lq.F64, 16)):
                def conv(x):
                    if prec == lq.F64:
                        return x
                    return x.to(torch.complex64) if prec == lq.F32 else to_f16(x)

                Ul = conv(torch.randn((4,) + dims + (3, 3), dtype=torch.complex128, device=dev, generator=g))
                xe = conv(torch.randn((vol // 2, 4, 3, NRHS), dtype=torch.complex128, device=dev, generator=g))
                ye = torch.empty_like(xe)
                wk = torch.empty(lq.dirac_apply_eo_workspace_bytes(dims, NRHS, prec), dtype=torch.uint8, device=dev)
                lq.autotune(Ul, xe, ye, layout=lq.LAYOUT2, eo=True, reps=3)
                ms = timed(lambda: lq.dirac_apply_eo_ws(Ul, xe, M0, wk, layout=lq.LAYOUT2, out=ye), args.steps,
                           args.warmup)
                foot = (4 * vol * 9 + 3 * (vol // 2) * 12 * NRHS) * esz  # links, input, output, odd temporary
                pts.append({"lattice": list(dims), "prec": pn, "ms": round(ms, 4), "working_set_mb": round(foot / 2**20),
                            "ns_per_even_site_rhs": round(ms * 1e6 / (vol // 2 * NRHS), 4)})
                log(f"schur-sizes: {json.dumps(pts[-1])}")
                del Ul, xe, ye, wk
                torch.cuda.empty_cache()
        out["points"] = pts
    elif args.only == "block-hard":
        # block against batched GMRES(30), odd-even, 16 rhs, to a true 1e-10 on
        # 16^3 x 32 near-identity links (eps 0.3) as m0 moves towards the
        # critical mass: steps and seconds of each
        import lqcd_synth as syn

        dims = (32, 16, 16, 16)
        Uh = torch.from_numpy(syn.gauge_field(dims, "near_identity", config=CONFIG, eps=EPS)).to(dev)
        bh = torch.randn(dims + (4, 3, NRHS), dtype=torch.complex128, device=dev, generator=g)
        pts = []
        for m0 in (-0.05, -0.15, -0.25, -0.35):
            kw = dict(restart=30, eo=True, tol=1e-10, max_restarts=2000)
            rec = {"lattice": list(dims), "nrhs": NRHS, "m0": m0}
            for name, fn in (("batched", lq.gmres_solve), ("block", lq.block_gmres_solve)):
                fn(Uh, bh, m0, layout=lq.LAYOUT2, **dict(kw, max_restarts=1))  # warm-up
                torch.cuda.synchronize()
                t = time.time()
                _, st, rc = fn(Uh, bh, m0, layout=lq.LAYOUT2, **kw)
                torch.cuda.synchronize()
                dt = time.time() - t
                steps = int(st["iters"].max())
                rec[name] = {"seconds": round(dt, 3), "steps": steps, "ms_per_step": round(dt * 1e3 / steps, 3),
                             "status": int(rc), "max_true_relres": float(st["true_relres"].max())}
            log(f"block-hard: {json.dumps(rec)}")
            pts.append(rec)
        out["points"] = pts
    elif args.only == "clover-f64":  # D = D_W - C: full apply, then the Schur apply (two passes)
        C = 0.1 * torch.randn(DIMS + (42,), dtype=torch.complex128, device=dev, generator=g)
        Ci = 0.1 * torch.randn(DIMS + (42,), dtype=torch.complex128, device=dev, generator=g)
        psi = torch.randn(DIMS + (4, 3, NRHS), dtype=torch.complex128, device=dev, generator=g)
        eta = torch.empty_like(psi)
        ms = timed(lambda: lq.dirac_apply_clover(U, C, psi, M0, layout=lq.LAYOUT2, out=eta), args.steps, args.warmup)
        xe = psi.reshape((v, 4, 3, NRHS))[: v // 2].contiguous()
        ye = torch.empty_like(xe)
        me = timed(lambda: lq.dirac_apply_eo_clover(U, C, Ci, xe, M0, layout=lq.LAYOUT2, out=ye), args.steps,
                   args.warmup)
        out.update(nrhs=NRHS, full_ms=round(ms, 4), schur_ms=round(me, 4))
        log(f"clover full {ms:.4f} ms, Schur {me:.4f} ms")
    elif args.only == "block-fixed":  # block GMRES, 100 block steps = 10 restarts of 10, odd-even
        U.mul_(0.3)
        b = torch.randn(DIMS + (4, 3, NRHS), dtype=torch.complex128, device=dev, generator=g)
        kw = dict(restart=10, max_restarts=10, eo=True, fixed_iters=True)
        work = torch.empty(lq.block_gmres_workspace_bytes(DIMS, NRHS, lq.solver_params(**kw)), dtype=torch.uint8,
                           device=dev)
        out["seconds"] = []
        for i in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t = time.time()
            lq.block_gmres_solve(U, b, M0, layout=lq.LAYOUT2, work=work, **kw)
            torch.cuda.synchronize()
            out["seconds"].append(round(time.time() - t, 3))
            log(f"block GMRES 100 steps ({'warmup' if i < args.warmup else 'timed'}): {out['seconds'][-1]} s")
    elif args.only == "gmres-ir":  # refinement solves to 1e-10 on the benchmark's near-identity links
        import lqcd_synth as syn

        U = torch.from_numpy(syn.gauge_field(DIMS, "near_identity", config=CONFIG, eps=EPS)).to(dev)
        b = torch.randn(DIMS + (4, 3, args.nrhs), dtype=torch.complex128, device=dev, generator=g)
        x = torch.empty_like(b)
        for mode in ("ir-f16", "ir-f32"):
            kw = dict(restart=30, eo=True, mode=mode, tol=1e-10, max_restarts=400, max_outer=60)
            # the full width if its workspace fits the free memory, else the library's chunk width
            p = lq.solver_params(**kw)
            free, _ = torch.cuda.mem_get_info()
            nbytes = min(lq.gmres_workspace_bytes(DIMS, args.nrhs, p), free - (8 << 30))
            kw["rhs_block"] = lq.gmres_rhs_block(DIMS, args.nrhs, p, nbytes)
            work = torch.empty(lq.gmres_workspace_bytes(DIMS, args.nrhs, lq.solver_params(**kw)), dtype=torch.uint8,
                               device=dev)
            out[mode] = []
            for i in range(args.warmup + args.steps):
                torch.cuda.synchronize()
                t = time.time()
                _, st, rc = lq.gmres_solve(U, b, M0, layout=lq.LAYOUT2, work=work, out=x, **kw)
                torch.cuda.synchronize()
                out[mode].append(round(time.time() - t, 3))
                log(f"{mode} to 1e-10 ({'warmup' if i < args.warmup else 'timed'}): {out[mode][-1]} s, "
                    f"{int(st['iters'].max())} steps, status {rc}, rhs_block {kw['rhs_block']}")
            del work
            torch.cuda.empty_cache()
    elif args.only == "gmres-sweep":  # the GMRES nrhs sweep of the full run, on the benchmark's links and rhs
        import lqcd_synth as syn

        U = torch.from_numpy(syn.gauge_field(DIMS, "near_identity", config=CONFIG, eps=EPS)).to(dev)
        psi = syn.spinor_block(DIMS, NRHS, config=CONFIG)
        psi = torch.from_numpy(np.ascontiguousarray(np.moveaxis(psi, 0, -1))).to(dev)
        out["points"] = gmres_nrhs_sweep(lq, U, psi)
    else:  # the paper's fixed protocol: 100 iterations = 10 restarts of 10, odd-even, FP64
        U.mul_(0.3)
        b = torch.randn(DIMS + (4, 3, NRHS), dtype=torch.complex128, device=dev, generator=g)
        kw = dict(restart=10, max_restarts=10, eo=True, fixed_iters=True)
        work = torch.empty(lq.gmres_workspace_bytes(DIMS, NRHS, lq.solver_params(**kw)), dtype=torch.uint8,
                           device=dev)
        out["seconds"] = []
        for i in range(args.warmup + args.steps):
            torch.cuda.synchronize()
            t = time.time()
            lq.gmres_solve(U, b, M0, layout=lq.LAYOUT2, work=work, **kw)
            torch.cuda.synchronize()
            out["seconds"].append(round(time.time() - t, 3))
            log(f"fixed 100 iterations ({'warmup' if i < args.warmup else 'timed'}): {out['seconds'][-1]} s")
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--fast-inputs", action="store_true",
                    help="draw the inputs on the GPU (seeded torch generator) instead of the seeded host "
                         "recipe; for profiling runs, where values do not matter (skips the solver sections, the "
                         "small workloads and the oracle baseline)")
    ap.add_argument("--no-gmres", action="store_true")
    ap.add_argument("--no-batch", action="store_true", help="skip the uneven eight-lattice batch")
    ap.add_argument("--no-clover", action="store_true", help="skip the clover-improved operator")
    ap.add_argument("--no-block", action="store_true", help="skip block GMRES")
    ap.add_argument("--no-small", action="store_true", help="skip the 4^4 and 16^3 x 32 workloads")
    ap.add_argument("--no-autograd", action="store_true", help="skip the differentiation timing")
    ap.add_argument("--gmres-nrhs", type=int, default=NRHS)
    ap.add_argument("--variant", type=int, default=0,
                    help="force a Wilson kernel variant (0 automatic; 1-8 as lqcd_set_kernel_config, 8 = the fused "
                         "Schur apply)")
    ap.add_argument("--pencil", type=str, default="",
                    help="tile Y,tile Z,t segments[,nontemporal[,workgroups per CU]] for the forced variant")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run a plain 2 GiB device copy (for scaling HBM byte counters)")
    ap.add_argument("--tune-file", default=TUNE_FILE,
                    help="kernel configurations measured by the autotuner on MI355X (used when present)")
    ap.add_argument("--retune", action="store_true", help="ignore the tune file and autotune every apply")
    ap.add_argument("--save-tune", default="", help="write the autotuner's table here at the end")
    ap.add_argument("--only", choices=["apply", "sweep-f64", "schur-f64", "schur-sizes", "clover-f64", "gmres-fixed",
                                       "block-fixed", "block-hard", "gmres-ir", "gmres-sweep"],
                    default="",
                    help="profiling mode: run one workload only (GPU-drawn inputs except the near-identity links of "
                         "gmres-ir, tune file), print its times")
    ap.add_argument("--prec", choices=["f64", "f32", "f16"], default="f64", help="--only apply: storage precision")
    ap.add_argument("--kind", choices=["full", "schur"], default="full", help="--only apply: full D_W or Schur S")
    ap.add_argument("--nrhs", type=int, default=NRHS, help="--only apply / gmres-ir: rhs count")
    ap.add_argument("--calibrate", action="store_true",
                    help="--only apply: also run the HBM probe's plain copy (for scaling byte counters)")
    ap.add_argument("--no-counters", action="store_true",
                    help="skip the rocprofv3 counter runs that measure the headline kernel's HBM traffic")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the multi-rhs apply and GMRES are single-device here "
              "(rhs or lattice sharding across GPUs is not built)", file=sys.stderr)
        sys.exit(2)
    if args.only:
        profile_only(args)
        return

    # the headline kernel's HBM traffic, counted in child processes before
    # this one touches the GPU
    traffic, traffic_note = None, "not measured (--no-counters or a forced kernel configuration)"
    if not (args.no_counters or args.variant or args.pencil or args.retune) and os.path.exists(args.tune_file):
        t0c = time.time()
        traffic, traffic_note = measure_traffic()
        log(f"counters: {traffic if traffic else traffic_note} ({time.time() - t0c:.0f}s)")

    import torch

    import lqcd_synth as syn
    import paper_2601_05816_amd as lq

    lq.load()
    if args.variant or args.pencil:
        pv = [int(v) for v in args.pencil.split(",")] if args.pencil else [0, 0, 0, 0]
        pv += [0] * (5 - len(pv))
        lq.set_kernel_config(args.variant or 2, *pv)
    dev = torch.device("cuda:0")
    v = int(np.prod(DIMS))
    t0 = time.time()
    if args.fast_inputs:
        args.no_gmres = args.no_block = args.no_small = True
        gen = torch.Generator(device=dev).manual_seed(CONFIG)
        U64 = torch.randn((4,) + DIMS + (3, 3), dtype=torch.complex128, device=dev, generator=gen)
        psi64 = torch.randn(DIMS + (4, 3, NRHS), dtype=torch.complex128, device=dev, generator=gen)
        U = psi_np = None
        args.no_cpu = True
    else:
        U = syn.gauge_field(DIMS, "near_identity", config=CONFIG, eps=EPS)
        log(f"gauge field generated ({time.time() - t0:.1f}s)")
        psi_np = syn.spinor_block(DIMS, NRHS, config=CONFIG)
        log(f"spinors generated ({time.time() - t0:.1f}s)")
        U64 = torch.from_numpy(U).to(dev)
        psi64 = torch.from_numpy(np.ascontiguousarray(np.moveaxis(psi_np, 0, -1))).to(dev)
    eta64 = torch.empty_like(psi64)
    torch.cuda.synchronize()
    log("inputs resident on the GPU")

    # ------------------------------------------------- measured HBM ceiling
    n = 1 << 30  # 8 GiB per array
    a = torch.zeros(n, dtype=torch.float64, device=dev)
    bb = torch.ones(n, dtype=torch.float64, device=dev)
    cc = torch.ones(n, dtype=torch.float64, device=dev)
    t_copy = lq.hbm_probe(a, bb, kind="copy")
    t_triad = lq.hbm_probe(a, bb, cc, kind="triad")
    ceiling = {"copy_gbs": round(2 * 8 * n / t_copy / 1e6, 1), "triad_gbs": round(3 * 8 * n / t_triad / 1e6, 1),
               "bytes_per_array": 8 * n}
    del a, bb, cc
    torch.cuda.empty_cache()
    log(f"HBM probe: copy {ceiling['copy_gbs']} GB/s, triad {ceiling['triad_gbs']} GB/s")

    # ---------------------------------------------------------------- headline
    tuned = None
    use_table = args.variant == 0 and not args.pencil and not args.retune and os.path.exists(args.tune_file)
    if use_table:
        lq.tune_load(args.tune_file)
        tuned = table_entry(args.tune_file, 0, DIMS, NRHS, lq.F64, lq.LAYOUT2)
    if args.variant == 0 and not args.pencil and tuned is None:
        tuned = lq.autotune(U64, psi64, eta64, M0, layout=lq.LAYOUT2, reps=3)
    log(f"kernel configuration: {tuned} ({'tune file' if use_table else 'autotuned now'})")

    def step():
        lq.dirac_apply(U64, psi64, M0, layout=lq.LAYOUT2, out=eta64)

    ms = timed(step, args.steps, args.warmup)
    gflops = FLOP_SITE_RHS * v * NRHS / (ms * 1e-3) / 1e9
    alg_bytes = bytes_full(v, NRHS, 16)
    achieved = alg_bytes / (ms * 1e-3) / 1e9
    log(f"D_W FP64 nrhs={NRHS}: {ms:.3f} ms, {gflops:.0f} GFLOP/s, {achieved:.0f} GB/s algorithmic")

    result = {
        "metric": "D_W mrhs apply GFLOP/s & HBM GB/s vs nrhs; mixed vs FP64 GMRES time-to-1e-10",
        "value": round(gflops, 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic: seeded near-identity SU(3) links exp(i 0.3 H), Gaussian spinors",
        "config": {"workload": "wilson_dirac_apply_32x32x32x64_nrhs16_f64", "lattice": list(DIMS),
                   "nrhs": NRHS, "m0": M0, "layout": "rhs-innermost [site][12][nrhs]",
                   "flop_per_site_rhs": FLOP_SITE_RHS},
        "hbm_gbs_algorithmic": round(achieved, 1),
        "measured_hbm_ceiling": ceiling,
        "frac_of_measured_triad": round(achieved / ceiling["triad_gbs"], 4),
        "kernel_config": tuned,
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None},
    }
    if traffic:
        result["roofline"]["traffic"] = traffic["total_bytes"]
        result["traffic_detail"] = dict(traffic, over_algorithmic=round(traffic["total_bytes"] / alg_bytes, 3),
                                        algorithmic_bytes=alg_bytes)
    else:
        result["traffic_detail"] = {"note": traffic_note}

    if args.copy_calibration:
        n = (2 << 30) // 16
        src = torch.ones(n, dtype=torch.complex128, device=dev)
        dst = torch.empty_like(src)
        t_copy = timed(lambda: dst.copy_(src), 3, 1)
        result["copy_calibration"] = {"bytes_read": n * 16, "bytes_written": n * 16, "ms": round(t_copy, 4),
                                      "gbs_read_plus_write": round(2 * n * 16 / t_copy / 1e6, 1)}
        log(f"copy calibration: {t_copy:.3f} ms for 2 GiB")
        del src, dst

    # ------------------------------------------------------------------ sweep
    if not args.no_sweep:
        sweep = []
        half = v // 2
        for prec_name, prec in (("f64", lq.F64), ("f32", lq.F32), ("f16", lq.F16)):
            Up = U64 if prec == lq.F64 else (U64.to(torch.complex64) if prec == lq.F32 else to_f16(U64))
            esz = {lq.F64: 16, lq.F32: 8, lq.F16: 4}[prec]
            for n in (1, 4, 8, 16, 32, 64):
                base = tile_rhs(psi64, n)
                x = base if prec == lq.F64 else (base.to(torch.complex64) if prec == lq.F32 else to_f16(base))
                y = torch.empty_like(x)
                steps = max(5, args.steps // 5)
                if args.variant == 0 and not args.pencil and not use_table:
                    lq.autotune(Up, x, y, M0, layout=lq.LAYOUT2, reps=2)
                t_full = timed(lambda: lq.dirac_apply(Up, x, M0, layout=lq.LAYOUT2, out=y), steps, 2)
                # a half-lattice block of the same rhs count (values do not affect timing)
                xe = x.reshape((v,) + tuple(x.shape[4:]))[:half].contiguous()
                ye = torch.empty_like(xe)
                if args.variant == 0 and not args.pencil and not use_table:
                    lq.autotune(Up, xe, ye, M0, layout=lq.LAYOUT2, eo=True, reps=2)
                wk = torch.empty(lq.dirac_apply_eo_workspace_bytes(DIMS, n, prec), dtype=torch.uint8, device=dev)
                t_eo = timed(lambda: lq.dirac_apply_eo_ws(Up, xe, M0, wk, layout=lq.LAYOUT2, out=ye), steps, 2)
                del wk
                rec = {"prec": prec_name, "nrhs": n,
                       "full_ms": round(t_full, 4),
                       "full_gflops": round(FLOP_SITE_RHS * v * n / t_full / 1e6, 1),
                       "full_gbs": round(bytes_full(v, n, esz) / t_full / 1e6, 1),
                       "schur_ms": round(t_eo, 4),
                       "schur_gflops": round(SCHUR_FLOP_SITE_RHS * half * n / t_eo / 1e6, 1),
                       "schur_gbs_two_pass": round(bytes_schur_two_pass(v, n, esz) / t_eo / 1e6, 1)}
                rec["full_frac_hbm"] = round(rec["full_gbs"] / HBM_PEAK_GBS, 3)
                log(json.dumps(rec))
                sweep.append(rec)
                del x, y, xe, ye, base
            del Up
            torch.cuda.empty_cache()
        result["sweep"] = sweep

    # ------------------------------------------------------------------ GMRES
    if not args.no_gmres:
        result["gmres"] = gmres_section(lq, U64, psi64, args.gmres_nrhs)
        result["gmres_nrhs_sweep"] = gmres_nrhs_sweep(lq, U64, psi64,
                                                      result["gmres"] if args.gmres_nrhs == 16 else None)
    if not args.no_block and args.gmres_nrhs <= lq.BLOCK_MAX_RHS:
        result["block_gmres"] = block_gmres_section(lq, U64, psi64, args.gmres_nrhs,
                                                    None if args.no_gmres else result["gmres"]["f64"])

    # ------------------------------- clover term, uneven batch, differentiation
    if not args.no_clover:
        result["clover"] = clover_section(lq, syn, U64, psi64, max(5, args.steps // 5))
    if not args.no_batch:
        result["batch"] = batch_section(lq, syn, max(5, args.steps // 5))
    if not args.no_autograd:
        result["autograd"] = autograd_section(lq, syn)
    if not args.no_small:
        result["small_workloads"] = small_section(lq, syn, not args.no_cpu)

    # ------------------------------------------------------- oracle baseline
    if not args.no_cpu:
        from oracle import dirac

        nb = 2
        t = time.time()
        dirac.apply_dw(U, psi_np[:nb], M0)
        dt = time.time() - t
        result["cpu_baseline"] = {
            "value": round(FLOP_SITE_RHS * v * nb / dt / 1e9, 3), "unit": "GFLOP/s", "cores": 1, "kind": "oracle",
            "sample": f"{nb} of the 16 rhs of the same 32^3x64 apply (complex128 NumPy, single-threaded), {dt:.1f} s",
            "host_cpus": os.cpu_count()}
        log(f"oracle: {dt:.1f} s for {nb} rhs")

    if args.save_tune:
        lq.tune_save(args.save_tune)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
