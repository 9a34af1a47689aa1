#!/usr/bin/env python3
"""Benchmark: matrix-free P1 apply on 288 jittered macro-tets at level 8.

Workload: the 4x4x3 Kuhn box (288 macro-tetrahedra, interior macro-vertices
jittered by U[-0.1, 0.1]^3, seed 3) refined to level 8: 802,687,743 interior
DoFs.  One step = one FP64 operator application y = A x (cell stencil kernel
+ ghost exchange), inputs resident in HBM.  Also reported: per-kernel device
time and HBM roofline of the dominant kernel, FP32 apply, time to a 1e-10
relative residual for FP64 V(2,2) cycles and for FP32-in-FP64 iterative
refinement, and the CPU oracle's assembled sparse apply timed on the host.

Prints exactly one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_DOF_F64 = 16.0   # read x, write y per interior DoF
BYTES_PER_DOF_F32 = 8.0
# div(k grad): read x and k, write y per interior DoF
DIVKGRAD_BYTES_PER_DOF = {"f64": 24.0, "f32": 12.0}
# per point: 24 micro-cells x (3-term coupling sum, 5 flops; coefficient
# sum, 3; scaled accumulate, 2) + 14 neighbour differences
DIVKGRAD_FLOPS_PER_DOF = 24 * 10 + 14
# stored rows: read 15 entries and x, write y per interior DoF
STORED_BYTES_PER_DOF = {"f64": 17 * 8.0, "f32": 17 * 4.0}
# P2 apply at P2 level L - 1 (its nodes are the level-L micro-vertices): read
# x, write y per DoF; 230 stencil entries over the 8 node parities, i.e.
# 28.75 multiply-adds per DoF on average.
P2_BYTES_PER_DOF = {"f64": 16.0, "f32": 8.0}
P2_FLOPS_PER_DOF = 2 * 230 / 8
FP64_PEAK_TFLOPS, FP32_PEAK_TFLOPS = 78.6, 157.3


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--level", type=int, default=8)
    p.add_argument("--no-solve", action="store_true")
    p.add_argument("--no-cpu", action="store_true")
    p.add_argument("--cpu-level", type=int, default=5)
    p.add_argument("--cpu-seconds", type=float, default=15.0)
    p.add_argument("--no-batch", action="store_true")
    p.add_argument("--batch-only-solves", action="store_true",
                   help="batch leg: only two batched FP32-in-FP64 solves "
                        "(warm-up, then timed), no loop and no tuning; for a "
                        "kernel trace of one batched solve")
    p.add_argument("--no-divkgrad", action="store_true")
    p.add_argument("--no-stored", action="store_true")
    p.add_argument("--no-p2", action="store_true")
    p.add_argument("--copy-calibration", action="store_true",
                   help="also run 3 plain device copies of one level vector "
                        "(counter calibration for rocprofv3 --pmc)")
    return p.parse_args()


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE + WRITE_SIZE, copy-calibrated), or None when the
    kernel sources changed since the counters were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "band_apply_box288_l8_traffic.json")
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    h = hashlib.sha256()
    for f in ("kernels.hip", "kernels.hpp", "device.hpp", "band.hip", "band.hpp"):
        with open(os.path.join(ROOT, "paper_2308_01792_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if rec.get("sources_sha256") != h.hexdigest() or rec.get("kernel") != kernel:
        return None
    return float(rec["hbm_bytes_per_launch"])


def batch_leg(ht, torch, only_solves=False):
    """256 independent small problems (1-24 cells, levels 3-6): one batched
    solve to 1e-10 against a loop of per-problem solves (both after a
    warm-up run that captures graphs and builds the coarse solvers)."""
    from workloads import batch_problems
    probs = batch_problems(count=256, seed=6, min_level=3, max_level=6)
    meshes = [ht.Mesh(p.xyz, p.cells, 2, p.level) for p in probs]
    bs = []
    for m, p in zip(meshes, probs):
        g = torch.Generator(device="cuda").manual_seed(1000 + p.index)
        f = torch.rand(m.n_slots(p.level), dtype=torch.float64, device="cuda",
                       generator=g) * 2 - 1
        m.sync(p.level, f)
        mass = torch.zeros_like(f)
        m.lumped_mass(p.level, mass)
        bs.append(mass * f)
    t0 = time.time()
    batch = ht.Batch(meshes, [p.level for p in probs])
    create_s = time.time() - t0
    info = batch.info()

    def run_batch(prec):
        us = [torch.zeros_like(b) for b in bs]
        torch.cuda.synchronize()
        st = batch.solve(us, bs, rel_tol=1e-10, max_cycles=100, precision=prec)
        return us, st

    def run_loop(prec):
        us = [torch.zeros_like(b) for b in bs]
        torch.cuda.synchronize()
        t1 = time.time()
        st = [m.solve(p.level, u, b, prec, 1e-10, 100)
              for m, p, u, b in zip(meshes, probs, us, bs)]
        torch.cuda.synchronize()
        return us, st, time.time() - t1

    if only_solves:
        run_batch(ht.HT_PREC_MIXED)
        _, stb = run_batch(ht.HT_PREC_MIXED)
        return {"problems": info["problems"], "cells": info["cells"],
                "dofs": info["dofs"], "mixed_batch_seconds": round(stb[0]["seconds"], 4),
                "cycles_max": max(x["cycles"] for x in stb)}
    out = {"workload": "256 problems (Kuhn boxes <= 4 cubes, jittered slabs; "
                       "levels 3-6; seed 6), V(2,2) to 1e-10: FP32-in-FP64 "
                       "refinement and FP64",
           "problems": info["problems"], "cells": info["cells"],
           "dofs": info["dofs"], "create_seconds": round(create_s, 3)}
    for name, prec in (("mixed", ht.HT_PREC_MIXED), ("f64", ht.HT_PREC_F64)):
        run_batch(prec)
        ub, stb = run_batch(prec)
        run_loop(prec)
        ul, stl, loop_s = run_loop(prec)
        batch_s = stb[0]["seconds"]
        diff = max(float((a - b).abs().max() / b.abs().max())
                   for a, b in zip(ub, ul))
        out[name] = {"batch_seconds": round(batch_s, 4),
                     "loop_seconds": round(loop_s, 4),
                     "speedup_vs_loop": round(loop_s / batch_s, 2),
                     "solves_per_s": round(info["problems"] / batch_s, 1),
                     "gdofs_solved_per_s": round(info["dofs"] / batch_s / 1e9, 4),
                     "cycles_max": max(x["cycles"] for x in stb),
                     "cycles_equal_to_loop": sum(a["cycles"] == b["cycles"]
                                                 for a, b in zip(stb, stl)),
                     "max_rel_diff_vs_loop": diff}
        del ub, ul
    # the union mesh tuned level by level on the problems present there
    # (apply kernel, sweep rows, arrangement, march segment), then the same
    # batched solves again
    torch.cuda.synchronize()
    t0 = time.time()
    batch.autotune()
    torch.cuda.synchronize()
    out["autotune_seconds"] = round(time.time() - t0, 2)
    out["tuned_shapes"] = batch.shapes(range(3, 7))
    for name, prec in (("mixed", ht.HT_PREC_MIXED), ("f64", ht.HT_PREC_F64)):
        run_batch(prec)
        ub, stb = run_batch(prec)
        out[name]["tuned_batch_seconds"] = round(stb[0]["seconds"], 4)
        out[name]["tuned_cycles_max"] = max(x["cycles"] for x in stb)
        del ub
    return out


def divkgrad_leg(mesh, L, x, ndof, args, stream):
    """Element-wise div(k grad) apply at the headline size, FP64 and FP32,
    with k = 1 + sin(2 pi x) sin(2 pi y) sin(2 pi z) / 2 evaluated at the
    slot coordinates."""
    import math
    import torch
    xyz = torch.empty((x.numel(), 3), dtype=torch.float64, device=x.device)
    mesh.coords_device(L, xyz)
    w = 2.0 * math.pi
    kap = 1.0 + 0.5 * (torch.sin(w * xyz[:, 0]) * torch.sin(w * xyz[:, 1]) *
                       torch.sin(w * xyz[:, 2]))
    del xyz
    res = {}
    for name, dt in (("f64", torch.float64), ("f32", torch.float32)):
        k_, x_ = kap.to(dt), x.to(dt)
        y_ = torch.zeros_like(x_)
        for _ in range(args.warmup):
            mesh.apply_divkgrad(L, k_, x_, y_)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            mesh.apply_divkgrad(L, k_, x_, y_)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        mesh.profile(True)
        mesh.profile_reset()
        for _ in range(args.steps):
            mesh.apply_divkgrad(L, k_, x_, y_)
        torch.cuda.synchronize()
        cms, cn = mesh.profile_query("cell_divkgrad")
        mesh.profile(False)
        cell = cms / cn
        gbs = DIVKGRAD_BYTES_PER_DOF[name] * ndof / (cell * 1e-3) / 1e9
        tfl = DIVKGRAD_FLOPS_PER_DOF * ndof / (cell * 1e-3) / 1e12
        peak = FP64_PEAK_TFLOPS if name == "f64" else FP32_PEAK_TFLOPS
        res[name] = {"ms": round(ms, 4), "gdofs": round(ndof / (ms * 1e-3) / 1e9, 3),
                     "cell_kernel_ms": round(cell, 4),
                     "algorithmic_gbs": round(gbs, 1),
                     "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                     "tflops": round(tfl, 2),
                     "valu_frac": round(tfl / peak, 4)}
        log(f"div(k grad) apply {name}: {ms:.3f} ms/step "
            f"({res[name]['gdofs']:.1f} GDoF/s), cell kernel {cell:.3f} ms, "
            f"{gbs:.0f} GB/s, {tfl:.1f} TFLOP/s")
        if not args.no_stored:
            # the same operator from rows stored in the iteration order
            y2 = torch.zeros_like(x_)
            t0 = time.time()
            rows = mesh.assemble_divkgrad(L, k_)
            torch.cuda.synchronize()
            t_asm = time.time() - t0
            for _ in range(args.warmup):
                mesh.apply_stored(L, rows, x_, y2)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(args.steps):
                mesh.apply_stored(L, rows, x_, y2)
            e1.record(stream)
            torch.cuda.synchronize()
            ms2 = e0.elapsed_time(e1) / args.steps
            mesh.profile(True)
            mesh.profile_reset()
            for _ in range(args.steps):
                mesh.apply_stored(L, rows, x_, y2)
            torch.cuda.synchronize()
            sms, sn = mesh.profile_query("cell_stored")
            mesh.profile(False)
            diff = float((y2 - y_).abs().max()) / float(y_.abs().max())
            gbs2 = STORED_BYTES_PER_DOF[name] * ndof / (sms / sn * 1e-3) / 1e9
            res[name]["stored"] = {
                "ms": round(ms2, 4), "gdofs": round(ndof / (ms2 * 1e-3) / 1e9, 3),
                "cell_kernel_ms": round(sms / sn, 4),
                "algorithmic_gbs": round(gbs2, 1),
                "hbm_frac": round(gbs2 / HBM_PEAK_GBS, 4),
                "rows_bytes": rows.numel() * rows.element_size(),
                "assemble_seconds": round(t_asm, 3),
                "max_rel_diff_vs_matrix_free": diff}
            log(f"stored rows {name}: {ms2:.3f} ms/step, {gbs2:.0f} GB/s, "
                f"rows {rows.numel() * rows.element_size() / 1e9:.1f} GB, "
                f"rel diff vs matrix-free {diff:.1e}")
            del rows, y2
        del k_, x_, y_
    del kap
    return res


def cpu_baseline(level: int, budget_s: float):
    """The oracle on the host: its assembled CSR matrix of the same mesh at a
    level the host can assemble, applied (a) with the threaded C product on
    every CPU this process may use (the reported value) and (b) with SciPy on
    one core; and (c) its V(2,2) solve to a 1e-10 relative residual over
    levels 2..level.  GDoF/s over interior DoFs."""
    import numpy as np
    from oracle import spmv
    from oracle.mg import Hierarchy
    from workloads import jittered_kuhn_box, uniform_values
    mesh_args = jittered_kuhn_box(4, 4, 3, 0.1, 3)
    t0 = time.time()
    H = Hierarchy(*mesh_args, max_level=level, min_level=2)
    S = H[level]
    setup = time.time() - t0
    x = uniform_values(S.mesh.num_vertices, 4)
    x[S.dirichlet] = 0.0
    dofs = int(S.interior.sum())

    def rate(apply_once, seconds):
        apply_once()
        reps, t1 = 0, time.time()
        while True:
            apply_once()
            reps += 1
            el = time.time() - t1
            if el >= seconds:
                return reps, el

    threads = spmv.host_threads()
    csr = spmv.CSR(S.A)
    y = np.empty(S.A.shape[0])
    reps_mt, el_mt = rate(lambda: csr.apply(x, y, threads), budget_s / 3)
    assert np.allclose(y, S.A @ x, rtol=0, atol=1e-12 * np.abs(y).max())
    reps_1, el_1 = rate(lambda: S.apply(x), budget_s / 3)
    # V(2,2) to 1e-10 from u0 = 0, b = m * f (f ~ U[-1, 1], seed 5)
    b = S.lumped_mass * uniform_values(S.mesh.num_vertices, 5)
    H.coarse_solve(2, np.zeros(H[2].mesh.num_vertices),
                   np.zeros(H[2].mesh.num_vertices))      # factor once
    t1 = time.time()
    _, hist = H.solve(level, b, rel_tol=1e-10, max_cycles=60, coarse_level=2)
    solve_s = time.time() - t1
    return {"value": round(dofs * reps_mt / el_mt / 1e9, 6), "unit": "GDoF/s",
            "cores": threads, "kind": "oracle",
            "cpu_model": spmv.cpu_model(),
            "host_cpus": os.cpu_count(),
            "sample": f"288-cell jittered mesh at level {level} ({dofs} interior "
                      f"DoFs, CSR nnz {S.A.nnz}) assembled element by element "
                      f"with levels 2..{level} and transfers ({setup:.1f} s, "
                      f"untimed); threaded C CSR apply on "
                      f"{threads} threads: {reps_mt} reps in {el_mt:.1f} s",
            "single_core": {"value": round(dofs * reps_1 / el_1 / 1e9, 6),
                            "unit": "GDoF/s", "cores": 1,
                            "sample": f"SciPy CSR apply, {reps_1} reps in {el_1:.1f} s"},
            "vcycle_to_1e-10": {"seconds": round(solve_s, 3),
                                "cycles": len(hist) - 1,
                                "rel_res": hist[-1], "levels": f"2..{level}",
                                "sample": "oracle V(2,2) with SciPy sparse "
                                          "products and a Cholesky coarse "
                                          "solve, b = m * f (f ~ U[-1, 1], seed 5)"}}


def p2_leg(mesh, L, x, ndof, args, stream):
    """P2 apply at P2 level L - 1 on the same mesh: its nodes are the level-L
    micro-vertices, so the vectors and the DoF count are those of level L.
    Bulk kernel (rows' inner points), face kernel (points on the faces
    i = 0 and i = n - j - k) and exchange, FP64 and FP32."""
    import torch
    res = {"p2_level": L - 1}
    for name, dt in (("f64", torch.float64), ("f32", torch.float32)):
        x_ = x.to(dt)
        y_ = torch.zeros_like(x_)
        for _ in range(args.warmup):
            mesh.apply_p2(L - 1, x_, y_)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(args.steps):
            mesh.apply_p2(L - 1, x_, y_)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / args.steps
        mesh.profile(True)
        mesh.profile_reset()
        for _ in range(args.steps):
            mesh.apply_p2(L - 1, x_, y_)
        torch.cuda.synchronize()
        kern = {k: mesh.profile_query(k) for k in ("cell_p2", "face_p2", "exchange")}
        mesh.profile(False)
        kern = {k: v[0] / v[1] for k, v in kern.items() if v[1] > 0}
        gbs = P2_BYTES_PER_DOF[name] * ndof / (ms * 1e-3) / 1e9
        res[name] = {"ms": round(ms, 4), "gdofs": round(ndof / (ms * 1e-3) / 1e9, 3),
                     "kernel_ms": {k: round(v, 4) for k, v in kern.items()},
                     "algorithmic_gbs": round(gbs, 1),
                     "hbm_frac": round(gbs / HBM_PEAK_GBS, 4),
                     "tflops": round(P2_FLOPS_PER_DOF * ndof / (ms * 1e-3) / 1e12, 2)}
        log(f"P2 apply {name} (P2 level {L - 1}): {ms:.3f} ms/step "
            f"({res[name]['gdofs']:.1f} GDoF/s, {gbs:.0f} GB/s), kernels " +
            ", ".join(f"{k} {v:.3f} ms" for k, v in kern.items()))
        del x_, y_
    return res


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU "
              "path (the design notes describe how it would shard); run with --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2308_01792_amd as ht
    from workloads import jittered_kuhn_box

    L = args.level
    log(f"mesh setup (levels 2..{L})")
    xyz, cells = jittered_kuhn_box(4, 4, 3, amplitude=0.1, seed=3)
    mesh = ht.Mesh(xyz, cells, 2, L)
    info = mesh.info(L)
    ndof, nslot = info["n_dofs"], info["n_slots"]
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    gen = torch.Generator(device=dev).manual_seed(4)
    x = torch.rand(nslot, dtype=torch.float64, device=dev, generator=gen) * 2 - 1
    mesh.sync(L, x)
    mesh.fill_dirichlet(L, x, 0.0)
    y = torch.zeros_like(x)
    torch.cuda.synchronize()
    t0 = time.time()
    rows64 = mesh.autotune(L, ht.HT_F64)
    rows32 = mesh.autotune(L, ht.HT_F32)
    log(f"autotuned tile rows: f64 {rows64}, f32 {rows32} "
        f"({time.time() - t0:.1f} s)")

    # ---------------- headline: FP64 apply -------------------------------
    log(f"FP64 apply: {args.warmup} warmup + {args.steps} timed steps, "
        f"{ndof} DoFs")
    for _ in range(args.warmup):
        mesh.apply(L, x, y)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        mesh.apply(L, x, y)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    gdofs = ndof / (ms * 1e-3) / 1e9
    log(f"apply: {ms:.3f} ms/step, {gdofs:.1f} GDoF/s")

    # per-kernel device time (HIP events around every library launch, on
    # the launch stream)
    mesh.profile(True)
    mesh.profile_reset()
    for _ in range(args.steps):
        mesh.apply(L, x, y)
    torch.cuda.synchronize()
    cell_ms, ncell = mesh.profile_query("cell_apply")
    exch_ms, nexch = mesh.profile_query("exchange")
    mesh.profile(False)
    cell_avg, exch_avg = cell_ms / ncell, exch_ms / nexch
    achieved = BYTES_PER_DOF_F64 * ndof / (cell_avg * 1e-3) / 1e9
    log(f"cell kernel {cell_avg:.3f} ms ({achieved:.0f} GB/s algorithmic), "
        f"exchange {exch_avg:.3f} ms")

    # streaming-copy reference: one level vector read + written (known bytes)
    copy_bytes = 2 * nslot * 8
    reps = 3 if args.copy_calibration else 10
    mesh.copy(L, x, y)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        mesh.copy(L, x, y)
    e1.record(stream)
    torch.cuda.synchronize()
    copy_ms = e0.elapsed_time(e1) / reps
    copy_gbs = copy_bytes / (copy_ms * 1e-3) / 1e9
    log(f"plain copy of {nslot * 8} B: {copy_ms:.3f} ms, {copy_gbs:.0f} GB/s")

    # ---------------- FP32 apply ------------------------------------------
    x32, y32 = x.float(), torch.zeros(nslot, dtype=torch.float32, device=dev)
    for _ in range(args.warmup):
        mesh.apply(L, x32, y32)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(args.steps):
        mesh.apply(L, x32, y32)
    e1.record(stream)
    torch.cuda.synchronize()
    ms32 = e0.elapsed_time(e1) / args.steps
    del x32, y32

    # tile rows 0 selects the band kernel (LDS-staged planes)
    kname = "k_band<double, 0>" if rows64 == 0 else f"k_cell<double, 0, {rows64}>"
    traffic = measured_traffic(kname)
    out = {
        "metric": "GDoF/s of matrix-free P1 apply + %HBM roofline; V-cycle "
                  "time to 1e-10 FP32/FP64",
        "value": round(gdofs, 3),
        "unit": "GDoF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"288 jittered macro-tets (4x4x3 Kuhn box, "
                               f"seed 3) at level {L}, FP64 apply",
                   "level": L, "macro_cells": 288, "dofs": ndof,
                   "slots": nslot},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic,
                     "kernel": kname,
                     "bytes_per_launch": BYTES_PER_DOF_F64 * ndof},
        "apply_hbm_frac": round(gdofs * BYTES_PER_DOF_F64 / HBM_PEAK_GBS, 4),
        "stream_copy": {"ms": round(copy_ms, 4), "gbs": round(copy_gbs, 1),
                        "bytes": copy_bytes, "kernel": "k_flat<double, double, copy>"},
        "tile_rows": {"f64": rows64, "f32": rows32},
        "sweep_shape": {name: dict(zip(("rows", "waves_in_i"), mesh.sweep_shape(L, code)))
                        for name, code in (("f64", ht.HT_F64), ("f32", ht.HT_F32))},
        "kernel_ms": {"cell_apply": round(cell_avg, 4),
                      "exchange": round(exch_avg, 4)},
        "apply_f32": {"ms": round(ms32, 4),
                      "gdofs": round(ndof / (ms32 * 1e-3) / 1e9, 3),
                      "hbm_frac": round(ndof * BYTES_PER_DOF_F32 / (ms32 * 1e-3)
                                        / 1e9 / HBM_PEAK_GBS, 4)},
    }

    # ---------------- variable coefficient: div(k grad) apply -------------
    if not args.no_divkgrad:
        out["divkgrad_apply"] = divkgrad_leg(mesh, L, x, ndof, args, stream)

    # ---------------- P2: vertex + edge DoFs ------------------------------
    if not args.no_p2:
        out["p2_apply"] = p2_leg(mesh, L, x, ndof, args, stream)

    # ---------------- solves to 1e-10 --------------------------------------
    if not args.no_solve:
        del y
        m = torch.zeros_like(x)
        mesh.lumped_mass(L, m)
        f = torch.rand(nslot, dtype=torch.float64, device=dev,
                       generator=torch.Generator(device=dev).manual_seed(5)) * 2 - 1
        mesh.sync(L, f)
        b = m * f
        del m, f, x
        solves = {}
        for name, prec in (("f64", ht.HT_PREC_F64), ("mixed", ht.HT_PREC_MIXED)):
            u = torch.zeros_like(b)
            mesh.solve(L, u, b, prec, 1e-10, 100, use_graph=True)   # warm-up
            u.zero_()
            torch.cuda.synchronize()
            st = mesh.solve(L, u, b, prec, 1e-10, 100, use_graph=True)
            solves[name] = {"seconds": round(st["seconds"], 4),
                            "cycles": st["cycles"],
                            "rel_res": st["rel_res"]}
            if name == "f64":
                u64 = u
            else:
                diff = u - u64
                solves[name]["rel_diff_vs_f64"] = mesh.norm(L, diff) / mesh.norm(L, u64)
            log(f"solve {name}: {st['cycles']} cycles, {st['seconds']:.3f} s, "
                f"rel res {st['rel_res']:.2e}")
        # Chebyshev-accelerated Jacobi (degree 2): V(1,1) makes as many
        # stencil passes per level as the Jacobi V(2,2)
        uc = torch.zeros_like(b)
        mesh.solve(L, uc, b, ht.HT_PREC_F64, 1e-10, 100, nu1=1, nu2=1,
                   smoother=ht.HT_SMOOTH_CHEBYSHEV, degree=2)
        uc.zero_()
        torch.cuda.synchronize()
        st = mesh.solve(L, uc, b, ht.HT_PREC_F64, 1e-10, 100, nu1=1, nu2=1,
                        smoother=ht.HT_SMOOTH_CHEBYSHEV, degree=2)
        solves["f64_chebyshev_v11_deg2"] = {
            "seconds": round(st["seconds"], 4), "cycles": st["cycles"],
            "rel_res": st["rel_res"],
            "rel_diff_vs_f64": mesh.norm(L, uc - u64) / mesh.norm(L, u64),
            "lambda_max_estimate": mesh.lambda_max(L)}
        log(f"solve f64 Chebyshev V(1,1) deg 2: {st['cycles']} cycles, "
            f"{st['seconds']:.3f} s")
        del uc
        # full multigrid: nested iteration with 5 V(2,2) per level, no
        # residual tolerance (first call captures the graph)
        fmg = {}
        for cyc in (2, 5):
            uf = torch.zeros_like(b)
            mesh.fmg(L, uf, b, cycles=cyc, want_residual=False)
            torch.cuda.synchronize()
            t1 = time.time()
            mesh.fmg(L, uf, b, cycles=cyc, want_residual=False)
            torch.cuda.synchronize()
            secs = time.time() - t1
            rel = mesh.fmg(L, uf, b, cycles=cyc)
            fmg[f"v22_x{cyc}"] = {
                "seconds": round(secs, 4), "rel_res": rel,
                "rel_diff_vs_solve_1e-10": mesh.norm(L, uf - u64) / mesh.norm(L, u64)}
            log(f"FMG {cyc} x V(2,2) per level: {secs:.3f} s, rel res {rel:.2e}")
            del uf
        solves["fmg"] = fmg
        # per-kernel device time of one eager FP64 and one mixed solve
        breakdown = {}
        for name, prec in (("f64", ht.HT_PREC_F64), ("mixed", ht.HT_PREC_MIXED)):
            u = torch.zeros_like(b)
            mesh.profile(True)
            mesh.profile_reset()
            mesh.solve(L, u, b, prec, 1e-10, 100, use_graph=False)
            parts = {}
            for kname in ("cell_apply", "cell_residual", "cell_jacobi", "exchange",
                          "restrict", "prolongate", "zero_guess", "coarse_solve",
                          "flat", "norm_sum", "dot"):
                ms_k, cnt = mesh.profile_query(kname)
                if cnt:
                    parts[kname] = {"ms": round(ms_k, 2), "launches": cnt}
            mesh.profile(False)
            breakdown[name] = parts
        log(f"solve kernel breakdown: {json.dumps(breakdown)}")
        solves["kernel_ms"] = breakdown
        out["solve_to_1e-10"] = solves

    if not args.no_batch:
        log("batched solves of 256 small problems")
        out["batch"] = batch_leg(ht, torch, args.batch_only_solves)
        log(f"batch: {json.dumps(out['batch'])}")

    if not args.no_cpu:
        log(f"CPU oracle baseline at level {args.cpu_level}")
        out["cpu_baseline"] = cpu_baseline(args.cpu_level, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
