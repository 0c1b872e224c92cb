#!/usr/bin/env python3
"""Throughput of the SSPRK3-SE step on one MI355X.

Workload (default): 512 x 512 doubly periodic hexagonal TRiSK mesh (262,144
cells, 786,432 edges), 60 z-star layers, bathymetry 1000 +- 100 m, linear-EOS
density front, SSPRK3-SE with M = 20 barotropic substeps, dt = 300 s, FP64.
Inputs are synthetic and seeded and resident in HBM before timing starts.

Prints ONE JSON line on stdout: cell-layer updates/s over the timed steps,
the roofline of the dominant kernel (algorithmic bytes / HIP-event time of
that kernel in a second timed region) and the FP64 CPU oracle timed on a
bounded sample of the same recipe.  Progress goes to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Algorithmic bytes per cell-layer of a whole SSPRK3-SE step in FP64 with
# every 3D array read once and written once per pass (13 edge-array and 14
# cell-array touches, E = 3C): (13*3 + 14) * 8.
STEP_BYTES_PER_CELL_LAYER = 424.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_bytes(cls, C, E, V, L, launches_by_stage=None):
    """Algorithmic bytes of one launch of a kernel class (FP64, state arrays only)."""
    b = 8.0
    if cls == "fe_edge":
        # X, h, rho, B, w, Z read; out written; u^n read by 2 of the 3 stages
        return b * L * (2 * E + 4 * C + V + (2.0 / 3.0) * E)
    if cls == "fe_cell":
        return b * L * (E + 4 * C)
    if cls == "fe_vertex":
        return b * L * (E + V)
    if cls == "bt_eval":
        return b * (5 * E + 4 * C)
    if cls == "thickness":
        return b * L * C * (3 + 2.0 / 3.0)
    if cls == "other":
        return b * L * (2 * E + C)
    raise KeyError(cls)


def cpu_baseline(n=128, steps=2):
    """The FP64 oracle on the same recipe at n x n cells (same L, M, dt)."""
    os.environ.setdefault("OMP_NUM_THREADS", "1")
    from oracle import ssprk_se
    from oracle.layered import Setup
    from synthetic import cases
    case = cases.c1(n=n, L=60, steps=steps)
    st = Setup.from_case(case)
    u, h = case.u.copy(), case.h.copy()
    t0 = time.perf_counter()
    for _ in range(steps):
        u, h = ssprk_se.step(u, h, st)
    dt = time.perf_counter() - t0
    cl = case.active_cell_layers
    return {"value": cl * steps / dt, "unit": "cell-layer updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} SSPRK3-SE steps of the same recipe on a {n}x{n} hex (C={case.mesh.nCells}, "
                      f"L=60, M=20), NumPy FP64, one thread; {dt:.1f} s",
            "cores_available": len(os.sched_getaffinity(0))}


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=512, help="hex mesh is n x n cells")
    ap.add_argument("--layers", type=int, default=60)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision timing")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the step would shard by horizontal domain decomposition; see the design notes).",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2105_13484_amd import ssprkse
    from synthetic import cases

    torch.cuda.set_device(0)
    log(f"[bench] building C1-recipe inputs n={args.n} L={args.layers}")
    case = cases.c1(n=args.n, L=args.layers)
    C, E, V, L = case.mesh.nCells, case.mesh.nEdges, case.mesh.nVertices, args.layers
    cell_layers = case.active_cell_layers
    dm, st = ssprkse.state_from_case(case, device="cuda:0")
    stream = torch.cuda.current_stream()
    log(f"[bench] uploaded: mesh {dm.nbytes / 1e9:.3f} GB, state {st.nbytes / 1e9:.3f} GB")

    rc = st.step(args.warmup)
    assert rc == 0, f"warmup returned {rc}"

    # per-class timing over a few steps: which kernel class dominates
    st.profile(ssprkse.PROF_CLASSES)
    assert st.step(3) == 0
    prof = st.profile_read()
    st.profile(())
    dom = max(prof, key=lambda k: prof[k][1])
    log(f"[bench] per-class ms over 3 steps: " + ", ".join(f"{k}={v[1]:.3f}({v[0]})" for k, v in prof.items()))

    # timed region 1: clean
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    ev0.record(stream)
    st.step_async(args.steps)
    ev1.record(stream)
    rc = st.sync()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    assert rc == 0, f"timed steps returned {rc}"
    ms_step = ev0.elapsed_time(ev1) / args.steps
    log(f"[bench] {args.steps} steps: {ms_step:.3f} ms/step (events), wall {wall * 1e3 / args.steps:.3f} ms/step")

    # timed region 2: the same steps with HIP events around the dominant kernel only
    st.profile((dom,))
    torch.cuda.synchronize()
    assert st.step(args.steps) == 0
    n_dom, ms_dom = st.profile_read()[dom]
    st.profile(())
    avg_ms = ms_dom / max(n_dom, 1)
    kb = kernel_bytes(dom, C, E, V, L)
    achieved = kb / (avg_ms * 1e-3) / 1e9
    log(f"[bench] dominant kernel {dom}: {n_dom} launches, {avg_ms * 1e3:.1f} us avg, {achieved:.0f} GB/s algorithmic")

    # the same workload in mixed precision (FP32 tendencies and substeps)
    ms_mixed = None
    if not args.no_mixed:
        dm_m, st_m = ssprkse.state_from_case(cases.with_params(case, precision=1), device="cuda:0")
        assert st_m.step(args.warmup) == 0
        torch.cuda.synchronize()
        ev0.record(stream)
        st_m.step_async(args.steps)
        ev1.record(stream)
        assert st_m.sync() == 0
        torch.cuda.synchronize()
        ms_mixed = ev0.elapsed_time(ev1) / args.steps
        log(f"[bench] mixed precision: {ms_mixed:.3f} ms/step")
        del st_m, dm_m

    value = cell_layers / (ms_step * 1e-3)
    step_gbs = STEP_BYTES_PER_CELL_LAYER * cell_layers / (ms_step * 1e-3) / 1e9
    final = st.read()
    assert np.isfinite(final["u"]).all() and np.isfinite(final["h"]).all()

    out = {
        "metric": "cell-layer updates/s per SSPRK3-SE step; % HBM peak; mixed vs FP64 speedup",
        "value": value,
        "unit": "cell-layer updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"C1: SSPRK3-SE on a {args.n}x{args.n} periodic hex TRiSK mesh "
                               f"({C} cells, {E} edges), {L} z-star layers, M=20, dt=300 s, "
                               f"bathymetry + density front, FP64",
                   "cells": C, "edges": E, "layers": L, "substeps": 20, "scheme": "SSPRK3-SE"},
        "hbm_frac_step": step_gbs / HBM_PEAK_GBS,
        "mixed_vs_fp64_speedup": (ms_step / ms_mixed) if ms_mixed else None,
        "mixed_ms_per_step": ms_mixed,
        "per_class_ms_per_step": {k: v[1] / 3.0 for k, v in prof.items()},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "bytes_per_launch": kb},
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
