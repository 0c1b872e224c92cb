#!/usr/bin/env python3
"""Throughput of the SSPRK3-SE step on one MI355X.

Workload (the headline line): 512 x 512 doubly periodic hexagonal TRiSK mesh
(262,144 cells, 786,432 edges), 60 z-star layers, bathymetry 1000 +- 100 m,
linear-EOS density front, SSPRK3-SE with M = 20 barotropic substeps,
dt = 300 s, FP64.  Inputs are synthetic and seeded and resident in HBM before
timing starts.

Prints ONE JSON line on stdout: cell-layer updates/s over the timed steps,
the roofline of the dominant kernel class (algorithmic bytes / HIP-event time
of that class in a second timed region), the same workload in mixed
precision, with implicit vertical mixing, with biharmonic viscosity and with an evolving
temperature tracer, the runtime to a fixed simulated time as the number of substeps
M varies (both schemes), the level-7 sphere (C2 recipe) in FP64 and mixed
precision, a batched ensemble, a served request stream, and the FP64 CPU
oracle timed on a bounded sample of the headline recipe.
Progress goes to stderr.

--copy-probe runs only a plain device copy of a known size (for scaling the
FETCH_SIZE / WRITE_SIZE counters of a rocprofv3 run) and exits.
"""
import argparse
import collections
import hashlib
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
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic.json")
# the sources the kernels are compiled from (the argument blocks and tables
# in the headers shape the code as well)
KERNEL_SOURCES = [os.path.join(ROOT, "paper_2105_13484_amd", "csrc", f)
                  for f in ("sse_kernels.hip", "sse_kernels.h", "sse_internal.h")]
COPY_PROBE_BYTES = 1 << 30


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_bytes(cls, C, E, V, L, b=8.0, bt_tiled=True):
    """Algorithmic bytes of one launch of a kernel class (state arrays only,
    each read once and written once; mesh tables excluded).  The barotropic
    class launches once per substep (bt_tiled, the default) or once per
    evaluation."""
    if cls == "fe_edge":
        # the forward-Euler passes at ideal fusion, averaged over the three
        # stages of SSPRK3-SE: FE1 reads u^n, h, rho and writes the stage
        # (2 edge and 2 cell touches); FE2 and FE3 also read u^n for the stage
        # combination (3 edge, 2 cell touches)
        return b * L * ((8.0 / 3.0) * E + 2 * C)
    if cls == "fe_cell":
        return b * L * (E + 4 * C)          # X, h, frac read; B, w written
    if cls == "fe_vertex":
        return b * L * (E + V)              # X read; Z written
    if cls == "bt_eval":
        if bt_tiled:
            # one whole substep: edges ubar in, G, F read; ubar out, F written;
            # cells zeta in read, zeta out written (the stages stay on chip)
            return b * (5 * E + 2 * C)
        # one evaluation: edges stage input, combination base, G, F read;
        # output, F written; cells stage input, base read, output written
        return b * (6 * E + 3 * C)
    if cls == "thickness":
        return b * L * C * (3 + 2.0 / 3.0)  # h_in, frac, h_out (+ h^n in 2 of 3)
    if cls == "other":
        return b * L * (2 * E + C)          # assembly: X read, u written, h read
    raise KeyError(cls)


def intermediate_bytes(cls, C, E, V, L, b=8.0):
    """Bytes a launch moves beyond the ideal-fusion count: for the edge pass
    the intermediates that the cell and vertex passes write for it (K - nu
    div u and w at cells, the relative vorticity at vertices), read back."""
    if cls == "fe_edge":
        return b * L * (2 * C + V)
    return 0.0


def copy_bandwidth(torch, nbytes=1 << 30, reps=10):
    """Achievable HBM bandwidth of a plain device copy (bytes read + written
    per second), HIP events around `reps` copies of `nbytes`."""
    a = torch.ones(nbytes // 8, dtype=torch.float64, device="cuda:0")
    bb = torch.empty_like(a)
    bb.copy_(a)
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(reps):
        bb.copy_(a)
    ev1.record(stream)
    torch.cuda.synchronize()
    s = ev0.elapsed_time(ev1) * 1e-3 / reps
    del a, bb
    return 2.0 * nbytes / s / 1e9


def kernel_source_sha256():
    """SHA-256 over the kernel sources, in order."""
    h = hashlib.sha256()
    for path in KERNEL_SOURCES:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def measured_traffic(dom):
    """HBM bytes per launch of the dominant class from the committed rocprofv3
    counter summary, or None when it is missing, covers another kernel class
    or was taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    c = t.get("classes", {}).get(dom)
    if c is None or t.get("kernel_source_sha256") != kernel_source_sha256():
        return None
    return float(c["fetch_bytes_per_launch"]) + float(c["write_bytes_per_launch"])


def cpu_baseline(n=128, steps=4):
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
                      f"L=60, M=20), NumPy FP64, one thread; {dt:.1f} s (one oracle step of the 512x512 mesh "
                      f"takes ~270 s on one core, ~5x slower per cell-layer than this sample: too long "
                      f"for this run, and this sample flatters the CPU)",
            "cores_available": len(os.sched_getaffinity(0))}


def gather_only(torch, st, E, L, reps=10):
    """The direct edge pass's 30 column gathers per edge without its
    arithmetic (sse_debug_edge_gathers), timed with HIP events on the state's
    stream: the time its memory accesses alone take at its access pattern."""
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    st.debug_edge_gathers()
    torch.cuda.synchronize()
    ev0.record(stream)
    for _ in range(reps):
        st.debug_edge_gathers()
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    rs = 8 if int(st.params.precision) == 0 else 4
    # u, u^n, K - nu div u, w, the 10 stencil edges and 10 vertices in the
    # state's real type; h and rho at both cells in FP64
    nbytes = float(E) * L * (26 * rs + 4 * 8)
    return {"gather_only_launch_ms": ms, "columns_gathered_per_edge": 30,
            "gathered_bytes_per_launch": nbytes, "gathered_gbs": nbytes / (ms * 1e-3) / 1e9}


def timed_steps(torch, st, steps):
    """ms per step of `steps` steps, HIP events on the state's stream."""
    stream = torch.cuda.current_stream()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record(stream)
    st.step_async(steps)
    ev1.record(stream)
    rc = st.sync()
    torch.cuda.synchronize()
    assert rc == 0, f"timed steps returned {rc}"
    return ev0.elapsed_time(ev1) / steps


def m_sweep_leg(torch, ssprkse, dm, case, T=1920.0, dt_btr=15.0, ms=(1, 2, 4, 8, 16, 32)):
    """Runtime to a fixed simulated time T at a fixed barotropic step dt_btr
    as the number of substeps M varies (dt = M dt_btr, T / dt steps), for
    both schemes on the same mesh and initial state (the cost study of
    Sec. 5: T = 1920 s, dt_btr = 15 s, M = 1 .. 32).  When the 3D work
    dominates, runtime falls like 1/M, and the SSPRK3-SE / SSPRK2-SE cost
    per step sits between 1.5 (3D-dominated) and 2.25 (2D-dominated)."""
    import math
    from dataclasses import replace
    rows = []
    for scheme in (3, 2):
        for M in ms:
            steps = int(round(T / (M * dt_btr)))
            p = replace(case.params, scheme=scheme, substeps=M, dt=M * dt_btr)
            st = ssprkse.DeviceState(dm, p, device="cuda:0")
            st.init(case.h, case.u, case.rho, case.h_ref)
            assert st.step(1) == 0
            st.init(case.h, case.u, case.rho, case.h_ref)
            ms_step = timed_steps(torch, st, steps)
            rows.append({"scheme": scheme, "M": M, "dt": M * dt_btr, "steps": steps,
                         "ms_per_step": ms_step, "runtime_ms": ms_step * steps})
            log(f"[bench] M sweep: SSPRK{scheme}-SE M={M:2d} dt={M * dt_btr:.0f} s: "
                f"{steps:3d} steps x {ms_step:.3f} ms = {ms_step * steps:.1f} ms")
            st.close()
            del st
    out = {"T_s": T, "dt_btr_s": dt_btr, "rows": rows}
    for scheme in (3, 2):
        r = [x for x in rows if x["scheme"] == scheme]
        # least-squares slope of log(runtime) against log(M)
        xs = [math.log(x["M"]) for x in r]
        ys = [math.log(x["runtime_ms"]) for x in r]
        mx, my = sum(xs) / len(xs), sum(ys) / len(ys)
        out[f"ssprk{scheme}_loglog_slope"] = (sum((a - mx) * (b - my) for a, b in zip(xs, ys))
                                              / sum((a - mx) ** 2 for a in xs))
    out["ssprk3_over_ssprk2_per_step"] = {
        str(M): next(x["ms_per_step"] for x in rows if x["scheme"] == 3 and x["M"] == M)
        / next(x["ms_per_step"] for x in rows if x["scheme"] == 2 and x["M"] == M) for M in ms}
    log(f"[bench] M sweep slopes: SSPRK3-SE {out['ssprk3_loglog_slope']:.3f}, "
        f"SSPRK2-SE {out['ssprk2_loglog_slope']:.3f}; cost ratio per step "
        + ", ".join(f"M={k}: {v:.2f}" for k, v in out["ssprk3_over_ssprk2_per_step"].items()))
    return out


def ensemble_leg(torch, ssprkse, cases, members=64, steps=10):
    """C3: a 64-member ensemble of uneven planar members in mixed precision,
    per-member loop vs one batch (autotuned launch geometry, HIP graph)."""
    from paper_2105_13484_amd import autotune
    stream = torch.cuda.Stream()
    log(f"[bench] ensemble: building {members} members")
    cs = [cases.c3_member(i) for i in range(members)]
    keep = [ssprkse.state_from_case(c, device="cuda:0", stream=stream) for c in cs]
    sts = [st for _, st in keep]
    cl = sum(c.active_cell_layers for c in cs)

    def loop(n):
        for _ in range(n):
            for st in sts:
                st.step_async(1)

    def reinit():
        # every timed section starts from the initial state: some members
        # (strong fronts on small domains) run close to their stability limit
        # and would otherwise accumulate the steps of all sections
        for c, st in zip(cs, sts):
            st.init(c.h, c.u, c.rho, c.h_ref)

    for st in sts:
        assert st.step(1) == 0
    ms_loop = autotune._time_steps(torch, stream, loop, steps)
    reinit()
    log(f"[bench] ensemble per-member loop: {ms_loop:.2f} ms/step")

    # the plain method: the same members in FP64, one after the other
    keep64 = [ssprkse.state_from_case(cases.with_params(c, precision=0), device="cuda:0", stream=stream) for c in cs]
    sts64 = [st for _, st in keep64]

    def loop64(n):
        for _ in range(n):
            for st in sts64:
                st.step_async(1)

    for st in sts64:
        assert st.step(1) == 0
    ms_loop64 = autotune._time_steps(torch, stream, loop64, steps)
    for dm, st in keep64:
        st.close()
        dm.close()
    del keep64, sts64
    log(f"[bench] ensemble per-member loop in FP64: {ms_loop64:.2f} ms/step")
    b = ssprkse.Batch(stream=stream)
    for st in sts:
        b.add(st)
    b.compile()
    assert b.step(1) == 0
    ms_plain = autotune._time_steps(torch, stream, lambda n: b.step_async(n), steps)
    tuned = autotune.tune_batch(b, steps=2)
    reinit()
    b.use_graph(True)
    assert b.step(1) == 0
    ms_batch = autotune._time_steps(torch, stream, lambda n: b.step_async(n), steps)
    assert b.sync() == 0
    ms_tuned = min(ms for _, ms in tuned["trials"] if ms is not None)
    log(f"[bench] ensemble batch: {ms_plain:.2f} ms/step default geometry, {ms_tuned:.2f} ms/step in the best "
        f"tuning trial, {ms_batch:.2f} ms/step tuned + graph ({tuned['best']})")
    out = {"workload": f"C3: {members} planar hex members, n in {{64,128,192,256}}, L in {{20,40,60}}, "
                       "M in [10,30], mixed precision",
           "cell_layers_per_step": cl, "per_member_loop_ms_per_step": ms_loop,
           "batch_default_geometry_ms_per_step": ms_plain, "batch_best_trial_ms_per_step": ms_tuned,
           "batch_tuned_graph_ms_per_step": ms_batch,
           "per_member_loop_cell_layer_updates_per_s": cl / (ms_loop * 1e-3),
           "per_member_loop_fp64_ms_per_step": ms_loop64,
           "batch_cell_layer_updates_per_s": cl / (ms_batch * 1e-3),
           "speedup_vs_per_member_loop": ms_loop / ms_batch,
           "speedup_vs_fp64_per_member_loop": ms_loop64 / ms_batch, "tuned": tuned["best"],
           "tuning_trials": len(tuned["trials"]), "launches_per_step": b.launches_per_step()}
    b.close()
    return out


def serve_leg(torch, ssprkse, cases, n_requests=64, loads=(0.8,), n_capacity=12, reduced=False):
    """C4: Poisson arrivals of sphere requests, continuous batching under an HBM
    budget.  The served recipe: icosahedral levels 5-8, 16-100 layers,
    50-500 steps, FP64 or mixed at random.  The service rate is measured
    first by serving the first `n_capacity` requests with all of them queued
    at t = 0 (cell-layer updates per second); the `n_requests` requests then
    arrive as a Poisson process at `load` times that rate divided by their
    mean work, once for every load in `loads` (the first one fills the
    top-level fields of the result, all of them `by_load`).  reduced=True
    serves a smaller mix (levels 4-6, 10-40 steps)."""
    import numpy as np
    from paper_2105_13484_amd.serve import Engine, Request, poisson_arrivals

    meshes = {}

    def make(i):
        if not reduced:
            c = cases.c4_request(i, meshes=meshes)
            return c, int(c.steps)
        rng = np.random.default_rng(cases.SEED_BASE + 400 + i)
        level = int(rng.integers(4, 7))
        L = int(rng.integers(16, 101))
        steps = int(rng.integers(10, 41))
        c = cases.sphere_case(level, L, cases.SEED_BASE + 400 + i, substeps=30, dt_btr=cases.served_dt_btr(level))
        c = cases.with_params(c, precision=int(rng.integers(0, 2)))
        return c, steps

    log(f"[bench] serving: building {n_requests} requests")
    made = [make(i) for i in range(n_requests)]
    levels = collections.Counter(int(round(np.log((c.mesh.nCells - 2) / 10) / np.log(4))) for c, _ in made)
    work = [c.active_cell_layers * s for c, s in made]
    log(f"[bench] serving: levels {dict(sorted(levels.items()))}, {sum(work):.3g} cell-layer updates in all")

    def requests(sel, arrivals):
        return [Request(rid=i, case=made[i][0], steps=made[i][1], arrival=a) for i, a in zip(sel, arrivals)]

    eng = Engine(budget_bytes=200 << 30, chunk_steps=10, keep_results=False)
    closed = eng.run(requests(range(n_capacity), [0.0] * n_capacity))
    rate = closed["cell_layer_updates_per_s"]
    cap = rate / (sum(work) / n_requests)
    log(f"[bench] serving capacity ({n_capacity} requests queued at t=0): {rate:.3g} cell-layer updates/s, "
        f"{cap:.3f} requests/s of the mix")
    # the plain method on the same requests: one at a time in arrival order,
    # each alone on the device (upload, its steps, result to the host), in the
    # precision it asks for, and once more with every request in FP64
    plain = {}
    for tag, prec in (("as_requested", None), ("fp64", 0)):
        t0 = time.perf_counter()
        done = 0
        for i in range(n_capacity):
            c, steps = made[i]
            if prec is not None:
                c = cases.with_params(c, precision=prec)
            dm, st = ssprkse.state_from_case(c, device="cuda:0")
            assert st.step(steps) == 0, f"request {i} failed alone"
            st.read()
            st.close()
            dm.close()
            done += work[i]
        plain[tag] = done / (time.perf_counter() - t0)
    log(f"[bench] serving the same {n_capacity} requests one at a time: {plain['as_requested']:.3g} cell-layer "
        f"updates/s as requested, {plain['fp64']:.3g} all in FP64")
    by_load = []
    for load in loads:
        arr = poisson_arrivals(n_requests, load * cap, cases.SEED_BASE + 499)
        shown = set()

        def progress(k, n):
            if k % 8 == 0 and k not in shown:
                shown.add(k)
                log(f"[bench] serving at {load:.1f}x: {k}/{n} done")

        opened = eng.run(requests(range(n_requests), arr), on_progress=progress)
        log(f"[bench] serving at {load:.1f}x capacity: p50 {opened['p50_s']:.3f} s, p99 {opened['p99_s']:.3f} s")
        by_load.append({"load": load, "p50_s": opened["p50_s"], "p99_s": opened["p99_s"], "max_s": opened["max_s"],
                        "cell_layer_updates_per_s": opened["cell_layer_updates_per_s"], "wall_s": opened["wall_s"],
                        "failed": opened["failed"]})
    eng.close()
    out = {"workload": ("C4 served recipe at reduced size: icosahedral levels 4-6, L 16-100, 10-40 steps" if reduced else
                        "C4 served recipe: icosahedral levels 5-8, L 16-100, 50-500 steps") +
                       ", FP64 or mixed at random, M = 30, HBM budget 200 GB",
           "requests": n_requests, "levels": dict(sorted(levels.items())),
           "capacity_cell_layer_updates_per_s": rate, "capacity_requests_per_s": cap,
           "capacity_sample_requests": n_capacity,
           "one_at_a_time_cell_layer_updates_per_s": plain["as_requested"],
           "one_at_a_time_fp64_cell_layer_updates_per_s": plain["fp64"],
           "capacity_speedup_vs_one_at_a_time": rate / plain["as_requested"],
           "capacity_speedup_vs_one_at_a_time_fp64": rate / plain["fp64"]}
    out.update(by_load[0])
    if len(by_load) > 1:
        out["by_load"] = by_load
    return out


def copy_probe():
    import torch
    a = torch.ones(COPY_PROBE_BYTES // 8, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    log(f"[bench] copy probe: {COPY_PROBE_BYTES} bytes read and written once")


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=512, help="hex mesh is n x n cells")
    ap.add_argument("--layers", type=int, default=60)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision timing")
    ap.add_argument("--no-c2", action="store_true", help="skip the level-7 sphere timings")
    ap.add_argument("--no-vmix", action="store_true", help="skip the implicit-vertical-mixing timing")
    ap.add_argument("--no-del4", action="store_true", help="skip the biharmonic-viscosity timing")
    ap.add_argument("--no-tracer", action="store_true", help="skip the evolving-tracer timing")
    ap.add_argument("--no-m-sweep", action="store_true", help="skip the runtime-vs-M sweep")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the batched-ensemble leg")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving leg")
    ap.add_argument("--serve-reduced", action="store_true", help="serving leg with a smaller request mix")
    ap.add_argument("--serve-requests", type=int, default=64, help="requests in the serving leg")
    ap.add_argument("--serve-loads", default="0.8",
                    help="comma-separated arrival rates of the serving leg, as fractions of its measured capacity")
    ap.add_argument("--copy-probe", action="store_true", help="run only a plain device copy and exit")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the step would shard by horizontal domain decomposition with whole columns and halo exchanges).",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe()
        return

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
    log(f"[bench] uploaded: mesh {dm.nbytes / 1e9:.3f} GB, state {st.nbytes / 1e9:.3f} GB, "
        f"edge variant {st.edge_variant}, barotropic variant {st.bt_variant}")

    assert st.step(args.warmup) == 0, "warmup failed"

    # per-class timing over a few steps: which kernel class dominates
    st.profile(ssprkse.PROF_CLASSES)
    assert st.step(3) == 0
    prof = st.profile_read()
    st.profile(())
    dom = max(prof, key=lambda k: prof[k][1])
    log("[bench] per-class ms over 3 steps: " + ", ".join(f"{k}={v[1]:.3f}({v[0]})" for k, v in prof.items()))

    copy_gbs = copy_bandwidth(torch)
    log(f"[bench] plain 1 GiB device copy: {copy_gbs:.0f} GB/s (bytes read + written)")

    # timed region 1: clean
    t0 = time.perf_counter()
    ms_step = timed_steps(torch, st, args.steps)
    wall = (time.perf_counter() - t0) * 1e3 / args.steps
    log(f"[bench] {args.steps} steps: {ms_step:.3f} ms/step (events), wall {wall:.3f} ms/step")

    # timed region 2: the same steps with HIP events around the dominant class only
    st.profile((dom,))
    torch.cuda.synchronize()
    assert st.step(args.steps) == 0
    n_dom, ms_dom = st.profile_read()[dom]
    st.profile(())
    avg_ms = ms_dom / max(n_dom, 1)
    kb = kernel_bytes(dom, C, E, V, L, bt_tiled=st.bt_variant == 1)
    ib = intermediate_bytes(dom, C, E, V, L)
    achieved = kb / (avg_ms * 1e-3) / 1e9
    traffic = measured_traffic(dom)
    log(f"[bench] dominant class {dom}: {n_dom} launches, {avg_ms * 1e3:.1f} us avg, "
        f"{achieved:.0f} GB/s algorithmic, measured traffic per launch {traffic}")
    # the edge pass's column gathers alone, beside the pass itself
    gather = gather_only(torch, st, E, L)
    edge_ms = avg_ms if dom == "fe_edge" else prof["fe_edge"][1] / max(prof["fe_edge"][0], 1)
    gather["edge_pass_launch_ms"] = edge_ms
    gather["launch_over_gather_only"] = edge_ms / gather["gather_only_launch_ms"]
    log(f"[bench] the edge pass's column gathers alone: {gather['gather_only_launch_ms'] * 1e3:.1f} us per "
        f"launch ({gather['gathered_gbs']:.0f} GB/s into registers); the pass takes "
        f"{gather['launch_over_gather_only']:.2f}x that")
    final = st.read()
    assert np.isfinite(final["u"]).all() and np.isfinite(final["h"]).all()
    del st

    # the same workload in mixed precision: FP32 tendencies and substeps
    # (SSE_MIXED), and FP32 tendencies with the barotropic loop in FP64
    # (SSE_MIXED_BT64)
    ms_mixed = ms_bt64 = None
    if not args.no_mixed:
        _, st_m = ssprkse.state_from_case(cases.with_params(case, precision=1), device="cuda:0")
        assert st_m.step(args.warmup) == 0
        ms_mixed = timed_steps(torch, st_m, args.steps)
        log(f"[bench] C1 mixed precision: {ms_mixed:.3f} ms/step")
        del st_m
        _, st_m = ssprkse.state_from_case(cases.with_params(case, precision=2), device="cuda:0")
        assert st_m.step(args.warmup) == 0
        ms_bt64 = timed_steps(torch, st_m, args.steps)
        log(f"[bench] C1 mixed precision with the barotropic loop in FP64: {ms_bt64:.3f} ms/step")
        del st_m

    # the same workload with implicit vertical mixing (Algorithm 2 in every stage)
    ms_vmix = None
    if not args.no_vmix:
        _, st_v = ssprkse.state_from_case(cases.with_params(case, vmix=1), device="cuda:0")
        assert st_v.step(args.warmup) == 0
        ms_vmix = timed_steps(torch, st_v, args.steps)
        log(f"[bench] C1 with implicit vertical mixing: {ms_vmix:.3f} ms/step")
        del st_v

    # the same workload with the biharmonic viscosity in place of the Laplacian
    # (nu_h = 1e9 m^4/s, about the paper's global value scaled to 5 km cells)
    ms_del4 = None
    if not args.no_del4:
        _, st_d = ssprkse.state_from_case(cases.with_params(case, hdiff=1, nu_h=1.0e9), device="cuda:0")
        assert st_d.step(args.warmup) == 0
        ms_del4 = timed_steps(torch, st_d, args.steps)
        log(f"[bench] C1 with biharmonic viscosity: {ms_del4:.3f} ms/step")
        del st_d

    # the same workload with the temperature evolving and the density following
    # the linear EOS every stage (kappa_h = 10 m^2/s, kappa_v = 1e-5 m^2/s)
    ms_tracer = None
    if not args.no_tracer:
        _, st_t = ssprkse.state_from_case(cases.with_params(case, tracer=1, kappa_h=10.0, kappa_v=1.0e-5),
                                          device="cuda:0")
        assert st_t.step(args.warmup) == 0
        ms_tracer = timed_steps(torch, st_t, args.steps)
        log(f"[bench] C1 with an evolving temperature tracer: {ms_tracer:.3f} ms/step")
        del st_t

    # runtime vs the number of substeps at fixed T and dt_btr, both schemes
    m_sweep = None if args.no_m_sweep else m_sweep_leg(torch, ssprkse, dm, case)
    del dm

    # C2 recipe: level-7 sphere, 60 layers, 30% land, M = 30, dt = 1800 s
    c2 = None
    if not args.no_c2:
        log("[bench] building the level-7 sphere (C2 recipe)")
        case2 = cases.c2()
        c2 = {"workload": "C2: SSPRK3-SE on an icosahedral level-7 sphere (163,842 cells, 491,520 edges), "
                          "60 z-star layers, 30% land, M=30, dt=1800 s",
              "active_cell_layers": case2.active_cell_layers}
        for prec, key in ((0, "fp64"), (1, "mixed")):
            dm2, st2 = ssprkse.state_from_case(cases.with_params(case2, precision=prec), device="cuda:0")
            assert st2.step(2) == 0
            ms2 = timed_steps(torch, st2, 20)
            c2[f"{key}_ms_per_step"] = ms2
            c2[f"{key}_cell_layer_updates_per_s"] = case2.active_cell_layers / (ms2 * 1e-3)
            log(f"[bench] C2 {key}: {ms2:.3f} ms/step")
            del st2, dm2
        c2["mixed_vs_fp64_speedup"] = c2["fp64_ms_per_step"] / c2["mixed_ms_per_step"]

    ensemble = None if args.no_ensemble else ensemble_leg(torch, ssprkse, cases)
    serving = None if args.no_serve else serve_leg(torch, ssprkse, cases, n_requests=args.serve_requests,
                                                    loads=tuple(float(x) for x in args.serve_loads.split(",")),
                                                    reduced=args.serve_reduced)

    value = cell_layers / (ms_step * 1e-3)
    step_gbs = STEP_BYTES_PER_CELL_LAYER * cell_layers / (ms_step * 1e-3) / 1e9
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
        "hbm_frac_step_target": 0.60,
        "mixed_vs_fp64_speedup": (ms_step / ms_mixed) if ms_mixed else None,
        "mixed_ms_per_step": ms_mixed,
        "mixed_bt64_vs_fp64_speedup": (ms_step / ms_bt64) if ms_bt64 else None,
        "mixed_bt64_ms_per_step": ms_bt64,
        "vmix_ms_per_step": ms_vmix,
        "del4_ms_per_step": ms_del4,
        "tracer_ms_per_step": ms_tracer,
        "per_class_ms_per_step": {k: v[1] / 3.0 for k, v in prof.items()},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_launch": kb, "intermediate_bytes_per_launch": ib, "launch_ms": avg_ms,
                     "achievable_copy_gbs": copy_gbs,
                     # the HBM side as measured: FETCH + WRITE bytes per launch over the launch time
                     "traffic_gbs": traffic / (avg_ms * 1e-3) / 1e9 if traffic else None,
                     "traffic_frac": traffic / (avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBS if traffic else None,
                     **(gather if dom == "fe_edge" else {})},
        "edge_gathers": gather,
        "c2": c2,
        "m_sweep": m_sweep,
        "ensemble": ensemble,
        "serving": serving,
    }
    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on a bounded sample")
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
