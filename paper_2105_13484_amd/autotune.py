"""Launch-configuration autotuner for single states and batches.

The knobs change how the work is laid out on the GPU, never the arithmetic
(results are bitwise identical for every choice; the GPU tests check it):

* column-kernel workgroup size: 1, 2, 4, 8 or 16 wavefronts (one vertical
  column per wavefront);
* 2D-kernel workgroup size (barotropic evaluations, reconciliation):
  64 .. 1024 threads;
* for single states, the edge-pass variant: direct gathers, or LDS tiles of
  8, 16 or 32 edges;
* the barotropic-loop kernel: one launch per substep over cell patches with
  their halo rings, one launch per forward-Euler evaluation, or (single
  states whose patches all fit the device at once) one cooperative launch for
  the whole loop; batch members choose between the first two.

The tuner times whole steps with HIP events on the state's (batch's) stream
and keeps the fastest setting.  It searches one knob at a time (coordinate
descent from the defaults), which needs 5 + 5 + 1 (+ 4) trials instead of the
full product.  Trial steps advance the state: tune a copy, or count them.
"""
from __future__ import annotations

import time

COLS_PER_BLOCK = (1, 2, 4, 8, 16)
BLOCK_2D = (64, 128, 256, 512, 1024)
BT_VARIANTS = (1, 0, 2)
BATCH_BT_VARIANTS = (1, 0)


def _time_steps(torch, stream, run, steps: int) -> float:
    """ms per step of run(steps) on `stream`."""
    s = stream if stream is not None else torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(s)
    run(steps)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / steps


def _descend(trial, start: dict, space: dict) -> tuple[dict, list]:
    """Coordinate descent over `space` (knob -> choices) from `start`."""
    best = dict(start)
    log = []
    best_ms = trial(best)
    log.append((dict(best), best_ms))
    for knob, choices in space.items():
        for v in choices:
            if v == best[knob]:
                continue
            cand = dict(best, **{knob: v})
            ms = trial(cand)
            log.append((dict(cand), ms))
            if ms is not None and (best_ms is None or ms < best_ms):
                best, best_ms = cand, ms
    return best, log


def tune_state(state, steps: int = 2, variants=None) -> dict:
    """Tune a DeviceState in place; returns the chosen setting and the trial log."""
    import torch
    from . import ssprkse
    variants = ssprkse.EDGE_VARIANTS if variants is None else variants

    def trial(cfg):
        state.set_geometry(cfg["cols_per_block"], cfg["block_2d"])
        if not state.try_edge_variant(cfg["edge_variant"]):
            return None
        if not state.try_bt_variant(cfg["bt_variant"]):
            return None
        state.step(1)  # first launch of a new configuration
        return _time_steps(torch, state.stream, lambda n: state.step_async(n), steps)

    t0 = time.perf_counter()
    start = {"cols_per_block": 4, "block_2d": 256, "edge_variant": -1, "bt_variant": state.bt_variant}
    best, log = _descend(trial, start, {"edge_variant": variants, "bt_variant": BT_VARIANTS,
                                        "cols_per_block": COLS_PER_BLOCK, "block_2d": BLOCK_2D})
    state.set_geometry(best["cols_per_block"], best["block_2d"])
    state.try_edge_variant(best["edge_variant"])
    state.try_bt_variant(best["bt_variant"])
    return {"best": best, "trials": log, "default_ms": log[0][1], "seconds": time.perf_counter() - t0}


def tune_batch(batch, steps: int = 2) -> dict:
    """Tune a Batch in place (recompiles its program per setting)."""
    import torch

    def set_bt(variant):
        return all(m.try_bt_variant(variant) for m in batch.members)

    def trial(cfg):
        if not set_bt(cfg["bt_variant"]):
            return None
        batch.set_geometry(cfg["cols_per_block"], cfg["block_2d"])
        batch.compile()
        batch.step(1)
        return _time_steps(torch, batch.stream, lambda n: batch.step_async(n), steps)

    t0 = time.perf_counter()
    first = batch.members[0].bt_variant if batch.members else 1
    best, log = _descend(trial, {"cols_per_block": 4, "block_2d": 256, "bt_variant": first},
                         {"bt_variant": BATCH_BT_VARIANTS, "block_2d": BLOCK_2D, "cols_per_block": COLS_PER_BLOCK})
    set_bt(best["bt_variant"])
    batch.set_geometry(best["cols_per_block"], best["block_2d"])
    batch.compile()
    return {"best": best, "trials": log, "default_ms": log[0][1], "seconds": time.perf_counter() - t0}
