"""Measures how far rounding alone moves each whole-step parity case, with
the oracle only, and writes ``tests/golden/parity_bounds.json``.

For every case of ``tests.parity_cases.CASES`` the oracle runs four times:

* ``exact``     column sums correctly rounded (the reference the GPU is compared with);
* ``top_down``  the layers of every column sum added from the surface down;
* ``bottom_up`` added from the bottom up;
* ``ulp``       correctly rounded sums, from initial u, h (and T) multiplied by
                1 + r 2^-52 with r drawn from {-1, 0, 1} (one unit in the last place).

For each field the file records the largest distance of the three variants
from ``exact``, as relative L2 and as the largest element error relative to
the field's largest magnitude.  ``tests.parity_cases.bounds`` turns these
spreads into the bounds of the GPU parity tests.

    python tests/golden/make_parity_bounds.py [--jobs N] [case ...]

With case names, only those entries are recomputed and merged into the file.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time
from dataclasses import replace
from multiprocessing import Pool

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import layered  # noqa: E402
from tests import parity_cases as P  # noqa: E402

ULP = 2.0 ** -52


def _perturbed(case, seed: int):
    rng = np.random.default_rng(seed)

    def bump(a):
        return a * (1.0 + ULP * rng.integers(-1, 2, size=a.shape))

    kw = {"u": bump(case.u), "h": bump(case.h)}
    if case.temp is not None and getattr(case.params, "tracer", 0):
        kw["temp"] = bump(case.temp)
    return replace(case, **kw)


def measure(name: str) -> tuple[str, dict, float]:
    t0 = time.perf_counter()
    case, steps = P.build(name)
    layered.set_sum_order("exact")
    ref = P.oracle_fields(case, steps)
    spread = {k: {"l2": 0.0, "max": 0.0} for k in ref}
    for variant in ("top_down", "bottom_up", "ulp"):
        if variant == "ulp":
            layered.set_sum_order("exact")
            alt = P.oracle_fields(_perturbed(case, 2105), steps)
        else:
            layered.set_sum_order(variant)
            alt = P.oracle_fields(case, steps)
        for k, e in P.errors(alt, ref).items():
            for m in ("l2", "max"):
                v = e[m] if np.isfinite(e[m]) else float("inf")
                spread[k][m] = max(spread[k][m], v)
    layered.set_sum_order("exact")
    return name, spread, time.perf_counter() - t0


def main() -> None:
    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=4)
    ap.add_argument("names", nargs="*")
    args = ap.parse_args()
    names = args.names or sorted(P.CASES)
    data = {"cases": {}}
    if args.names and os.path.exists(P.BOUNDS_FILE):
        with open(P.BOUNDS_FILE) as f:
            data = json.load(f)
    data["rule"] = (f"bound = max(TOL, {P.AMPLIFICATION:g} x spread) per field and measure; "
                    f"TOL = {P.TOL_L2:g} (relative L2), {P.TOL_MAX:g} (max element error / max |field|); "
                    "spread = largest distance from the correctly rounded oracle run of the top-down, "
                    "bottom-up and one-ulp-perturbed oracle runs")
    with Pool(args.jobs) as pool:
        for name, spread, secs in pool.imap_unordered(measure, names):
            data["cases"][name] = spread
            worst = max(v["l2"] for v in spread.values())
            print(f"{name}: {secs:.0f} s, largest l2 spread {worst:.2e}", flush=True)
    data["cases"] = dict(sorted(data["cases"].items()))
    with open(P.BOUNDS_FILE, "w") as f:
        json.dump(data, f, indent=1, sort_keys=False)
        f.write("\n")


if __name__ == "__main__":
    main()
