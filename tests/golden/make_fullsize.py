"""Writes the stored oracle values of the full-size whole-step parity tests.

Three SSPRK3-SE steps of the two throughput workloads, run by the FP64 oracle
on the host (one step of the 512 x 512 x 60 hex takes several minutes, so the
GPU tests compare against values stored here instead of running the oracle):

* ``c1``: 512 x 512 periodic hex, 60 layers, M = 20, dt = 300 s, FP64;
* ``c2``: icosahedral level-7 sphere, 60 layers, 30 % land, M = 30,
  dt = 1800 s (the mixed-precision workload; the oracle is FP64).

Each workload is run three times: with correctly rounded column sums (the
oracle's default, the values the tests compare with) and with the layers added
top-down and bottom-up.  The spread between them measures how far rounding in
the column sums alone moves three full-size steps; the file records it per
field beside the sampled values.

Usage (each run writes its fields under TMP; ``combine`` reads all three):

    python tests/golden/make_fullsize.py run c1 exact TMP
    python tests/golden/make_fullsize.py run c1 top_down TMP
    python tests/golden/make_fullsize.py run c1 bottom_up TMP
    python tests/golden/make_fullsize.py combine c1 TMP

``combine`` writes ``tests/golden/fullsize_<case>.npz``: for each field
(u, h, zeta, ubar) a seeded sample of flat indices and the oracle's values
there, the full-field L2 and max norms, and the order spreads.  Only the
oracle and the seeded input generators are called.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import layered, ssprk_se  # noqa: E402
from synthetic import cases  # noqa: E402

STEPS = 3
FIELDS = ("u", "h", "zeta", "ubar")
SAMPLES = {"u": 65536, "h": 32768, "zeta": 32768, "ubar": 32768}
SAMPLE_SEED = 2105_13484 + 9


def build(name: str):
    if name == "c1":
        return cases.c1(n=512, L=60, steps=STEPS)
    if name == "c2":
        return cases.c2(level=7, L=60, mixed=True)
    raise ValueError(name)


def run(name: str, order: str, tmp: str) -> None:
    case = build(name)
    layered.set_sum_order(order)
    t0 = time.perf_counter()
    u, h, zeta, ubar = ssprk_se.run(case, STEPS)
    print(f"{name} {order}: {STEPS} steps in {time.perf_counter() - t0:.0f} s", flush=True)
    for f, a in zip(FIELDS, (u, h, zeta, ubar)):
        np.save(os.path.join(tmp, f"{name}_{order}_{f}.npy"), a)


def combine(name: str, tmp: str) -> str:
    rng = np.random.default_rng(SAMPLE_SEED)
    out = {"steps": np.array(STEPS)}
    spreads = {}
    for f in FIELDS:
        ref = np.load(os.path.join(tmp, f"{name}_exact_{f}.npy"))
        flat = ref.ravel()
        idx = np.sort(rng.choice(flat.size, size=min(SAMPLES[f], flat.size), replace=False))
        out[f"idx_{f}"] = idx.astype(np.int64)
        out[f"val_{f}"] = flat[idx]
        out[f"norm2_{f}"] = np.array(np.linalg.norm(flat))
        out[f"normmax_{f}"] = np.array(np.abs(flat).max())
        l2, linf = 0.0, 0.0
        for order in ("top_down", "bottom_up"):
            alt = np.load(os.path.join(tmp, f"{name}_{order}_{f}.npy")).ravel()
            l2 = max(l2, float(np.linalg.norm(alt - flat) / np.linalg.norm(flat)))
            linf = max(linf, float(np.abs(alt - flat).max() / np.abs(flat).max()))
        out[f"spread_l2_{f}"] = np.array(l2)
        out[f"spread_inf_{f}"] = np.array(linf)
        spreads[f] = (l2, linf)
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"fullsize_{name}.npz")
    np.savez_compressed(path, **out)
    print(json.dumps({name: spreads}), flush=True)
    return path


if __name__ == "__main__":
    if sys.argv[1] == "run":
        run(sys.argv[2], sys.argv[3], sys.argv[4])
    elif sys.argv[1] == "combine":
        print(combine(sys.argv[2], sys.argv[3]))
    else:
        raise SystemExit(__doc__)
