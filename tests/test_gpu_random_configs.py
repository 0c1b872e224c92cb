"""Whole steps of seeded random configurations against the FP64 oracle.

The named cases of ``tests/parity_cases.py`` pin each option on its own
recipe; here every option is drawn at random, so that combinations the named
cases do not list run through the library: planar hexes and land-masked
spheres, 1 to 128 layers (across the 64-lane chunk boundary), either scheme,
M from 1 to 13, the three precision modes, both vertical coordinates, the
three reconciliation modes, implicit vertical mixing (Algorithm 2),
biharmonic viscosity and the temperature tracer.  Two steps each.

Bounds.  u, ubar, h and T as in the named cases: relative L2 <= 1e-11 and
element-wise <= 1e-10 of the field's largest value in FP64, or four times
the distance by which the oracle itself moves when its layer sums are taken
top-down or bottom-up instead of correctly rounded, or when its initial state
moves by one ulp (measured here, on the CPU, for each configuration).  zeta = sum h - H
cancels all but a small part of the column height (H ~ 10^3 m against
zeta ~ 10^-2 m on these recipes), so its error is measured against zeta + H,
the column height the thickness update carries: a layer sum of at most 128
terms of size <= H, taken in a different order, differs by a few ulps of H,
~1e-15 of it; the bound is 1e-13.  In mixed precision (Section 3.4 with the
3D fields in FP32): velocities 1e-5, h and T 1e-8, and zeta + H 1e-9 (the
reading of the SSH bound relative to the column height).
"""
from dataclasses import replace

import numpy as np
import pytest

from oracle import layered
from synthetic import cases
from tests import parity_cases as P

pytestmark = pytest.mark.gpu

N_CONFIGS = 48


def _configs(seed=2105, n=N_CONFIGS):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(n):
        kind = rng.choice(["hex", "hex", "sphere"])
        L = int(rng.choice([1, 2, 3, 7, 31, 63, 64, 65, 100, 127, 128]))
        kw = dict(scheme=int(rng.choice([2, 3])), precision=int(rng.choice([0, 0, 1, 2])),
                  substeps=int(rng.choice([1, 2, 5, 13])), reconcile=int(rng.choice([0, 1, 2])))
        size = int(rng.choice([4, 6, 8, 10, 12, 14]))
        if kind == "hex" and L > 64:
            size = min(size, 8)
        if L >= 2 and rng.random() < 0.25:
            kw["vcoord"] = 1
        if rng.random() < 0.3:
            kw.update(vmix=1, nu_v=1e-3, c_drag=2e-3)
        if rng.random() < 0.3:
            kw.update(hdiff=1, nu_h=1e9 if kind == "hex" else 1e13)
        if rng.random() < 0.3:
            kw.update(tracer=1, kappa_h=20.0, kappa_v=1e-4)
        out.append((i, str(kind), size, L, kw))
    return out


CONFIGS = _configs()


def _label(cfg):
    i, kind, size, L, kw = cfg
    mesh = f"hex{size}" if kind == "hex" else "sphere2"
    return f"{i:02d}-{mesh}-L{L}-" + "-".join(f"{k}{v}" for k, v in kw.items() if k in (
        "scheme", "precision", "substeps", "vcoord", "reconcile", "vmix", "hdiff", "tracer"))


def _case(cfg):
    i, kind, size, L, kw = cfg
    if kind == "hex":
        base = cases.c1(n=size, L=L, steps=2)
    else:
        base = cases.sphere_case(2, L, 500 + i, substeps=5, dt_btr=200.0)
    dt_btr = base.params.dt / base.params.substeps
    return cases.with_params(base, dt=dt_btr * kw["substeps"], **kw)


def _oracle_spread(case, steps, ref):
    """Largest distance of the oracle from ref over the three rounding variants."""
    spread = {k: {"l2": 0.0, "max": 0.0} for k in ref}
    rng = np.random.default_rng(2105)

    def bump(a):
        return a * (1.0 + 2.0 ** -52 * rng.integers(-1, 2, size=a.shape))

    try:
        for variant in ("top_down", "bottom_up", "ulp"):
            if variant == "ulp":
                layered.set_sum_order("exact")
                kw = {"u": bump(case.u), "h": bump(case.h)}
                if case.temp is not None and case.params.tracer:
                    kw["temp"] = bump(case.temp)
                alt = P.oracle_fields(replace(case, **kw), steps)
            else:
                layered.set_sum_order(variant)
                alt = P.oracle_fields(case, steps)
            for k, e in P.errors(alt, ref).items():
                for m in ("l2", "max"):
                    spread[k][m] = max(spread[k][m], e[m])
    finally:
        layered.set_sum_order("exact")
    return spread


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2105_13484_amd import ssprkse
    ssprkse.load()
    return ssprkse


@pytest.mark.parametrize("cfg", CONFIGS, ids=[_label(c) for c in CONFIGS])
def test_random_configuration_two_steps(dev, cfg):
    case = _case(cfg)
    steps = 2
    print(f"\n[random] {_label(cfg)}", flush=True)
    dm, st = dev.state_from_case(case)
    assert st.step(steps) == 0, dev.last_error()
    gpu = st.read()
    if case.params.tracer:
        gpu["T"] = st.read_tracer()
    ref = P.oracle_fields(case, steps)
    errs = P.errors(gpu, ref)
    colh = ref["zeta"] + case.H
    dz = np.asarray(gpu["zeta"]) - ref["zeta"]
    wet = case.cell_mask.astype(bool)
    errs["zeta+H"] = {"l2": float(np.linalg.norm(dz[wet]) / np.linalg.norm(colh[wet])),
                      "max": float(np.abs(dz[wet]).max() / np.abs(colh[wet]).max())}
    print(f"[random] {_label(cfg)}: " + P.format_errors(errs), flush=True)
    if case.params.precision == 0:
        spread = _oracle_spread(case, steps, ref)
        bound = {k: {m: max(P.TOL_L2 if m == "l2" else P.TOL_MAX, P.AMPLIFICATION * spread[k][m])
                     for m in ("l2", "max")} for k in ("u", "ubar", "h", "T") if k in ref}
        bound["zeta+H"] = {"l2": 1e-13, "max": 1e-13}
    else:
        bound = {k: {"l2": b, "max": 10 * b} for k, b in (("u", 1e-5), ("ubar", 1e-5), ("h", 1e-8), ("T", 1e-8))
                 if k in ref}
        bound["zeta+H"] = {"l2": 1e-9, "max": 1e-9}
    for k, b in bound.items():
        for m in ("l2", "max"):
            assert errs[k][m] <= b[m], (k, m, errs[k][m], b[m])
