"""Whole-step FP64 parity cases, their error measures and their bounds.

Every FP64 comparison of whole steps between the HIP library and the oracle
takes its case from ``CASES`` (a builder of seeded inputs and a step count),
so that the bounds recorded for a case belong to exactly the run that is
compared.

Error measures, per field (u, h, zeta, ubar, and T when a tracer is carried):

* ``l2``:  ||gpu - oracle||_2 / ||oracle||_2 (relative L2 over all entries);
* ``max``: max_i |gpu_i - oracle_i| / max_i |oracle_i| (the largest element
  error, relative to the field's largest magnitude).

Bounds.  FP64 results must agree to ``TOL_L2`` = 1e-11 in relative L2 and
``TOL_MAX`` = 1e-10 element-wise.  Rounding is amplified by long windows (the
split system cancels four digits in zeta = sum h - H, and without the exact
reconciliation errors in h grow by orders of magnitude per step), so the
oracle alone is measured first: ``tests/golden/make_parity_bounds.py`` runs
every case with the oracle four times -- column sums correctly rounded (the
reference), added top-down, added bottom-up, and from inputs perturbed by one
unit in the last place -- and records the largest distance of the three
variants from the reference per field in ``tests/golden/parity_bounds.json``.
A field's bound is ``max(TOL, AMPLIFICATION * spread)``: the GPU rounds
differently from the oracle at every operation, not only in column sums, so it
may sit a few times further from the reference than any one variant.
"""
from __future__ import annotations

import json
import os

import numpy as np

from synthetic import cases
from tests.helpers import smooth_case

TOL_L2 = 1e-11
TOL_MAX = 1e-10
AMPLIFICATION = 4.0
BOUNDS_FILE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "parity_bounds.json")


# --- term switches ---------------------------------------------------------
def del4(case, nu):
    return cases.with_params(case, hdiff=1, nu_h=nu)


def vmix(case, nu_v=2e-2, c_drag=3e-3):
    return cases.with_params(case, vmix=1, nu_v=nu_v, c_drag=c_drag)


def tracer(case, **kw):
    kw.setdefault("tracer", 1)
    return cases.with_params(case, **kw)


def with_temp(case, T):
    from dataclasses import replace
    return replace(case, temp=T)


def all_terms(case, nu4=1e9):
    return cases.with_params(case, vmix=1, hdiff=1, tracer=1, nu_h=nu4, nu_v=1e-3, c_drag=2e-3,
                             kappa_h=20.0, kappa_v=1e-4)


def _smooth_tracer(scheme):
    base = smooth_case(n=10, L=5, scheme=scheme, M=6, dt=180.0)
    L = base.h.shape[1]
    x = base.mesh.xCell[:, 0]
    T0 = 8.0 + 2.0 * np.arange(L)[None, :] + 0.5 * np.sin(2 * np.pi * x / base.mesh.Lx)[:, None]
    return with_temp(tracer(base, kappa_h=20.0, kappa_v=1e-3), T0)


def drop_stencil_pairs(case, n_pairs=24, seed=5):
    """The case on a copy of its mesh where n_pairs symmetric pairs of
    reconstruction-stencil entries (e' in the stencil of e and e in that of e')
    are removed, weights included.  The weights stay antisymmetric, so the
    Coriolis and vorticity terms stay energy neutral, but those stencils are no
    longer "all other edges of the two cells": the library cannot put them in
    its canonical two-cell order and its edge pass takes the generic tables
    (every stencil edge with its own two vertices)."""
    from dataclasses import replace
    m = case.mesh
    rng = np.random.default_rng(seed)
    eoe, neoe, w = m.edgesOnEdge.copy(), m.nEdgesOnEdge.copy(), m.weightsOnEdge.copy()

    def remove(e, ep):
        n = int(neoe[e])
        j = int(np.nonzero(eoe[e, :n] == ep)[0][0])
        eoe[e, j:n - 1], w[e, j:n - 1] = eoe[e, j + 1:n].copy(), w[e, j + 1:n].copy()
        eoe[e, n - 1], w[e, n - 1] = -1, 0.0
        neoe[e] = n - 1

    done, touched = 0, set()
    for e in rng.permutation(m.nEdges):
        if done == n_pairs:
            break
        if e in touched:
            continue
        cand = [int(x) for x in eoe[e, :neoe[e]] if int(x) not in touched and int(x) != e]
        if not cand:
            continue
        ep = cand[0]
        remove(e, ep)
        remove(ep, e)
        touched.update((int(e), ep))
        done += 1
    mesh = replace(m, edgesOnEdge=eoe, nEdgesOnEdge=neoe, weightsOnEdge=w)
    return replace(case, mesh=mesh)


def _c2_small(**kw):
    return cases.sphere_case(3, 60, cases.SEED_BASE + 200, substeps=30, dt_btr=240.0, **kw)


# --- the cases: name -> (builder, steps) ------------------------------------
CASES = {
    # plain method (test_gpu_parity)
    "c0_ssprk3_100": (lambda: cases.with_params(cases.c0(), scheme=3), 100),
    "c0_ssprk3_20": (lambda: cases.with_params(cases.c0(), scheme=3), 20),
    "c0_ssprk2_30": (lambda: cases.c0(), 30),
    "c1_recipe_32x32x60": (lambda: cases.c1(n=32, L=60, steps=4), 4),
    "c2_recipe_level3x60": (lambda: _c2_small(), 3),
    "hex8_L100": (lambda: cases.c1(n=8, L=100, steps=2), 2),
    # implicit vertical mixing (test_gpu_vmix)
    "vmix_ssprk2": (lambda: vmix(smooth_case(n=10, L=5, scheme=2, M=6, dt=180.0)), 6),
    "vmix_ssprk3": (lambda: vmix(smooth_case(n=10, L=5, scheme=3, M=6, dt=180.0)), 12),
    "vmix_c1_recipe_32x32x60": (lambda: vmix(cases.c1(n=32, L=60, steps=4), nu_v=1e-4, c_drag=1e-3), 4),
    "vmix_c2_recipe_level3x60": (lambda: vmix(_c2_small(), nu_v=1e-4, c_drag=1e-3), 3),
    "vmix_hex8_L100": (lambda: vmix(cases.c1(n=8, L=100, steps=2)), 2),
    # biharmonic viscosity (test_gpu_del4)
    "del4_ssprk2": (lambda: del4(smooth_case(n=10, L=5, scheme=2, M=6, dt=180.0), 2e10), 6),
    "del4_ssprk3": (lambda: del4(smooth_case(n=10, L=5, scheme=3, M=6, dt=180.0), 2e10), 12),
    "del4_c1_recipe_32x32x60": (lambda: del4(cases.c1(n=32, L=60, steps=4), 1e9), 4),
    "del4_c2_recipe_level3x60": (lambda: del4(_c2_small(), 1e16), 3),
    "del4_vmix_16x16x20": (lambda: cases.with_params(del4(cases.c1(n=16, L=20, steps=3), 1e9), vmix=1,
                                                     nu_v=1e-2, c_drag=2e-3), 3),
    # tracer and EOS (test_gpu_tracer)
    "tracer_ssprk2": (lambda: _smooth_tracer(2), 6),
    "tracer_ssprk3": (lambda: _smooth_tracer(3), 12),
    "tracer_c1_recipe_32x32x60": (lambda: tracer(cases.c1(n=32, L=60, steps=4), kappa_h=10.0, kappa_v=1e-5), 4),
    "tracer_c2_recipe_level3x60": (lambda: tracer(_c2_small(), kappa_h=1e3, kappa_v=1e-5), 3),
    "tracer_isopycnal_8x8x100": (lambda: tracer(cases.c1(n=8, L=100, steps=2), vcoord=1, kappa_h=10.0,
                                                kappa_v=1e-4), 2),
    # every optional term at once (test_gpu_combined, test_gpu_extremes)
    "all_terms_hex12_L20_ssprk3": (lambda: all_terms(cases.c1(n=12, L=20, steps=4)), 4),
    "all_terms_hex12_L20_ssprk2": (lambda: all_terms(cases.with_params(cases.c1(n=12, L=20, steps=4),
                                                                       scheme=2)), 2),
    "all_terms_hex8_L100": (lambda: all_terms(cases.c1(n=8, L=100, steps=2)), 2),
    "all_terms_sphere3_land_L7": (lambda: all_terms(cases.sphere_case(3, 7, 77, substeps=5, dt_btr=200.0),
                                                    nu4=1e13), 3),
    "all_terms_hex8_L128": (lambda: all_terms(cases.c1(n=8, L=128, steps=2)), 2),
    # reconstruction stencils the library cannot put in canonical two-cell order
    "generic_stencils_hex12_L20": (lambda: drop_stencil_pairs(cases.c1(n=12, L=20, steps=3)), 3),
    "generic_stencils_sphere3_land_L7": (lambda: drop_stencil_pairs(
        cases.sphere_case(3, 7, 77, substeps=5, dt_btr=200.0)), 3),
    # ends of the accepted ranges (test_gpu_extremes)
    "hex8_L128": (lambda: cases.c1(n=8, L=128, steps=2), 2),
    "hex10_L65": (lambda: cases.c1(n=10, L=65, steps=2), 2),
    "hex12_L1_ssprk3": (lambda: cases.c1(n=12, L=1, steps=6), 6),
    "hex12_L1_ssprk2": (lambda: cases.with_params(cases.c1(n=12, L=1, steps=4), scheme=2), 4),
    "sphere3_land_L1": (lambda: cases.sphere_case(3, 1, 91, substeps=5, dt_btr=200.0), 4),
    "hex10_L20_M1_ssprk3": (lambda: cases.c1(n=10, L=20, substeps=1, dt_btr=15.0, steps=6), 6),
    "hex10_L20_M1_ssprk2": (lambda: cases.with_params(cases.c1(n=10, L=20, substeps=1, dt_btr=15.0, steps=4),
                                                      scheme=2), 4),
}
for _rec in (0, 1, 2):
    for _scheme in (2, 3):
        # without the exact reconciliation roundoff in h is amplified by orders of
        # magnitude per step, so those modes are compared over a short window
        CASES[f"reconcile{_rec}_ssprk{_scheme}"] = (
            (lambda r=_rec, s=_scheme: smooth_case(n=10, L=5, scheme=s, reconcile=r, M=6, dt=180.0)),
            12 if _rec == 1 else 3)
for _scheme in (2, 3):
    CASES[f"isopycnal_ssprk{_scheme}"] = (
        (lambda s=_scheme: cases.with_params(smooth_case(n=10, L=5, scheme=s, M=6, dt=180.0), vcoord=1)), 12)


def build(name: str):
    make, steps = CASES[name]
    return make(), steps


# --- oracle runs ------------------------------------------------------------
def oracle_fields(case, steps: int) -> dict:
    """The oracle's state after ``steps`` steps, by field name."""
    from oracle import ssprk_se as S
    out = S.run(case, steps)
    names = ("u", "h", "zeta", "ubar", "T")[:len(out)]
    return dict(zip(names, out))


# --- errors and bounds ------------------------------------------------------
def field_errors(a: np.ndarray, ref: np.ndarray) -> dict:
    d = np.asarray(a, float) - np.asarray(ref, float)
    n2, nmax = np.linalg.norm(ref), np.abs(ref).max() if np.size(ref) else 0.0
    return {"l2": float(np.linalg.norm(d) / max(n2, 1e-300)),
            "max": float(np.abs(d).max() / max(nmax, 1e-300)) if np.size(d) else 0.0}


def errors(gpu: dict, ref: dict) -> dict:
    return {k: field_errors(gpu[k], ref[k]) for k in ref}


_bounds_cache = None


def recorded_spreads() -> dict:
    global _bounds_cache
    if _bounds_cache is None:
        with open(BOUNDS_FILE) as f:
            _bounds_cache = json.load(f)
    return _bounds_cache


def bounds(name: str) -> dict:
    """{field: {"l2": bound, "max": bound}} for a case of ``CASES``."""
    spreads = recorded_spreads()["cases"][name]
    return {k: {"l2": max(TOL_L2, AMPLIFICATION * s["l2"]), "max": max(TOL_MAX, AMPLIFICATION * s["max"])}
            for k, s in spreads.items()}


def format_errors(errs: dict) -> str:
    return ", ".join(f"{k}: l2={v['l2']:.2e} max={v['max']:.2e}" for k, v in errs.items())


def check(name: str, gpu: dict, ref: dict, report=print) -> dict:
    """Compares every field of ``ref`` with ``gpu`` against the case's bounds."""
    errs = errors(gpu, ref)
    bnd = bounds(name)
    report(f"[parity] {name}: {format_errors(errs)}")
    for k, e in errs.items():
        for m in ("l2", "max"):
            assert e[m] <= bnd[k][m], (name, k, m, e[m], bnd[k][m])
    return errs
