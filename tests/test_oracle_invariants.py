"""Invariants the paper states or implies, checked on the oracle.

* free condition after Algorithm 1: sum_k h_k ut^1_k = 0 (Algorithm 1, the
  G-bar subtraction);
* SSH reconciliation (Section 3.4): the layer SSH sum h - H equals the
  barotropic SSH at stage 1 (both schemes), at stage 2 (SSPRK3-SE) and at the
  end of the step in the "exact" mode; in the "literal" mode the final
  mismatch is exactly -(dt/2) div D^e_1 (SSPRK2-SE) or
  -(dt/6) div(D^e_1 + D^e_2) (SSPRK3-SE), derived from the printed formulas;
* total volume is conserved (flux form, Section 1's argument for flux-form
  reconciliation); per-layer volume too when isopycnal;
* lake at rest stays at rest: flat bottom with stratification (bitwise), and
  with bathymetry or land under uniform density (to roundoff: zeta = sum h - H
  carries ~1e-12 m of rounding for H ~ 1000 m, which forces at most
  g dt |grad zeta| ~ 1e-12 m/s per step, so 100 steps stay below 1e-10 m/s);
* one layer: the baroclinic velocity vanishes and h_1 = zeta + H.
"""
import numpy as np
import pytest

from oracle import ssprk_se as S
from oracle import trisk
from oracle.layered import Setup
from synthetic import cases
from tests.helpers import smooth_case, uniform_case


def test_free_condition_after_baroclinic_feuler():
    case = smooth_case()
    st = Setup.from_case(case)
    ubar, ut = S.split(case.u, case.h, st)
    he = trisk.cell_to_edge(case.h, case.mesh)
    assert np.abs((he * ut).sum(1)).max() < 1e-14 * (he * np.abs(ut)).sum(1).max()
    zeta = S.ssh(case.h, st)
    ut1, G = S.baroclinic_feuler(case.u, ut, zeta, case.h, case.params.dt, st)
    assert np.abs((he * ut1).sum(1)).max() < 1e-14 * (he * np.abs(ut1)).sum(1).max()
    assert np.abs(G).max() > 0


@pytest.mark.parametrize("scheme", [2, 3])
@pytest.mark.parametrize("reconcile", [1, 2, 0])
def test_reconciliation_identities(scheme, reconcile):
    case = smooth_case(scheme=scheme, reconcile=reconcile, M=6, dt=360.0)
    st = Setup.from_case(case)
    m, dt = case.mesh, case.params.dt
    u, h = case.u.copy(), case.h.copy()
    for _ in range(2):                      # a non-trivial state first
        u, h = S.step(u, h, st)
    d = {}
    S.step(u, h, st, d)
    tol = 1e-12 * case.H.max()              # roundoff of sum h - H
    if reconcile == 0:
        assert np.abs(d["zeta1"] - d["zeta_bt1"]).max() > 1e3 * tol
        return
    np.testing.assert_allclose(d["zeta1"], d["zeta_bt1"], rtol=0, atol=tol)
    if scheme == 3:
        zl2 = S.ssh(d["h2"], st)
        np.testing.assert_allclose(zl2, d["zeta_bt2"], rtol=0, atol=tol)
        final_bt = d["zeta_bt3"]
        if reconcile == 2:
            De1 = d["Fz1"] - d["Fh1"]
            De2 = d["Fz2"] - d["Fh2"]
            final_bt = final_bt - dt / 6.0 * trisk.divergence(De1 + De2, m)
    else:
        final_bt = d["zeta_bt2"]
        if reconcile == 2:
            final_bt = final_bt - dt / 2.0 * trisk.divergence(d["Fz1"] - d["Fh1"], m)
    np.testing.assert_allclose(d["zeta_new"], final_bt, rtol=0, atol=tol)


@pytest.mark.parametrize("scheme", [2, 3])
def test_volume_conservation(scheme):
    # SSPRK2 is unstable for undamped gravity waves (|R_2(iy)| > 1): keep its CFL small
    case = smooth_case(scheme=scheme, M=5, dt=100.0 if scheme == 2 else 300.0)
    st = Setup.from_case(case)
    a = case.mesh.areaCell
    u, h = case.u.copy(), case.h.copy()
    v0 = (a[:, None] * h).sum()
    for _ in range(40):
        u, h = S.step(u, h, st)
    assert abs((a[:, None] * h).sum() / v0 - 1.0) < 1e-13


def test_volume_conservation_sphere_with_land():
    case = cases.sphere_case(3, 6, 1234, substeps=8, dt_btr=240.0)
    st = Setup.from_case(case)
    a = case.mesh.areaCell
    rng = np.random.default_rng(3)
    u = np.where(st.edge_mask[:, None], rng.normal(0, 0.01, case.u.shape), 0.0)
    h = case.h.copy()
    v0 = (a[:, None] * h).sum()
    for _ in range(10):
        u, h = S.step(u, h, st)
    assert np.isfinite(u).all()
    assert abs((a[:, None] * h).sum() / v0 - 1.0) < 1e-13
    assert (u[~st.edge_mask] == 0.0).all()
    assert (h[~st.cell_mask] == case.h[~st.cell_mask]).all()


def test_layer_volume_conservation_isopycnal():
    case = cases.with_params(smooth_case(M=5, dt=300.0), vcoord=1)
    st = Setup.from_case(case)
    a = case.mesh.areaCell
    u, h = case.u.copy(), case.h.copy()
    v0 = (a[:, None] * h).sum(0)
    for _ in range(20):
        u, h = S.step(u, h, st)
    np.testing.assert_allclose((a[:, None] * h).sum(0), v0, rtol=1e-13)


@pytest.mark.parametrize("scheme", [2, 3])
def test_lake_at_rest_flat_stratified_is_bitwise(scheme):
    case = uniform_case(L=5, scheme=scheme, M=4, dt=600.0, nu_v=1e-3, c_drag=1e-3)
    st = Setup.from_case(case)
    u, h = case.u.copy(), case.h.copy()
    for _ in range(20):
        u, h = S.step(u, h, st)
    assert (u == 0.0).all() and (h == case.h).all()


def test_lake_at_rest_bathymetry_uniform_density():
    case = cases.c1(n=16, L=10, steps=100)
    case.rho[:] = 1025.0
    st = Setup.from_case(case)
    u, h = case.u.copy(), case.h.copy()
    for _ in range(100):
        u, h = S.step(u, h, st)
    assert np.abs(u).max() < 1e-10


def test_lake_at_rest_sphere_land_uniform_density():
    case = cases.sphere_case(3, 8, 4321, substeps=8, dt_btr=240.0)
    case.rho[:] = np.where(case.cell_mask[:, None] > 0, 1025.0, 0.0)
    st = Setup.from_case(case)
    u, h = case.u.copy(), case.h.copy()
    for _ in range(100):
        u, h = S.step(u, h, st)
    assert np.abs(u).max() < 1e-10


@pytest.mark.parametrize("scheme", [2, 3])
def test_single_layer_reduction(scheme):
    base = smooth_case(L=1, scheme=scheme, M=4, dt=240.0)
    st = Setup.from_case(base)
    u, h = base.u.copy(), base.h.copy()
    for _ in range(10):
        u, h = S.step(u, h, st)
        ubar, ut = S.split(u, h, st)
        assert np.abs(ut).max() <= 1e-15 * np.abs(u).max()
        np.testing.assert_allclose(h[:, 0] - base.H, S.ssh(h, st), rtol=0, atol=1e-12 * base.H.max())


def _growth(reconcile, scheme, steps=12, eps=1e-15):
    case = smooth_case(n=10, L=5, scheme=scheme, reconcile=reconcile, M=6, dt=180.0)
    st = Setup.from_case(case)
    rng = np.random.default_rng(0)
    u1, h1 = case.u.copy(), case.h.copy()
    u2, h2 = case.u.copy(), case.h * (1 + eps * rng.standard_normal(case.h.shape))
    for _ in range(steps):
        u1, h1 = S.step(u1, h1, st)
        u2, h2 = S.step(u2, h2, st)
    return np.linalg.norm(u2 - u1) / np.linalg.norm(u1)


@pytest.mark.parametrize("scheme", [2, 3])
def test_reconciliation_conditioning(scheme):
    """A roundoff-sized perturbation of the layer thicknesses stays at roundoff
    with the exact reconciliation but is amplified by orders of magnitude
    without it: the layer SSH then carries a fast mode that the barotropic
    solve does not control (Remark 3.1 and the stability discussion of
    Section 5 on reconciliation)."""
    exact, off = _growth(1, scheme), _growth(0, scheme)
    assert exact < 1e-11
    assert off > 100 * exact
