"""Pins of the oracle's implicit vertical mixing (Algorithm 2).

* The tridiagonal solver against a banded LU of a library (scipy).
* The solve against the explicit operator: the returned u satisfies
  u - dt D^u(u) = r with the explicit D^u of the oracle (an independent code
  path that builds no matrix), the drag speed frozen, on a stratified planar
  case and on a sphere with land.
* Column momentum budget: the interior viscous fluxes telescope, so
  sum_k h_k u_k = sum_k h_k r_k - dt c_drag |u| u_bottom.
* Special cases: a vertically uniform column without drag is left alone; one
  layer gives u = r / (1 + dt c_drag |u| / h).
* Algorithm 2 without viscosity and drag is Algorithm 1.
* Whole step, f = 0, horizontally uniform layers: every horizontal operator
  vanishes and the SSPRK-SE step reduces to column algebra with dense
  backward-Euler maps (I - dt D)^{-1}, G-bar formed before the solve and the
  barotropic loop integrating the constant forcing exactly.
* Flux-form volume conservation and the lake at rest with mixing on.
"""
import numpy as np
import pytest
from scipy.linalg import solve_banded

from oracle import ssprk_se as S
from oracle import trisk
from oracle.layered import D_u, Setup, bottom_speed, thomas, vertical_diffusion_solve
from synthetic import cases
from tests.helpers import smooth_case, uniform_case


def test_thomas_matches_banded_lu():
    rng = np.random.default_rng(5)
    N, L = 40, 37
    a = rng.uniform(-1, 0, (N, L))
    c = rng.uniform(-1, 0, (N, L))
    b = 2.5 + rng.uniform(0, 1, (N, L))
    d = rng.normal(size=(N, L))
    x = thomas(a, b, c, d)
    for i in range(N):
        ab = np.zeros((3, L))
        ab[0, 1:] = c[i, :-1]
        ab[1] = b[i]
        ab[2, :-1] = a[i, 1:]
        ref = solve_banded((1, 1), ab, d[i])
        np.testing.assert_allclose(x[i], ref, rtol=1e-13, atol=1e-14)


def _residual_check(case, dt, seed):
    st = Setup.from_case(case)
    rng = np.random.default_rng(seed)
    E, L = case.u.shape
    u_in = np.where(st.edge_mask[:, None], rng.normal(0, 0.3, (E, L)), 0.0)
    r = np.where(st.edge_mask[:, None], rng.normal(0, 0.3, (E, L)), 0.0)
    s = bottom_speed(u_in, st)
    x = vertical_diffusion_solve(r, case.h, s, dt, st)
    back = x - dt * D_u(x, case.h, st, speed=s)
    assert np.abs(back - r).max() <= 1e-13 * np.abs(r).max()
    assert np.all(x[~st.edge_mask] == 0.0)
    return st, x, r, s


@pytest.mark.parametrize("nu_v,cd", [(1e-4, 1e-3), (5e-2, 2e-2), (1.0, 0.0)])
def test_solve_inverts_explicit_operator_planar(nu_v, cd):
    case = cases.with_params(smooth_case(n=8, L=7), nu_v=nu_v, c_drag=cd)
    _residual_check(case, 900.0, 1)


def test_solve_inverts_explicit_operator_sphere_with_land():
    case = cases.sphere_case(2, 9, 41, substeps=4, dt_btr=60.0)
    case = cases.with_params(case, nu_v=1e-2, c_drag=3e-3)
    _residual_check(case, 1800.0, 2)


def test_column_budget():
    case = cases.with_params(smooth_case(n=8, L=6), nu_v=3e-2, c_drag=4e-3)
    dt = 1200.0
    st, x, r, s = _residual_check(case, dt, 3)
    he = trisk.cell_to_edge(case.h, case.mesh)
    lhs = (he * x).sum(1)
    rhs = (he * r).sum(1) - dt * case.params.c_drag * s * x[:, -1]
    assert np.abs(lhs - rhs).max() <= 1e-12 * np.abs(he * r).sum(1).max()


def test_uniform_column_without_drag_is_unchanged():
    case = cases.with_params(smooth_case(n=8, L=5), nu_v=0.5, c_drag=0.0)
    st = Setup.from_case(case)
    E = case.u.shape[0]
    r = np.repeat(np.random.default_rng(4).normal(size=(E, 1)), 5, axis=1)
    x = vertical_diffusion_solve(r, case.h, np.ones(E), 600.0, st)
    assert np.abs(x - r).max() <= 1e-14 * np.abs(r).max()


def test_single_layer_closed_form():
    case = uniform_case(L=1, U=np.array([[0.3, -0.1]]), h_layers=[40.0], c_drag=2e-3, nu_v=1e-2)
    st = Setup.from_case(case)
    E = case.u.shape[0]
    r = np.random.default_rng(6).normal(size=(E, 1))
    s = np.full(E, 0.7)
    dt = 500.0
    x = vertical_diffusion_solve(r, case.h, s, dt, st)
    np.testing.assert_allclose(x, r / (1.0 + dt * 2e-3 * 0.7 / 40.0), rtol=1e-15)


def test_algorithm2_without_mixing_is_algorithm1():
    case = cases.with_params(smooth_case(n=8, L=4), nu_v=0.0, c_drag=0.0)
    st = Setup.from_case(case)
    ubar, ut = S.split(case.u, case.h, st)
    zeta = S.ssh(case.h, st)
    a1, g1 = S.baroclinic_feuler(case.u, ut, zeta, case.h, 300.0, st)
    a2, g2 = S.baroclinic_feuler_mixing(case.u, ut, ubar, zeta, case.h, 300.0, st)
    assert np.array_equal(g1, g2)
    assert np.abs(a1 - a2).max() <= 1e-15 * np.abs(case.u).max()


def _column_D(hk, nu_v, cd, speed):
    """Dense L x L matrix of D^u on horizontally uniform columns, drag speed frozen."""
    L = len(hk)
    D = np.zeros((L, L))
    for j in range(L):
        e = np.zeros(L)
        e[j] = 1.0
        tau = np.zeros(L + 1)
        for k in range(1, L):
            tau[k] = nu_v * (e[k - 1] - e[k]) / (0.5 * (hk[k - 1] + hk[k]))
        tau[L] = cd * speed * e[L - 1]
        D[:, j] = (tau[:-1] - tau[1:]) / hk
    return D


def _bfe_mix_column(V, Vbar, hk, nu_v, cd, dt):
    """Algorithm 2 on uniform columns with f = 0: returns (ut1, G)."""
    Vt = V - Vbar
    G = (hk[:, None] * Vt).sum(0) / hk.sum() / dt
    A = np.eye(len(hk)) - dt * _column_D(hk, nu_v, cd, np.linalg.norm(V[-1]))
    U1 = np.linalg.solve(A, Vt - dt * G + Vbar)
    return U1 - Vbar, G


def _column_step(scheme, U, hk, nu_v, cd, dt):
    ub = (hk[:, None] * U).sum(0) / hk.sum()
    ut = U - ub
    ut1, G0 = _bfe_mix_column(U, ub, hk, nu_v, cd, dt)
    ub1 = ub + dt * G0                        # constant forcing, integrated exactly
    ut2, G1 = _bfe_mix_column(ub1 + ut1, ub1, hk, nu_v, cd, dt)
    if scheme == 2:
        return ub + dt * 0.5 * (G0 + G1) + 0.5 * (ut + ut2)
    ub2 = ub1 + dt * G1
    ut_h, ub_h = 0.75 * ut + 0.25 * ut2, 0.75 * ub + 0.25 * ub2
    ut3, Gh = _bfe_mix_column(ub_h + ut_h, ub_h, hk, nu_v, cd, dt)
    return ub + dt * (G0 / 6.0 + G1 / 6.0 + 2.0 * Gh / 3.0) + ut / 3.0 + 2.0 * ut3 / 3.0


@pytest.mark.parametrize("scheme", [2, 3])
@pytest.mark.parametrize("M", [1, 5])
def test_implicit_column_closed_form(scheme, M):
    rng = np.random.default_rng(17 + M + scheme)
    L, dt, nu_v, cd = 5, 900.0, 2.0e-2, 5.0e-3
    hk = np.array([50.0, 80.0, 120.0, 200.0, 300.0])
    U = rng.normal(0.0, 0.2, size=(L, 2))
    case = uniform_case(L=L, U=U, h_layers=hk, f0=0.0, scheme=scheme, M=M, dt=dt, nu_v=nu_v,
                        c_drag=cd, vmix=1)
    st = Setup.from_case(case)
    u, h = case.u.copy(), case.h.copy()
    ref = U.copy()
    for _ in range(4):
        u, h = S.step(u, h, st)
        ref = _column_step(scheme, ref, hk, nu_v, cd, dt)
    expect = case.mesh.normalEdge[:, :2] @ ref.T
    assert np.abs(u - expect).max() < 1e-13 * np.abs(U).max()
    assert np.abs(h - case.h).max() < 1e-13 * hk.max()
    # the mixing changed the answer: the explicit scheme gives another one
    ex = uniform_case(L=L, U=U, h_layers=hk, f0=0.0, scheme=scheme, M=M, dt=dt, nu_v=nu_v, c_drag=cd)
    ue, _ = S.step(ex.u.copy(), ex.h.copy(), Setup.from_case(ex))
    u1, _ = S.step(case.u.copy(), case.h.copy(), st)
    assert np.abs(ue - u1).max() > 1e-6 * np.abs(U).max()


# SSPRK2-SE grows on this oscillatory case after about a dozen steps (its
# stability polynomial exceeds one on the imaginary axis), with or without
# mixing, so it runs fewer steps.
@pytest.mark.parametrize("scheme,steps", [(2, 6), (3, 20)])
def test_volume_conserved_with_mixing(scheme, steps):
    case = cases.with_params(smooth_case(n=8, L=4, scheme=scheme), nu_v=1e-2, c_drag=2e-3, vmix=1)
    st = Setup.from_case(case)
    A = case.mesh.areaCell
    u, h = case.u.copy(), case.h.copy()
    v0 = (A[:, None] * h).sum()
    for _ in range(steps):
        u, h = S.step(u, h, st)
    assert abs((A[:, None] * h).sum() - v0) <= 1e-13 * v0


def test_lake_at_rest_with_mixing():
    case = uniform_case(L=4, scheme=3, nu_v=1e-2, c_drag=1e-3, vmix=1)
    st = Setup.from_case(case)
    u, h = case.u.copy(), case.h.copy()
    for _ in range(10):
        u, h = S.step(u, h, st)
    assert np.all(u == 0.0) and np.array_equal(h, case.h)
