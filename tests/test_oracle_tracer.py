"""Pins of the oracle's tracer (temperature) stages and the density they drive.

* A uniform tracer stays uniform (to rounding) through whole steps with
  bathymetry, flow, reconciliation and tracer diffusion: its fluxes are the
  thickness fluxes times the constant, so the tracer equation reduces to the
  thickness equation.  Also with isopycnal layers (per-layer constants).
* The tracer content sum_i A_i sum_k h T is conserved (flux form, no flux
  through the surface, the bottom or across coasts).
* With alpha = 0 the density never changes, and (u, h) equal those of the
  same run with the density frozen at rho0, bit for bit.
* Vertical diffusion of a lake at rest: every step is the textbook SSPRK of
  the column ODE dT/dt = A T with A the three-point diffusion matrix of the
  layer interfaces (no flux at the surface and the bottom).
* Horizontal diffusion of a temperature plane wave on the regular hex at rest:
  div(h kappa grad T) = h kappa lambda T with the closed-form eigenvalue of the
  hexagonal Laplacian, so every step multiplies T by the SSPRK stability
  polynomial R_p(kappa lambda dt).
* Vertical advection with centred interface values: for a temperature linear
  in the layer index, the tendency differs from T times the thickness tendency
  by exactly (b / 2)(w_k + w_{k+1}).
* Each baroclinic stage takes its density from that stage's temperature.
"""
import numpy as np
import pytest

from oracle import ssprk_se as S
from oracle.layered import Setup, T_h, eos, tracer_tendency, vertical_velocity
from synthetic import cases
from tests.helpers import smooth_case, uniform_case


def _tracer(case, **kw):
    kw.setdefault("tracer", 1)
    return cases.with_params(case, **kw)


def _run(case, T, steps):
    st = Setup.from_case(case)
    u, h = case.u.copy(), case.h.copy()
    for _ in range(steps):
        u, h, T = S.step(u, h, st, T=T)
    return u, h, T


@pytest.mark.parametrize("scheme,steps,vcoord", [(2, 5, 0), (3, 10, 0), (3, 8, 1)])
def test_uniform_tracer_stays_uniform(scheme, steps, vcoord):
    case = _tracer(smooth_case(n=10, L=5, scheme=scheme), kappa_h=50.0, kappa_v=1e-3, vcoord=vcoord)
    C, L = case.h.shape
    T0 = np.tile(10.0 + 2.0 * np.arange(L), (C, 1)) if vcoord == 1 else np.full((C, L), 12.5)
    if vcoord == 1:
        case = _tracer(case, kappa_v=0.0)      # per-layer constants: no vertical exchange
    u, h, T = _run(case, T0.copy(), steps)
    assert np.isfinite(u).all()
    assert np.abs(T - T0).max() <= 1e-12 * np.abs(T0).max()


@pytest.mark.parametrize("scheme,steps", [(2, 5), (3, 10)])
def test_tracer_content_conserved(scheme, steps):
    case = _tracer(cases.sphere_case(3, 6, 21, substeps=5, dt_btr=200.0), kappa_h=2e3, kappa_v=1e-3,
                   scheme=scheme)
    st = Setup.from_case(case)
    T0 = case.temp.copy()
    A = case.mesh.areaCell[:, None]
    c0 = (A * case.h * T0).sum()
    u, h, T = _run(case, T0, steps)
    assert np.isfinite(T).all()
    assert abs((A * h * T).sum() - c0) <= 1e-13 * abs(c0)
    assert np.abs(T - T0).max() > 1e-6          # the tracer did move


def test_alpha_zero_equals_frozen_density():
    base = smooth_case(n=8, L=4, scheme=3)
    C, L = base.h.shape
    frozen = cases.with_params(base)
    frozen.rho[...] = base.params.rho0
    st = Setup.from_case(frozen)
    u, h = frozen.u.copy(), frozen.h.copy()
    for _ in range(4):
        u, h = S.step(u, h, st)
    tr = _tracer(frozen, eos_alpha=0.0, kappa_h=10.0)
    T0 = np.random.default_rng(1).uniform(5, 20, size=(C, L))
    u2, h2, _ = _run(tr, T0, 4)
    assert np.array_equal(u, u2) and np.array_equal(h, h2)


def _textbook(scheme, x, dt, A):
    x1 = x + dt * A @ x
    if scheme == 2:
        return 0.5 * x + 0.5 * (x1 + dt * A @ x1)
    x2 = 0.75 * x + 0.25 * (x1 + dt * A @ x1)
    return x / 3.0 + 2.0 * (x2 + dt * A @ x2) / 3.0


@pytest.mark.parametrize("scheme", [2, 3])
def test_vertical_diffusion_of_a_lake_at_rest(scheme):
    hk = np.array([30.0, 50.0, 80.0, 140.0])
    L, kv, dt = 4, 5e-3, 600.0
    case = _tracer(uniform_case(L=L, h_layers=hk, scheme=scheme, dt=dt), kappa_v=kv, eos_alpha=2e-4)
    C = case.h.shape[0]
    Tcol = np.array([20.0, 15.0, 9.0, 4.0])
    A = np.zeros((L, L))
    for k in range(1, L):
        g = kv / (0.5 * (hk[k - 1] + hk[k]))   # interface k between layers k-1 and k
        A[k - 1, k - 1] -= g / hk[k - 1]
        A[k - 1, k] += g / hk[k - 1]
        A[k, k] -= g / hk[k]
        A[k, k - 1] += g / hk[k]
    u, h, T = case.u.copy(), case.h.copy(), np.tile(Tcol, (C, 1))
    st = Setup.from_case(case)
    ref = Tcol.copy()
    for _ in range(3):
        u, h, T = S.step(u, h, st, T=T)
        ref = _textbook(scheme, ref, dt, A)
    assert np.all(u == 0.0)
    assert np.abs(T - ref).max() <= 1e-12 * np.abs(ref).max()


@pytest.mark.parametrize("scheme", [2, 3])
def test_horizontal_diffusion_plane_wave(scheme):
    from synthetic.mesh import planar_hex
    dc, kh, dt, L = 1.0e4, 400.0, 3600.0, 2
    mesh = planar_hex(12, 12, dc, f0=0.0)
    k = 2 * np.pi * np.array([2 / mesh.Lx, 1 / mesh.Ly])
    case = _tracer(uniform_case(L=L, mesh=mesh, scheme=scheme, dt=dt, f0=0.0), kappa_h=kh, eos_alpha=0.0)
    T0 = 10.0 + np.cos(mesh.xCell[:, :2] @ k)[:, None] * np.array([1.0, 0.5])[None, :]
    dirs = dc * np.array([[1.0, 0.0], [0.5, np.sqrt(3) / 2], [-0.5, np.sqrt(3) / 2]])
    lam = 4.0 / (3.0 * dc ** 2) * np.sum(np.cos(dirs @ k) - 1.0)
    z = kh * lam * dt
    R = 1 + z + z * z / 2 + (z ** 3 / 6 if scheme == 3 else 0.0)
    _, _, T = _run(case, T0.copy(), 3)
    expect = 10.0 + (T0 - 10.0) * R ** 3
    assert np.abs(T - expect).max() <= 1e-12 * 10.0


def test_density_follows_the_eos_each_stage():
    """The first baroclinic stage sees eos(T^n); a step from a temperature whose
    EOS equals the frozen density reproduces the frozen run's first stage."""
    case = cases.c1(n=8, L=6, steps=1)
    st = Setup.from_case(case)
    assert np.allclose(eos(case.temp, st), case.rho, rtol=0, atol=1e-12)
    d1, d2 = {}, {}
    S.step(case.u.copy(), case.h.copy(), st, diag=d1)
    S.step(case.u.copy(), case.h.copy(), st, diag=d2, T=case.temp.copy())
    assert np.array_equal(d1["G0"], d2["G0"]) and np.array_equal(d1["ut1"], d2["ut1"])


@pytest.mark.parametrize("scheme", [2, 3])
def test_advection_of_a_plane_wave_by_uniform_flow(scheme):
    """Uniform flow U on the regular hex (f = 0, flat, uniform layers) stays
    steady; a temperature wave exp(i k.x) is advected by the centred flux
    with the closed-form eigenvalue -i omega, omega = 2/(3 d^2) sum_j
    (U.delta_j) sin(k.delta_j) over the three neighbour directions, so each
    step multiplies it by R_p(-i omega dt)."""
    from synthetic.mesh import planar_hex
    dc, dt, L = 1.0e4, 400.0, 2
    mesh = planar_hex(12, 12, dc, f0=0.0)
    U = np.array([[0.3, 0.1], [0.3, 0.1]])
    k = 2 * np.pi * np.array([3 / mesh.Lx, 2 / mesh.Ly])
    case = _tracer(uniform_case(L=L, U=U, mesh=mesh, scheme=scheme, dt=dt, f0=0.0, nu_h=0.0), eos_alpha=0.0)
    phase = mesh.xCell[:, :2] @ k
    T0 = 10.0 + np.cos(phase)[:, None] * np.ones(L)[None, :]
    dirs = dc * np.array([[1.0, 0.0], [0.5, np.sqrt(3) / 2], [-0.5, np.sqrt(3) / 2]])
    omega = 2.0 / (3.0 * dc ** 2) * np.sum((dirs @ U[0]) * np.sin(dirs @ k))
    z = -1j * omega * dt
    R = 1 + z + z * z / 2 + (z ** 3 / 6 if scheme == 3 else 0.0)
    u, h, T = _run(case, T0.copy(), 3)
    expect = 10.0 + np.real(R ** 3 * np.exp(1j * phase))[:, None]
    assert np.abs(u - case.u).max() <= 1e-13
    assert np.abs(T - expect).max() <= 1e-11 * 10.0


def test_vertical_advection_of_a_linear_profile():
    """z-star, a divergent flow (so w is not zero), and a temperature that is
    horizontally uniform in each layer and linear in the layer index,
    T_k = a + b k: the horizontal flux of layer k carries exactly T_k times the
    thickness flux, and the centred interface values (T_k + T_{k+1}) / 2 leave
    tendency(h T)_k - T_k T^h_k = (b / 2)(w_k + w_{k+1}), w at the interfaces
    of layer k (zero through the surface and the bottom)."""
    case = _tracer(cases.sphere_case(3, 7, 41, substeps=4, dt_btr=200.0), kappa_h=0.0, kappa_v=0.0)
    st = Setup.from_case(case)
    rng = np.random.default_rng(3)
    C, L = case.h.shape
    h = case.h * (1.0 + 0.1 * rng.uniform(-1.0, 1.0, case.h.shape))
    v = np.where(st.edge_mask[:, None], rng.normal(0.0, 0.2, case.u.shape), 0.0)
    a, b = 11.0, -0.75
    T = np.tile(a + b * np.arange(L, dtype=float), (C, 1))
    tend = tracer_tendency(h, T, v, st)
    w = vertical_velocity(h, v, st)
    expect = T * T_h(h, v, st) + 0.5 * b * (w[:, :-1] + w[:, 1:])
    wet = st.cell_mask.astype(bool)
    scale = np.abs(tend[wet]).max()
    assert np.abs(w[wet]).max() > 0
    assert np.abs(tend[wet] - expect[wet]).max() <= 1e-11 * scale


@pytest.mark.parametrize("scheme", [2, 3])
def test_later_stages_see_the_density_of_their_own_temperature(scheme):
    """Every baroclinic stage takes its density from the temperature of that
    stage (the stage's thickness and tracer content), not from the step's
    initial temperature: the second stage's G-bar equals Algorithm 1 run on
    the stage-1 state with rho = eos(T of stage 1)."""
    case = _tracer(cases.c1(n=8, L=6, steps=1), scheme=scheme, kappa_h=20.0, kappa_v=1e-4, eos_alpha=2e-3)
    st = Setup.from_case(case)
    d = {}
    S.step(case.u.copy(), case.h.copy(), st, diag=d, T=case.temp.copy())
    T1 = d["T1"]
    assert np.abs(T1 - case.temp).max() > 1e-6            # the temperature moved in stage 1
    st1 = Setup.from_case(case)
    st1.rho = eos(T1, st)
    u1 = S.mask_edges(d["ub1"][:, None] + d["ut1"], st)
    _, G1 = S.baroclinic_feuler(u1, d["ut1"], d["zeta1"], d["h1"], case.params.dt, st1)
    assert np.array_equal(G1, d["G1"])
