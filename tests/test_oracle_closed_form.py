"""Closed-form pins of the oracle's whole SSPRK2-SE / SSPRK3-SE step.

* Inertial oscillation (f-plane, horizontally uniform layers, no viscosity):
  every spatial operator vanishes except the Coriolis term, G-bar = 0, and
  the step multiplies the complex baroclinic velocity by R_p(-i f dt) and the
  barotropic one by R_p(-i f dt / M)^M, with R_2(z) = 1 + z + z^2/2 and
  R_3 = R_2 + z^3/6 (the SSPRK2/SSPRK3 stability polynomials of (SSPRK2),
  (SSPRK3)).  Fixes every stage coefficient of the baroclinic stages and of
  Algorithms 3 and 4.
* Proposition 1: the Delta t^3 coefficient of the Algorithm 3 output, from the
  exact rational expansion of R_2(z/M)^M, is (M^2-1)/(6M^2); the printed
  (M^2-1)/(3M^2) cannot be right because M -> infinity must give the exact
  Taylor coefficient 1/6.
* f = 0 with vertical viscosity and bottom drag on uniform layers: the whole
  SE step reduces to the textbook SSPRK2 / SSPRK3 of the column ODE for any M,
  which fixes the Interp_2 / Interp_3 weights and the G-bar coupling.
* Vertical viscosity of a linear profile: interior layers feel nothing, the top
  and bottom layers feel the boundary fluxes (D_{z^m}(nu_v D_{z^t} u)).
"""
from fractions import Fraction

import numpy as np
import pytest

from oracle import ssprk_se as S
from oracle.layered import D_u, Setup
from tests.helpers import uniform_case


def _R(scheme, z):
    r = 1 + z + z * z / 2
    return r if scheme == 2 else r + z ** 3 / 6


@pytest.mark.parametrize("scheme", [2, 3])
@pytest.mark.parametrize("M", [1, 3, 8])
def test_inertial_oscillation_closed_form(scheme, M):
    rng = np.random.default_rng(11 + M + scheme)
    L, f, dt = 4, 1.0e-4, 600.0
    U = rng.normal(0.0, 0.1, size=(L, 2))
    case = uniform_case(L=L, U=U, f0=f, scheme=scheme, M=M, dt=dt)
    st = Setup.from_case(case)
    u, h = case.u.copy(), case.h.copy()
    hk = case.h[0]
    W = U[:, 0] + 1j * U[:, 1]
    for _ in range(3):
        u, h = S.step(u, h, st)
        Wbar = (hk * W).sum() / hk.sum()
        Wt = W - Wbar
        z = -1j * f * dt
        W = _R(scheme, z) * Wt + _R(scheme, z / M) ** M * Wbar
    expect = np.outer(case.mesh.normalEdge[:, 0], W.real) + np.outer(case.mesh.normalEdge[:, 1], W.imag)
    assert np.abs(u - expect).max() < 1e-13 * np.abs(U).max()
    assert np.abs(h - case.h).max() < 1e-13 * hk.max()


def _poly_mul(a, b):
    out = [Fraction(0)] * (len(a) + len(b) - 1)
    for i, x in enumerate(a):
        for j, y in enumerate(b):
            out[i + j] += x * y
    return out


@pytest.mark.parametrize("M", [1, 2, 3, 5, 16, 64])
def test_proposition1_cubic_coefficient(M):
    a = [Fraction(1), Fraction(1, M), Fraction(1, 2 * M * M)]     # R_2(z/M) in powers of z
    p = [Fraction(1)]
    for _ in range(M):
        p = _poly_mul(p, a)
    p = p + [Fraction(0)] * 4
    assert p[1] == 1 and p[2] == Fraction(1, 2)
    assert p[3] == Fraction(M * M - 1, 6 * M * M)
    if M > 1:
        assert p[3] != Fraction(M * M - 1, 3 * M * M)


def _column_rhs(U, hk, nu_v, c_drag):
    """dU_k/dt of horizontally uniform 2-vectors U_k under vertical viscosity + drag."""
    L = len(hk)
    tau = np.zeros((L + 1, 2))
    for k in range(1, L):
        tau[k] = nu_v * (U[k - 1] - U[k]) / (0.5 * (hk[k - 1] + hk[k]))
    tau[L] = c_drag * np.linalg.norm(U[L - 1]) * U[L - 1]
    return (tau[:-1] - tau[1:]) / hk[:, None]


def _textbook_ssprk(scheme, U, dt, F):
    u1 = U + dt * F(U)
    if scheme == 2:
        return 0.5 * U + 0.5 * (u1 + dt * F(u1))
    u2 = 0.75 * U + 0.25 * (u1 + dt * F(u1))
    return U / 3.0 + 2.0 * (u2 + dt * F(u2)) / 3.0


@pytest.mark.parametrize("scheme", [2, 3])
@pytest.mark.parametrize("M", [1, 5])
def test_viscous_column_reduces_to_textbook_ssprk(scheme, M):
    rng = np.random.default_rng(3 + M)
    L, dt, nu_v, cd = 5, 900.0, 2.0e-2, 5.0e-3
    hk = np.array([50.0, 80.0, 120.0, 200.0, 300.0])
    U = rng.normal(0.0, 0.2, size=(L, 2))
    case = uniform_case(L=L, U=U, h_layers=hk, f0=0.0, scheme=scheme, M=M, dt=dt, nu_v=nu_v, c_drag=cd)
    st = Setup.from_case(case)
    u, h = case.u.copy(), case.h.copy()
    ref = U.copy()
    for _ in range(4):
        u, h = S.step(u, h, st)
        ref = _textbook_ssprk(scheme, ref, dt, lambda V: _column_rhs(V, hk, nu_v, cd))
    expect = case.mesh.normalEdge[:, :2] @ ref.T
    assert np.abs(u - expect).max() < 1e-13 * np.abs(U).max()


def test_vertical_viscosity_linear_profile():
    L, nu_v, a = 6, 1.0e-3, 0.01
    hk = np.full(L, 20.0)
    U = np.stack([a * np.arange(L), np.zeros(L)], 1)
    case = uniform_case(L=L, U=U, h_layers=hk, nu_v=nu_v, c_drag=0.0)
    st = Setup.from_case(case)
    du = D_u(case.u, case.h, st)
    nx = case.mesh.normalEdge[:, 0]
    flux = nu_v * (-a) / 20.0                  # nu_v (u_{k-1} - u_k) / h, uniform
    expect = np.zeros(L)
    expect[0] = (0.0 - flux) / 20.0
    expect[-1] = (flux - 0.0) / 20.0
    np.testing.assert_allclose(du, np.outer(nx, expect), atol=1e-18)
