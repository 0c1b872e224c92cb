"""Pins of the oracle's layered terms whose discrete forms the paper leaves
to readings (pressure gradient in z-star layers, z-star vertical velocity,
vertical boundary fluxes, vorticity flux, barotropic thickness at edges).
Each is checked against something the readings do not assume:

* pressure gradient: exactly -g (rho / rho0) grad zeta for a uniform density
  over bathymetry (the hydrostatic pressure plus the layer-midpoint height is
  g rho zeta in every layer); exactly the hydrostatic integral of a linear
  horizontal density gradient for flat layers, and over a sloping bottom,
  where the density at the edge (the mean of the two cells) enters;
* z-star: every layer's thickness tendency is the same fraction of its
  reference thickness, the column tendencies add up to minus the column flux
  divergence, and w vanishes at the bottom and, to roundoff, at the surface;
* vertical boundary fluxes: the column budget sum_k h_k D^u_k is exactly
  the bottom drag (no surface stress, interior fluxes telescope), and the drag
  speed of a uniform flow is |U| of the lowest layer;
* vorticity flux: converges at second order to -(k . curl U) k x U for a
  smooth flow (sign and factors); a steady parallel shear flow, where the
  vorticity flux balances the kinetic-energy gradient, gets a tendency that
  vanishes at second order;
* barotropic thickness at edges: the mean of zeta + H of the two cells is the
  column sum of the layer thicknesses at the edge (reading c9 against c2).
"""
from dataclasses import replace

import numpy as np
import pytest

from oracle import ssprk_se as S
from oracle import trisk
from oracle.layered import (D_u, Setup, T_h, T_u, bottom_speed, pressure_gradient_force,
                            thickness_flux_divergence, vertical_velocity)
from synthetic import cases
from synthetic.mesh import planar_hex
from tests.helpers import smooth_case, uniform_case


def _interior_edges(m):
    c = m.xCell[m.cellsOnEdge]
    return (np.abs(c[:, 1] - c[:, 0]).max(1) < 2 * m.dc)


def _perturbed(case, seed):
    """Random positive layer thicknesses and a random masked velocity."""
    rng = np.random.default_rng(seed)
    st = Setup.from_case(case)
    h = case.h * (1.0 + 0.2 * rng.uniform(-1.0, 1.0, case.h.shape))
    u = np.where(st.edge_mask[:, None], rng.normal(0.0, 0.3, case.u.shape), 0.0)
    return st, h, u


@pytest.mark.parametrize("rho_u", [1025.0, 1031.5])
def test_pgf_of_uniform_density_is_minus_g_grad_zeta(rho_u):
    case = smooth_case(n=8, L=6)
    case.rho[:] = rho_u
    st, h, _ = _perturbed(case, 11)
    zeta = h.sum(1) - case.H
    c1, c2 = case.mesh.cellsOnEdge[:, 0], case.mesh.cellsOnEdge[:, 1]
    ref = -case.params.gravity * (rho_u / case.params.rho0) * (zeta[c2] - zeta[c1]) / case.mesh.dcEdge
    pgf = pressure_gradient_force(h, st)
    scale = np.abs(ref).max()
    assert scale > 0
    for k in range(h.shape[1]):
        assert np.abs(pgf[:, k] - ref).max() <= 1e-11 * scale, k


def test_pgf_of_a_horizontal_density_gradient_in_flat_layers():
    hk = np.array([40.0, 70.0, 120.0, 200.0])
    case = uniform_case(L=4, h_layers=hk, n=8)
    m = case.mesh
    a = np.array([[2e-6, -1e-6], [1e-6, 3e-6], [-2e-6, 1e-6], [4e-6, 2e-6]])   # d rho_k / d(x, y)
    case.rho[:] = case.params.rho0 + m.xCell[:, :2] @ a.T
    st = Setup.from_case(case)
    pgf = pressure_gradient_force(case.h, st)
    an = m.normalEdge[:, :2] @ a.T                      # d rho_k / dn at every edge
    ref = np.zeros_like(pgf)
    for k in range(4):
        ref[:, k] = -(case.params.gravity / case.params.rho0) * (
            (an[:, :k] * hk[:k]).sum(1) + an[:, k] * 0.5 * hk[k])
    ok = _interior_edges(m)                              # the linear density does not wrap around
    assert ok.sum() > m.nEdges // 2
    # rho h ~ 1e5 against differences ~ 1: roundoff is ~1e-11 of the result
    assert np.abs(pgf[ok] - ref[ok]).max() <= 1e-10 * np.abs(ref[ok]).max()


def test_pgf_of_density_gradients_over_a_sloping_bottom():
    """Layers of uniform thickness over a linear bottom slope, each with its own
    linear horizontal density gradient: the layer mid-depths all follow the
    bottom, z_k = -H + sum_{l>k} h_l + h_k / 2, and the hydrostatic pressure at
    them is p_k = g (sum_{l<k} rho_l h_l + rho_k h_k / 2), so the force is
    -(g / rho0) [sum_{l<k} h_l drho_l/dn + h_k/2 drho_k/dn - rho_k dH/dn] with
    rho_k taken at the edge.  For linear fields the centred differences are
    exact and rho at the edge is the mean of the two cells, so this holds to
    roundoff at every edge that does not wrap around the periodic domain."""
    hk = np.array([40.0, 70.0, 120.0, 200.0])
    case = uniform_case(L=4, h_layers=hk, n=8)
    m = case.mesh
    a = np.array([[2e-6, -1e-6], [1e-6, 3e-6], [-2e-6, 1e-6], [4e-6, 2e-6]])   # d rho_k / d(x, y)
    slope = np.array([1.5e-3, -0.8e-3])                                          # dH / d(x, y)
    case.rho[:] = case.params.rho0 + m.xCell[:, :2] @ a.T
    case.H[:] = hk.sum() + 60.0 + m.xCell[:, :2] @ slope
    st = Setup.from_case(case)
    pgf = pressure_gradient_force(case.h, st)
    an = m.normalEdge[:, :2] @ a.T                      # d rho_k / dn at every edge
    Hn = m.normalEdge[:, :2] @ slope                    # dH / dn
    c1, c2 = m.cellsOnEdge[:, 0], m.cellsOnEdge[:, 1]
    xe = 0.5 * (m.xCell[c1, :2] + m.xCell[c2, :2])      # edge midpoints (interior edges)
    rho_e = case.params.rho0 + xe @ a.T
    g, rho0 = case.params.gravity, case.params.rho0
    ref = np.zeros_like(pgf)
    for k in range(4):
        ref[:, k] = -(g / rho0) * ((an[:, :k] * hk[:k]).sum(1) + an[:, k] * 0.5 * hk[k] - rho_e[:, k] * Hn)
    ok = _interior_edges(m)
    assert ok.sum() > m.nEdges // 2
    assert np.abs(pgf[ok] - ref[ok]).max() <= 1e-10 * np.abs(ref[ok]).max()


def test_zstar_layers_stretch_in_proportion():
    case = cases.sphere_case(3, 7, 4451, substeps=4, dt_btr=200.0)
    st, h, u = _perturbed(case, 12)
    th = T_h(h, u, st)
    wet = st.cell_mask.astype(bool)
    ratio = th[wet] / st.h_ref[wet]
    np.testing.assert_allclose(ratio, np.repeat(ratio[:, :1], h.shape[1], axis=1), rtol=1e-12, atol=0)
    div = thickness_flux_divergence(h, u, st)
    col = np.abs(div[wet]).sum(1)
    assert np.abs(th[wet].sum(1) + div[wet].sum(1)).max() <= 1e-12 * col.max()
    w = vertical_velocity(h, u, st)
    assert np.all(w[:, -1] == 0.0)                       # no flux through the bottom
    assert np.all(np.abs(w[wet, 0]) <= 1e-12 * col)      # none through the surface, to roundoff
    # and w is the one the layer thickness equation dh_k/dt = -div_k - (w_k - w_{k+1})
    # gives for this T^h: the momentum and tracer equations move with the same w
    dw = w[:, :-1] - w[:, 1:]
    assert np.abs(dw[wet] + div[wet] + th[wet]).max() <= 1e-12 * col.max()


def test_vertical_boundary_fluxes_close_the_column_budget():
    case = cases.with_params(smooth_case(n=8, L=7), nu_v=3e-2, c_drag=4e-3)
    st, h, u = _perturbed(case, 13)
    he = trisk.cell_to_edge(h, case.mesh)
    budget = (he * D_u(u, h, st)).sum(1)
    drag = -case.params.c_drag * bottom_speed(u, st) * u[:, -1]
    ok = st.edge_mask.astype(bool)
    scale = np.abs(he * D_u(u, h, st)).sum(1).max()
    assert np.abs(budget[ok] - drag[ok]).max() <= 1e-12 * scale
    assert np.all(budget[~ok] == 0.0)


def test_drag_speed_of_a_uniform_flow_is_the_bottom_speed():
    U = np.array([[0.3, -0.1], [0.05, 0.2], [-0.4, 0.25]])
    case = uniform_case(L=3, U=U)
    st = Setup.from_case(case)
    np.testing.assert_allclose(bottom_speed(case.u, st), np.linalg.norm(U[-1]), rtol=1e-14)


def test_vorticity_flux_converges_to_the_continuous_term():
    errs = []
    for n in (16, 32, 64):
        m = planar_hex(n, n, 1.0e4 * 16 / n)
        kx, ky = 2 * np.pi / m.Lx, 2 * np.pi / m.Ly
        A, B = 0.7, -0.4
        xe, ye = m.xEdge[:, 0], m.xEdge[:, 1]
        U = np.stack([A * np.sin(ky * ye), B * np.sin(kx * xe)], -1)
        zeta = B * kx * np.cos(kx * xe) - A * ky * np.cos(ky * ye)
        u = np.einsum("ej,ej->e", U, m.normalEdge[:, :2])
        vort = trisk.tangential_flux(trisk.vorticity_on_edges(trisk.curl(u, m), m), u, m)
        # normal component of -zeta k x U is zeta times the tangential component (t = k x n)
        ref = zeta * np.einsum("ej,ej->e", U, m.tangentEdge[:, :2])
        errs.append(np.linalg.norm(vort - ref) / np.linalg.norm(ref))
    assert errs[-1] < 5e-3
    assert errs[0] / errs[1] > 3.5 and errs[1] / errs[2] > 3.5     # second order


def test_steady_shear_flow_has_no_tendency():
    rates = []
    for n in (16, 32, 64):
        m = planar_hex(n, n, 1.0e4 * 16 / n, f0=0.0)
        case = uniform_case(L=3, mesh=m, nu_h=0.0, f0=0.0)
        kx, B = 2 * np.pi / m.Lx, 0.5
        xe = m.xEdge[:, 0]
        U = np.stack([np.zeros_like(xe), B * np.sin(kx * xe)], -1)
        u = np.repeat(np.einsum("ej,ej->e", U, m.normalEdge[:, :2])[:, None], 3, axis=1)
        case = replace(case, u=u)
        t = T_u(u, case.h, Setup.from_case(case))
        rates.append(np.abs(t).max() / (B * B * kx))      # each term alone is of size B^2 kx
    assert rates[-1] < 5e-4
    assert rates[0] / rates[1] > 3.5 and rates[1] / rates[2] > 3.5


def test_barotropic_thickness_at_edges_is_the_layer_sum():
    case = cases.sphere_case(3, 6, 4452, substeps=4, dt_btr=200.0)
    st, h, u = _perturbed(case, 14)
    ubar, _ = S.split(u, h, st)
    flux = S.barotropic_flux(ubar, S.ssh(h, st), st)
    ref = np.where(st.edge_mask, ubar * trisk.cell_to_edge(h, case.mesh).sum(1), 0.0)
    assert np.abs(flux - ref).max() <= 1e-13 * np.abs(ref).max()
