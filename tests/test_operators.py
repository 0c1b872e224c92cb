"""Pins of the oracle's TRiSK operators against exact properties.

* linear fields: exact normal gradients, divergence and curl (midpoint rule is
  exact for linear integrands on straight edges);
* uniform flow on the regular hexagon: exact tangential reconstruction and
  kinetic energy |U|^2 / 2;
* energy neutrality of the weights and W(curl psi) = grad(R psi) (Thuburn et
  al. 2009), on the hexagon and on the sphere (pentagons included).
"""
import numpy as np

from oracle import trisk
from synthetic.mesh import periodic_delta


def _interior_edges(m):
    """Edges whose two cells and two vertices do not straddle the periodic seam."""
    c = m.xCell[m.cellsOnEdge]
    v = m.xVertex[m.verticesOnEdge]
    ok = (np.abs(c[:, 1] - c[:, 0]).max(1) < 2 * m.dc) & (np.abs(v[:, 1] - v[:, 0]).max(1) < 2 * m.dc)
    return ok


def test_gradient_of_linear_field(hex16):
    m = hex16
    a = np.array([3.0e-5, -7.0e-5])
    phi = m.xCell[:, :2] @ a
    g = trisk.gradient(phi, m)
    ok = _interior_edges(m)
    np.testing.assert_allclose(g[ok], (m.normalEdge[:, :2] @ a)[ok], rtol=1e-12, atol=1e-18)


def _cells_away_from_seam(m):
    ring = m.xCell[np.where(m.cellsOnCell >= 0, m.cellsOnCell, 0)]
    d = np.abs(ring[:, :, :2] - m.xCell[:, None, :2]).max((1, 2))
    return d < 2 * m.dc


def test_divergence_and_curl_of_linear_flows(hex16):
    m = hex16
    x0 = np.array([m.Lx / 2, m.Ly / 2])
    # radial flow a (x - x0): divergence 2a, curl 0
    a, om = 2.0e-6, 3.0e-6
    rel = m.xEdge[:, :2] - x0
    u_rad = a * np.einsum("ij,ij->i", rel, m.normalEdge[:, :2])
    rot = om * np.stack([-rel[:, 1], rel[:, 0]], 1)                # solid-body rotation
    u_rot = np.einsum("ij,ij->i", rot, m.normalEdge[:, :2])
    inner = _cells_away_from_seam(m)
    np.testing.assert_allclose(trisk.divergence(u_rad, m)[inner], 2 * a, rtol=1e-10)
    np.testing.assert_allclose(trisk.divergence(u_rot, m)[inner], 0.0, atol=1e-15)
    vin = np.ones(m.nVertices, bool)
    for j in range(3):
        vin &= _interior_edges(m)[m.edgesOnVertex[:, j]]
    zr = trisk.curl(u_rot, m)
    assert (zr[vin] > 0).all()                                        # counter-clockwise -> positive
    np.testing.assert_allclose(zr[vin], 2 * om, rtol=1e-10)
    np.testing.assert_allclose(trisk.curl(u_rad, m)[vin], 0.0, atol=1e-15)


def test_uniform_flow_reconstruction_and_kinetic_energy(hex16):
    m = hex16
    U = np.array([0.37, -1.21, 0.0])
    u = m.normalEdge @ U
    v = trisk.tangential_flux(np.ones(m.nEdges), u, m)
    np.testing.assert_allclose(v, m.tangentEdge @ U, rtol=0, atol=1e-15)
    np.testing.assert_allclose(trisk.kinetic_energy(u, m), 0.5 * U @ U, rtol=1e-14)
    np.testing.assert_allclose(trisk.divergence(u, m), 0.0, atol=1e-16)
    np.testing.assert_allclose(trisk.curl(u, m), 0.0, atol=1e-16)
    np.testing.assert_allclose(trisk.laplacian(u, m), 0.0, atol=1e-20)


def test_energy_neutrality(hex16, sphere3):
    rng = np.random.default_rng(5)
    for m in (hex16, sphere3):
        u = rng.standard_normal(m.nEdges)
        q = rng.standard_normal(m.nEdges)
        for coef in (np.ones(m.nEdges), q):
            v = trisk.tangential_flux(coef, u, m)
            ref = (m.dvEdge * m.dcEdge * np.abs(u * v)).sum()
            assert abs((m.dvEdge * m.dcEdge * u * v).sum()) < 1e-13 * ref


def test_perp_maps_curls_to_gradients(hex16, sphere3):
    """W K psi = G (R psi): the Coriolis weights map every discrete
    divergence-free flow u_e = -(psi_v2 - psi_v1)/l_e to the gradient of the
    kite-weighted cell average sum_v (A_iv / A_i) psi_v (Thuburn et al. 2009;
    follows by summation by parts around each cell from the weight formula).
    """
    rng = np.random.default_rng(6)
    for m in (hex16, sphere3):
        psi = rng.standard_normal(m.nVertices)
        v1, v2 = m.verticesOnEdge[:, 0], m.verticesOnEdge[:, 1]
        u = -(psi[v2] - psi[v1]) / m.dvEdge
        np.testing.assert_allclose(trisk.divergence(u, m), 0.0, atol=1e-12 * np.abs(u).max() / m.dcEdge.min())
        psibar = np.zeros(m.nCells)
        for s in range(6):
            valid = s < m.nEdgesOnCell
            vv = np.where(valid, m.verticesOnCell[:, s], 0)
            psibar += np.where(valid, m.kiteAreasOnCell[:, s] * psi[vv], 0.0)
        psibar /= m.areaCell
        wu = trisk.tangential_flux(np.ones(m.nEdges), u, m)
        g = trisk.gradient(psibar, m)
        np.testing.assert_allclose(wu, g, rtol=0, atol=1e-12 * np.abs(g).max())


def test_periodic_delta(hex16):
    m = hex16
    d = periodic_delta(m, m.xCell[m.cellsOnEdge[:, 0]], m.xCell[m.cellsOnEdge[:, 1]])
    np.testing.assert_allclose(np.linalg.norm(d, axis=1), m.dcEdge, rtol=1e-12)
    np.testing.assert_allclose(d / m.dcEdge[:, None], m.normalEdge[:, :2], atol=1e-12)
