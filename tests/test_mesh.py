"""Pins of the synthetic meshes (entity counts, Euler characteristic, areas, kites).

The TRiSK tables are inputs to both the oracle and the library; these checks
fix them against closed-form facts of the two mesh families.
"""
import numpy as np
import pytest

from synthetic.mesh import icosahedral, planar_hex


@pytest.mark.parametrize("nx,ny", [(4, 4), (16, 16), (12, 8)])
def test_hex_counts_and_areas(nx, ny):
    dc = 1.0e4
    m = planar_hex(nx, ny, dc)
    C = nx * ny
    assert (m.nCells, m.nEdges, m.nVertices) == (C, 3 * C, 2 * C)
    assert m.nCells - m.nEdges + m.nVertices == 0           # torus: chi = 0
    s3 = np.sqrt(3.0)
    np.testing.assert_allclose(m.areaCell.sum(), m.Lx * m.Ly, rtol=1e-12)
    np.testing.assert_allclose(m.areaTriangle.sum(), m.Lx * m.Ly, rtol=1e-12)
    np.testing.assert_allclose(m.areaCell, s3 / 2 * dc * dc, rtol=1e-14)
    np.testing.assert_allclose(m.dvEdge, dc / s3, rtol=1e-14)
    np.testing.assert_allclose(m.kiteAreasOnCell / m.areaCell[:, None], 1.0 / 6.0, rtol=1e-14)
    np.testing.assert_allclose(m.kiteAreasOnVertex.sum(1), m.areaTriangle, rtol=1e-12)
    assert (m.nEdgesOnEdge == 10).all()


def _check_topology(m):
    C, E, V = m.nCells, m.nEdges, m.nVertices
    # every edge appears in exactly the two cells it separates
    cnt = np.zeros(E, int)
    for j in range(6):
        valid = j < m.nEdgesOnCell
        np.add.at(cnt, m.edgesOnCell[valid, j], 1)
    assert (cnt == 2).all()
    # every vertex is touched by three edges whose endpoints include it
    for j in range(3):
        e = m.edgesOnVertex[:, j]
        assert ((m.verticesOnEdge[e, 0] == np.arange(V)) | (m.verticesOnEdge[e, 1] == np.arange(V))).all()
    # edge ordering: slot m of a cell and slot m+1 share the vertex in slot m
    for j in range(6):
        valid = j < m.nEdgesOnCell
        ci = np.nonzero(valid)[0]
        n = m.nEdgesOnCell[ci]
        v = m.verticesOnCell[ci, j]
        ea, eb = m.edgesOnCell[ci, j], m.edgesOnCell[ci, (j + 1) % n]
        for e in (ea, eb):
            assert ((m.verticesOnEdge[e, 0] == v) | (m.verticesOnEdge[e, 1] == v)).all()
    # t = k x n points from v1 to v2
    d = m.xVertex[m.verticesOnEdge[:, 1]] - m.xVertex[m.verticesOnEdge[:, 0]]
    if m.kind == "planar":
        d[:, 0] -= m.Lx * np.round(d[:, 0] / m.Lx)
        d[:, 1] -= m.Ly * np.round(d[:, 1] / m.Ly)
    assert (np.einsum("ij,ij->i", d, m.tangentEdge) > 0).all()
    _ = C


def test_hex_topology(hex16):
    _check_topology(hex16)


@pytest.mark.parametrize("level", [1, 2, 3, 4])
def test_sphere_counts_and_areas(level):
    m = icosahedral(level, 1.0)
    n4 = 4 ** level
    assert (m.nCells, m.nEdges, m.nVertices) == (10 * n4 + 2, 30 * n4, 20 * n4)
    assert m.nCells - m.nEdges + m.nVertices == 2            # sphere: chi = 2
    np.testing.assert_allclose(m.areaCell.sum(), 4 * np.pi, rtol=1e-12)
    np.testing.assert_allclose(m.areaTriangle.sum(), 4 * np.pi, rtol=1e-12)
    np.testing.assert_allclose(m.kiteAreasOnCell.sum(1), m.areaCell, rtol=1e-12)
    np.testing.assert_allclose(m.kiteAreasOnVertex.sum(1), m.areaTriangle, rtol=1e-12)
    assert (m.nEdgesOnCell == 5).sum() == 12 and (m.nEdgesOnCell == 6).sum() == m.nCells - 12
    # Voronoi property: the primal edge is perpendicular to the dual edge
    dv = m.xVertex[m.verticesOnEdge[:, 1]] - m.xVertex[m.verticesOnEdge[:, 0]]
    cos = np.einsum("ij,ij->i", dv, m.normalEdge) / np.linalg.norm(dv, axis=1)
    assert np.abs(cos).max() < 1e-12
    _check_topology(m)


def test_weights_antisymmetric(hex16, sphere3):
    """l_e d_e W_{e,e'} = -l_e' d_e' W_{e',e} (Thuburn et al. 2009, energy neutrality)."""
    for m in (hex16, sphere3):
        for e in range(0, m.nEdges, max(1, m.nEdges // 97)):
            scale = np.abs(m.dvEdge[e] * m.dcEdge[e] * m.weightsOnEdge[e]).max()
            for j in range(m.nEdgesOnEdge[e]):
                ep = m.edgesOnEdge[e, j]
                back = np.nonzero(m.edgesOnEdge[ep, :m.nEdgesOnEdge[ep]] == e)[0]
                assert len(back) == 1
                a = m.dvEdge[e] * m.dcEdge[e] * m.weightsOnEdge[e, j]
                b = m.dvEdge[ep] * m.dcEdge[ep] * m.weightsOnEdge[ep, back[0]]
                assert abs(a + b) <= 1e-12 * scale
