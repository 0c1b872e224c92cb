"""Pins of the oracle's biharmonic horizontal viscosity -nu_h lap(lap u).

On the regular periodic hex both halves of the TRiSK vector Laplacian have
plane-wave eigenvalues that follow from the geometry alone (d the cell
spacing, A_i = (sqrt 3 / 2) d^2, l = d / sqrt 3, dual triangles of area
(sqrt 3 / 4) d^2):

* a gradient field u = grad(phi), phi = cos(k.x) at cells: div u = lambda phi
  with lambda = 4/(3 d^2) sum_j (cos(k.delta_j) - 1) over the three neighbour
  directions, curl u = 0, so lap u = lambda u and lap(lap u) = lambda^2 u;
* a rotational field u = (psi_v2 - psi_v1) / l with psi at vertices: div u = 0
  and lap u = -k x grad(curl u) = mu u when psi is an eigenvector of the
  vertex (honeycomb) graph Laplacian (4/d^2) sum_nb (psi_nb - psi_v).  The
  honeycomb has two sublattices; with delta'_j the three neighbour vectors of
  a sublattice-A vertex and S(k) = sum_j exp(i k.delta'_j), the Bloch vector
  psi_A = cos(k.x), psi_B = cos(k.x - arg S) has mu = 4/d^2 (|S| - 3), so
  lap(lap u) = mu^2 u.

Plus: the operator is self-adjoint and positive semidefinite in the l d
weighted inner product (so -nu lap(lap u) dissipates energy), uniform flow
feels nothing, and whole steps with it conserve volume and keep a lake at
rest.
"""
import numpy as np
import pytest

from oracle import ssprk_se as S
from oracle import trisk
from oracle.layered import Setup, horizontal_viscosity
from synthetic import cases
from synthetic.mesh import planar_hex
from tests.helpers import smooth_case, uniform_case

DC = 1.0e4


def _wave(n, a, b):
    m = planar_hex(n, n, DC)
    return m, 2 * np.pi * np.array([a / m.Lx, b / m.Ly])


@pytest.mark.parametrize("a,b", [(1, 0), (0, 1), (2, 3), (5, 2)])
def test_gradient_wave_eigenvalue(a, b):
    m, k = _wave(12, a, b)
    phi = np.cos(m.xCell[:, :2] @ k)
    u = trisk.gradient(phi, m)[:, None]
    dirs = DC * np.array([[1.0, 0.0], [0.5, np.sqrt(3) / 2], [-0.5, np.sqrt(3) / 2]])
    lam = 4.0 / (3.0 * DC ** 2) * np.sum(np.cos(dirs @ k) - 1.0)
    lap = trisk.laplacian(u, m)
    scale = np.abs(lam * u).max()
    assert np.abs(lap - lam * u).max() <= 1e-12 * scale
    lap2 = trisk.laplacian(lap, m)
    assert np.abs(lap2 - lam ** 2 * u).max() <= 1e-12 * lam ** 2 * np.abs(u).max()


def _vertex_neighbour_vectors(m, v):
    out = []
    for e in np.nonzero((m.verticesOnEdge == v).any(1))[0]:
        w = m.verticesOnEdge[e, 1] if m.verticesOnEdge[e, 0] == v else m.verticesOnEdge[e, 0]
        d = m.xVertex[w, :2] - m.xVertex[v, :2]
        d[0] -= m.Lx * np.round(d[0] / m.Lx)
        d[1] -= m.Ly * np.round(d[1] / m.Ly)
        out.append(d)
    return np.array(out)


@pytest.mark.parametrize("a,b", [(1, 0), (1, 1), (0, 2), (3, 2)])
def test_rotational_wave_eigenvalue(a, b):
    m, k = _wave(12, a, b)
    dA = _vertex_neighbour_vectors(m, 0)
    assert dA.shape == (3, 2) and np.allclose(np.linalg.norm(dA, axis=1), DC / np.sqrt(3))
    S_k = np.exp(1j * (dA @ k)).sum()
    # sublattice of every vertex: its neighbour vectors are those of vertex 0 (A) or their negatives (B)
    sub_b = np.array([np.allclose(np.sort(_vertex_neighbour_vectors(m, v), 0), np.sort(-dA, 0), atol=1e-6)
                      for v in range(m.nVertices)])
    assert 0 < sub_b.sum() < m.nVertices
    phase = m.xVertex[:, :2] @ k - np.where(sub_b, np.angle(S_k), 0.0)
    psi = np.cos(phase)
    v1, v2 = m.verticesOnEdge[:, 0], m.verticesOnEdge[:, 1]
    u = ((psi[v2] - psi[v1]) / m.dvEdge)[:, None]
    mu = 4.0 / DC ** 2 * (abs(S_k) - 3.0)
    assert np.abs(trisk.divergence(u, m)).max() <= 1e-12 * np.abs(u).max() / DC
    lap = trisk.laplacian(u, m)
    assert np.abs(lap - mu * u).max() <= 1e-11 * np.abs(mu * u).max()
    lap2 = trisk.laplacian(lap, m)
    assert np.abs(lap2 - mu ** 2 * u).max() <= 1e-11 * mu ** 2 * np.abs(u).max()


@pytest.mark.parametrize("sphere", [False, True])
def test_self_adjoint_and_dissipative(sphere):
    if sphere:
        c = cases.sphere_case(3, 3, 11, substeps=4, dt_btr=60.0, land_fraction=0.0)
    else:
        c = smooth_case(n=10, L=3)
    m = c.mesh
    rng = np.random.default_rng(3)
    u, w = rng.normal(size=(m.nEdges, 3)), rng.normal(size=(m.nEdges, 3))
    ld = (m.dvEdge * m.dcEdge)[:, None]
    lap = lambda x: trisk.laplacian(x, m)
    a, b = (ld * u * lap(lap(w))).sum(), (ld * lap(lap(u)) * w).sum()
    assert abs(a - b) <= 1e-11 * max(abs(a), abs(b))
    e = (ld * u * lap(lap(u))).sum(0)
    assert np.all(e > 0)
    assert np.allclose(e, (ld * lap(u) ** 2).sum(0), rtol=1e-11)


def test_uniform_flow_feels_nothing():
    c = uniform_case(L=3, U=np.array([[0.3, -0.2], [0.1, 0.4], [-0.2, 0.0]]), nu_h=1e12, hdiff=1)
    st = Setup.from_case(c)
    assert np.abs(horizontal_viscosity(c.u, st)).max() <= 1e-13 * 1e12 * 0.4 / DC ** 4


def test_hyperviscosity_term_sign_and_masking():
    c = cases.with_params(cases.sphere_case(3, 3, 12, substeps=4, dt_btr=60.0), nu_h=1e15, hdiff=1)
    st = Setup.from_case(c)
    rng = np.random.default_rng(2)
    u = np.where(st.edge_mask[:, None], rng.normal(size=c.u.shape), 0.0)
    hv = horizontal_viscosity(u, st)
    from oracle.layered import mask_edges
    inner = mask_edges(trisk.laplacian(u, c.mesh), st)
    assert np.array_equal(hv, -1e15 * trisk.laplacian(inner, c.mesh))
    assert np.any(inner[~st.edge_mask] == 0.0) and np.all(inner[~st.edge_mask] == 0.0)


@pytest.mark.parametrize("scheme,steps", [(2, 6), (3, 20)])
def test_volume_conserved_with_del4(scheme, steps):
    case = cases.with_params(smooth_case(n=8, L=4, scheme=scheme), nu_h=1e11, hdiff=1)
    st = Setup.from_case(case)
    A = case.mesh.areaCell
    u, h = case.u.copy(), case.h.copy()
    v0 = (A[:, None] * h).sum()
    for _ in range(steps):
        u, h = S.step(u, h, st)
    assert np.isfinite(u).all()
    assert abs((A[:, None] * h).sum() - v0) <= 1e-13 * v0


def test_lake_at_rest_with_del4():
    case = uniform_case(L=4, scheme=3, nu_h=1e12, hdiff=1)
    st = Setup.from_case(case)
    u, h = case.u.copy(), case.h.copy()
    for _ in range(10):
        u, h = S.step(u, h, st)
    assert np.all(u == 0.0) and np.array_equal(h, case.h)
