"""Pins of the two T^u terms that no whole-step property fixes by itself:
the vertical advection of momentum \\bar(w D_{z^t}(u))^m and the horizontal
viscosity nu_h lap u (Section 2, the vertical operators and the grouping T^u;
the biharmonic form of the remark on horizontal dissipation as well).

Both are checked through ``T_u`` itself, so a wrong sign or factor where T_u
assembles them fails here:

* vertical advection: with u_k = (a + beta z_k) U.n in every layer (z_k the
  layer mid-depths), D_{z^t}(u) is exactly beta U.n at every interior
  interface, whatever the layer thicknesses, because mid-depths of adjacent
  layers lie \\bar(h)^t apart.  A horizontally uniform flow makes every other
  term of T^u vanish (uniform K, no curl, no pressure gradient over flat
  layers, no Laplacian).  With a prescribed uniform w the tendency of every
  interior layer is then exactly -w du/dz = -w beta U.n; with w varying in the
  vertical and between cells it is -beta U.n times the mean of the two edge
  interfaces of the layer, w at an edge being the mean of its two cells.
* viscosity: nu_h lap u is the only term of T^u that is odd in u (kinetic
  energy, vorticity flux and vertical advection are quadratic, the pressure
  gradient does not depend on u), so [T^u(u) - T^u(-u)] / 2 is exactly the
  viscosity.  For the plane waves whose eigenvalues the biharmonic pins fix in
  closed form (a gradient wave with eigenvalue lambda, a rotational Bloch wave
  with mu) it must equal nu_h lambda u and nu_h mu u, and -nu_h lambda^2 u,
  -nu_h mu^2 u for the biharmonic form; and for any velocity it must remove
  energy (negative l d weighted inner product with u).
"""
import numpy as np
import pytest

from oracle.layered import Setup, T_u
from synthetic import cases
from synthetic.mesh import planar_hex
from tests.helpers import uniform_case
from tests.test_oracle_del4 import DC, _vertex_neighbour_vectors, _wave

H_LAYERS = np.array([30.0, 50.0, 80.0, 120.0, 200.0, 320.0])
U_DIR = np.array([0.3, -0.2])
A0, BETA = 0.1, 2.0e-3


def _sheared_case():
    """Horizontally uniform flow, linear in depth: u_k = (A0 + BETA z_k) U_DIR . n."""
    hk = H_LAYERS
    z = -(np.concatenate([[0.0], np.cumsum(hk)[:-1]]) + 0.5 * hk)
    U = np.outer(A0 + BETA * z, U_DIR)
    case = uniform_case(L=len(hk), U=U, h_layers=hk, n=10)
    un = case.mesh.normalEdge[:, :2] @ U_DIR
    return case, un


def test_vertical_advection_of_a_uniform_w_is_minus_w_dudz():
    case, un = _sheared_case()
    st = Setup.from_case(case)
    L = case.params.n_layers
    W = 3.0e-4
    w = np.full((case.mesh.nCells, L + 1), W)
    t = T_u(case.u, case.h, st, w=w)
    ref = -W * BETA * un
    scale = np.abs(ref).max()
    for k in range(1, L - 1):
        assert np.abs(t[:, k] - ref).max() <= 1e-12 * scale, k
    # no flux through the surface and the bottom: only the inner interface acts
    assert np.abs(t[:, 0] - 0.5 * ref).max() <= 1e-12 * scale
    assert np.abs(t[:, L - 1] - 0.5 * ref).max() <= 1e-12 * scale


def test_vertical_advection_averages_the_layer_interfaces():
    case, un = _sheared_case()
    st = Setup.from_case(case)
    m, L = case.mesh, case.params.n_layers
    kx = 2 * np.pi / m.Lx
    prof = np.array([0.0, 1.0, -0.5, 2.0, 0.7, -1.2, 0.0]) * 1.0e-4
    w = (1.0 + 0.5 * np.cos(kx * m.xCell[:, 0]))[:, None] * prof[None, :]
    t = T_u(case.u, case.h, st, w=w)
    c1, c2 = m.cellsOnEdge[:, 0], m.cellsOnEdge[:, 1]
    w_e = 0.5 * (w[c1] + w[c2])
    ref = -BETA * un[:, None] * 0.5 * (w_e[:, :L] + w_e[:, 1:])
    assert np.abs(t - ref).max() <= 1e-12 * np.abs(ref).max()


def test_no_vertical_advection_without_shear():
    case, _ = _sheared_case()
    st = Setup.from_case(case)
    L = case.params.n_layers
    uni = np.repeat(case.u[:, :1], L, axis=1)
    w = np.full((case.mesh.nCells, L + 1), 3.0e-4)
    t = T_u(uni, case.h, st, w=w)
    assert np.abs(t).max() <= 1e-15 * np.abs(uni).max()


def _odd_part(u, case):
    st = Setup.from_case(case)
    return 0.5 * (T_u(u, case.h, st) - T_u(-u, case.h, st))


AMPS = np.array([0.02, -0.01, 0.005])


def _gradient_wave(a, b):
    m, k = _wave(12, a, b)
    phi = np.cos(m.xCell[:, :2] @ k)
    c1, c2 = m.cellsOnEdge[:, 0], m.cellsOnEdge[:, 1]
    u = ((phi[c2] - phi[c1]) / m.dcEdge)[:, None] * AMPS[None, :] * DC
    dirs = DC * np.array([[1.0, 0.0], [0.5, np.sqrt(3) / 2], [-0.5, np.sqrt(3) / 2]])
    lam = 4.0 / (3.0 * DC ** 2) * np.sum(np.cos(dirs @ k) - 1.0)
    return m, u, lam


def _rotational_wave(a, b):
    m, k = _wave(12, a, b)
    dA = _vertex_neighbour_vectors(m, 0)
    S_k = np.exp(1j * (dA @ k)).sum()
    sub_b = np.array([np.allclose(np.sort(_vertex_neighbour_vectors(m, v), 0), np.sort(-dA, 0), atol=1e-6)
                      for v in range(m.nVertices)])
    psi = np.cos(m.xVertex[:, :2] @ k - np.where(sub_b, np.angle(S_k), 0.0))
    v1, v2 = m.verticesOnEdge[:, 0], m.verticesOnEdge[:, 1]
    u = ((psi[v2] - psi[v1]) / m.dvEdge)[:, None] * AMPS[None, :] * DC
    return m, u, 4.0 / DC ** 2 * (abs(S_k) - 3.0)


@pytest.mark.parametrize("wave", ["gradient", "rotational"])
@pytest.mark.parametrize("a,b", [(1, 0), (2, 3)])
@pytest.mark.parametrize("hdiff", [0, 1])
def test_viscosity_of_plane_waves(wave, a, b, hdiff):
    m, u, ev = (_gradient_wave if wave == "gradient" else _rotational_wave)(a, b)
    nu = 1.0e5 if hdiff == 0 else 1.0e13
    case = uniform_case(L=3, mesh=m, nu_h=nu, hdiff=hdiff)
    odd = _odd_part(u, case)
    ref = nu * ev * u if hdiff == 0 else -nu * ev ** 2 * u
    assert np.abs(ref).max() > 0
    assert np.abs(odd - ref).max() <= 1e-10 * np.abs(ref).max()


@pytest.mark.parametrize("hdiff", [0, 1])
def test_viscosity_removes_energy_on_a_sphere_with_land(hdiff):
    case = cases.with_params(cases.sphere_case(3, 3, 4461, substeps=4, dt_btr=200.0),
                             nu_h=1.0e4 if hdiff == 0 else 1.0e14, hdiff=hdiff)
    st = Setup.from_case(case)
    rng = np.random.default_rng(21)
    u = np.where(st.edge_mask[:, None], rng.normal(0.0, 0.1, case.u.shape), 0.0)
    odd = _odd_part(u, case)
    ld = (case.mesh.dvEdge * case.mesh.dcEdge)[:, None]
    energy_rate = (ld * u * odd).sum(0)
    assert np.all(energy_rate < 0.0)
    assert np.all(odd[~st.edge_mask] == 0.0)


def test_odd_part_vanishes_without_viscosity():
    m, u, _ = _gradient_wave(2, 3)
    case = uniform_case(L=3, mesh=m, nu_h=0.0)
    assert np.abs(_odd_part(u, case)).max() <= 1e-15 * np.abs(u).max()
