"""Algorithms 3 and 4 against a generic Shu-Osher integrator, and the flux identity.

Algorithm 3 (4) must equal M steps of the textbook SSPRK2 (SSPRK3) scheme of
(SSPRK2) / (SSPRK3) applied to the barotropic right-hand side with G-bar
frozen, and the returned accumulated flux must satisfy
zeta_M = zeta_0 - dt div F^zeta (Section 3.4, both reconciliation paragraphs),
with sum_i A_i zeta_i conserved.
"""
import numpy as np
import pytest

from oracle import ssprk_se as S
from oracle import trisk
from oracle.layered import Setup
from synthetic import cases


def _shu_osher(scheme, y, tau, F):
    y1 = [a + tau * b for a, b in zip(y, F(*y))]
    if scheme == 2:
        y2 = [a + tau * b for a, b in zip(y1, F(*y1))]
        return [0.5 * a + 0.5 * b for a, b in zip(y, y2)]
    y2 = [a + tau * b for a, b in zip(y1, F(*y1))]
    y2 = [0.75 * a + 0.25 * b for a, b in zip(y, y2)]
    y3 = [a + tau * b for a, b in zip(y2, F(*y2))]
    return [a / 3.0 + 2.0 * b / 3.0 for a, b in zip(y, y3)]


@pytest.mark.parametrize("scheme", [2, 3])
@pytest.mark.parametrize("kind", ["hex", "sphere"])
def test_substep_is_shu_osher(scheme, kind):
    if kind == "hex":
        case = cases.c0()
    else:
        case = cases.sphere_case(3, 4, 99, substeps=6, dt_btr=120.0)
    st = Setup.from_case(case)
    rng = np.random.default_rng(21)
    zeta = np.where(st.cell_mask, rng.normal(0.0, 0.05, case.mesh.nCells), 0.0)
    ubar = np.where(st.edge_mask, rng.normal(0.0, 0.05, case.mesh.nEdges), 0.0)
    G = np.where(st.edge_mask, rng.normal(0.0, 1e-5, case.mesh.nEdges), 0.0)
    dt, M = case.params.dt, case.params.substeps
    sub = S.barotropic_ssprk2_substep if scheme == 2 else S.barotropic_ssprk3_substep
    u1, z1, F = sub(ubar, zeta, G, dt, M, st)
    y = [ubar, zeta]
    for _ in range(M):
        y = _shu_osher(scheme, y, dt / M, lambda a, b: S.barotropic_rhs(a, b, G, st))
    np.testing.assert_allclose(u1, y[0], rtol=0, atol=1e-14 * np.abs(y[0]).max())
    np.testing.assert_allclose(z1, y[1], rtol=0, atol=1e-14 * np.abs(y[1]).max())
    # flux identity and conservation of sum A zeta
    zf = zeta - dt * trisk.divergence(F, case.mesh)
    np.testing.assert_allclose(z1, zf, rtol=0, atol=1e-13 * np.abs(zeta).max())
    a = case.mesh.areaCell
    assert abs((a * z1).sum() - (a * zeta).sum()) < 1e-13 * (a * np.abs(zeta)).sum()


@pytest.mark.parametrize("scheme", [2, 3])
def test_no_flow_through_coasts(scheme):
    """Land edges carry no barotropic velocity and land cells no SSH at any
    substep: a state with SSH and flow right up to the coast, and a forcing
    there, leaves ubar and F^zeta exactly zero on every edge that touches land
    and zeta zero on land, while the wet part moves."""
    from oracle.layered import Setup
    case = cases.sphere_case(3, 4, 61, substeps=6, dt_btr=200.0)
    st = Setup.from_case(case)
    assert (~st.edge_mask.astype(bool)).sum() > 0
    rng = np.random.default_rng(9)
    wet_e, wet_c = st.edge_mask.astype(bool), st.cell_mask.astype(bool)
    ubar = np.where(wet_e, rng.normal(0, 0.1, case.mesh.nEdges), 0.0)
    zeta = np.where(wet_c, rng.normal(0, 0.3, case.mesh.nCells), 0.0)
    G = np.where(wet_e, rng.normal(0, 1e-5, case.mesh.nEdges), 0.0)
    sub = S.barotropic_ssprk2_substep if scheme == 2 else S.barotropic_ssprk3_substep
    u1, z1, F = sub(ubar, zeta, G, case.params.dt, 6, st)
    assert np.all(u1[~wet_e] == 0.0) and np.all(F[~wet_e] == 0.0)
    assert np.all(z1[~wet_c] == 0.0)
    assert np.abs(u1[wet_e] - ubar[wet_e]).max() > 0
