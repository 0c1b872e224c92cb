"""Physical invariants of the GPU step itself, independent of the oracle's
numbers (Section 1's flux form; the lake at rest):

* a flat-bottomed lake at rest with stratified layers stays at rest exactly,
  in FP64 and in mixed precision (every pressure-gradient difference is zero
  when neighbouring columns are identical);
* over bathymetry, and on a sphere with land, a lake of uniform density stays
  at rest to 1e-10 m/s over 100 steps (FP64);
* total volume sum_i A_i sum_k h_ik is conserved to roundoff by whole steps
  on a sphere with land, in both precisions and both schemes.
"""
import numpy as np
import pytest

from synthetic import cases
from tests.helpers import uniform_case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2105_13484_amd import ssprkse
    ssprkse.load()
    return ssprkse


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("scheme", [2, 3])
def test_flat_stratified_lake_stays_exactly_at_rest(dev, scheme, precision):
    case = cases.with_params(uniform_case(L=5, scheme=scheme, M=4, dt=600.0, nu_v=1e-3, c_drag=1e-3),
                             precision=precision)
    _, st = dev.state_from_case(case)
    assert st.step(20) == 0, dev.last_error()
    out = st.read()
    assert np.all(out["u"] == 0.0) and np.all(out["ubar"] == 0.0)
    assert np.array_equal(out["h"], case.h)


def test_lake_over_bathymetry_stays_at_rest(dev):
    case = cases.c1(n=16, L=10, steps=100)
    case.rho[:] = 1025.0
    _, st = dev.state_from_case(case)
    assert st.step(100) == 0, dev.last_error()
    assert np.abs(st.read()["u"]).max() < 1e-10


def test_lake_on_a_sphere_with_land_stays_at_rest(dev):
    case = cases.sphere_case(3, 8, 4321, substeps=8, dt_btr=240.0)
    case.rho[:] = np.where(case.cell_mask[:, None] > 0, 1025.0, 0.0)
    _, st = dev.state_from_case(case)
    assert st.step(100) == 0, dev.last_error()
    assert np.abs(st.read()["u"]).max() < 1e-10


# SSPRK2-SE grows on this noisy state (its stability polynomial exceeds one on
# the imaginary axis), so it runs fewer steps.
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("scheme,steps", [(2, 6), (3, 20)])
def test_volume_conserved_on_a_sphere_with_land(dev, scheme, steps, precision):
    case = cases.with_params(cases.sphere_case(3, 9, 4322, substeps=6, dt_btr=200.0),
                             scheme=scheme, precision=precision)
    mask = case.cell_mask.astype(bool)
    A = case.mesh.areaCell[:, None]
    v0 = float(np.sum((A * case.h)[mask]))
    _, st = dev.state_from_case(case)
    assert st.step(steps) == 0, dev.last_error()
    out = st.read()
    v1 = float(np.sum((A * out["h"])[mask]))
    assert abs(v1 - v0) <= 1e-13 * v0
    assert np.all(out["u"][~_wet_edges(case)] == 0.0)    # coast edges carry no flow


def _wet_edges(case):
    c = case.mesh.cellsOnEdge
    m = case.cell_mask.astype(bool)
    return m[c[:, 0]] & m[c[:, 1]]
