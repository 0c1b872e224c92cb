"""The library on the same flow described differently: relabelled entities and
reversed edge normals.

* Relabelling: cells, edges and vertices renumbered by random permutations
  (every index table, every per-entity array and the state alike).  The
  library renumbers meshes for locality and cuts its barotropic patches from
  the numbering it is given, but the arithmetic of every column and entity
  (the order of a cell's edges, of a vertex's edges, of a stencil) follows
  the mesh's own slot orders, so the results, mapped back, are bit for bit
  those of the original numbering.
* Reversed normals: 40% of the edges with c1/c2 and v1/v2 swapped, u_e and
  every reconstruction weight involving a reversed edge negated (the same
  transformation the oracle's orientation pin uses): h and zeta are the same
  and the velocities the same up to the reversed signs, to roundoff.  Not
  bit for bit: a reversed edge lists the stencil of its other cell first, so
  its ten reconstruction terms are added in another order.  Bounds (largest
  element error over the field's largest value; for ubar, over the largest
  velocity, of which it is the layer-weighted mean): 1e-12 in FP64 (3 steps of
  ~1e-16 per operation), zeta against zeta + H at 1e-13, since zeta cancels all
  but a small part of the column; in mixed precision 1e-5 for velocities
  (FP32), 1e-9 for h and T and 1e-11 for zeta against zeta + H.
"""
from dataclasses import replace

import numpy as np
import pytest

from synthetic import cases
from tests import parity_cases as P
from tests.test_oracle_orientation import _reverse_normals

pytestmark = pytest.mark.gpu

CASES = {
    "hex_c1_recipe": lambda: cases.c1(n=10, L=20, steps=3),
    "hex_vmix_del4_tracer": lambda: P.all_terms(cases.c1(n=10, L=20, steps=3)),
    "sphere_land_ssprk2": lambda: cases.with_params(cases.sphere_case(3, 8, 71, substeps=5, dt_btr=200.0), scheme=2),
    "sphere_land_mixed": lambda: cases.with_params(cases.sphere_case(3, 8, 72, substeps=5, dt_btr=200.0), precision=1),
}


def _relabel(case, seed):
    """The case with cells, edges and vertices renumbered at random; returns it
    and the new index of every old cell, edge and vertex."""
    m = case.mesh
    rng = np.random.default_rng(seed)
    old_c, old_e, old_v = (rng.permutation(n) for n in (m.nCells, m.nEdges, m.nVertices))
    new_c, new_e, new_v = (np.argsort(o) for o in (old_c, old_e, old_v))

    def vals(a, new):
        return np.where(a >= 0, new[np.maximum(a, 0)], a).astype(a.dtype)

    mesh = replace(
        m,
        cellsOnEdge=vals(m.cellsOnEdge[old_e], new_c), edgesOnCell=vals(m.edgesOnCell[old_c], new_e),
        nEdgesOnCell=m.nEdgesOnCell[old_c], verticesOnCell=vals(m.verticesOnCell[old_c], new_v),
        cellsOnCell=vals(m.cellsOnCell[old_c], new_c), verticesOnEdge=vals(m.verticesOnEdge[old_e], new_v),
        edgesOnVertex=vals(m.edgesOnVertex[old_v], new_e), cellsOnVertex=vals(m.cellsOnVertex[old_v], new_c),
        edgesOnEdge=vals(m.edgesOnEdge[old_e], new_e), nEdgesOnEdge=m.nEdgesOnEdge[old_e],
        weightsOnEdge=m.weightsOnEdge[old_e], dcEdge=m.dcEdge[old_e], dvEdge=m.dvEdge[old_e],
        areaCell=m.areaCell[old_c], areaTriangle=m.areaTriangle[old_v], kiteAreasOnCell=m.kiteAreasOnCell[old_c],
        kiteAreasOnVertex=m.kiteAreasOnVertex[old_v], fEdge=m.fEdge[old_e], fVertex=m.fVertex[old_v],
        fCell=m.fCell[old_c], xCell=m.xCell[old_c], xEdge=m.xEdge[old_e], xVertex=m.xVertex[old_v],
        normalEdge=m.normalEdge[old_e], tangentEdge=m.tangentEdge[old_e])
    out = replace(case, mesh=mesh, H=case.H[old_c], h_ref=case.h_ref[old_c], rho=case.rho[old_c], h=case.h[old_c],
                  u=case.u[old_e], cell_mask=case.cell_mask[old_c],
                  temp=None if case.temp is None else case.temp[old_c])
    return out, new_c, new_e


def _run(dev, case, steps):
    _, st = dev.state_from_case(case)
    assert st.step(steps) == 0, dev.last_error()
    out = st.read()
    if case.params.tracer:
        out["T"] = st.read_tracer()
    return out


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2105_13484_amd import ssprkse
    ssprkse.load()
    return ssprkse


@pytest.mark.parametrize("name", sorted(CASES))
def test_relabelled_mesh_gives_the_same_bits(dev, name):
    case = CASES[name]()
    other, new_c, new_e = _relabel(case, 23)
    a = _run(dev, case, 3)
    b = _run(dev, other, 3)
    back = {"u": b["u"][new_e], "ubar": b["ubar"][new_e], "h": b["h"][new_c], "zeta": b["zeta"][new_c]}
    if "T" in b:
        back["T"] = b["T"][new_c]
    for k, v in back.items():
        assert np.array_equal(a[k], v), (name, k, float(np.abs(a[k] - v).max()))


@pytest.mark.parametrize("name", sorted(CASES))
def test_reversed_normals_give_the_same_flow(dev, name):
    case = CASES[name]()
    flip = np.random.default_rng(17).random(case.mesh.nEdges) < 0.4
    sgn = np.where(flip, -1.0, 1.0)
    a = _run(dev, case, 3)
    b = _run(dev, _reverse_normals(case, flip), 3)
    b["u"] = b["u"] * sgn[:, None]
    b["ubar"] = b["ubar"] * sgn
    scale = {k: np.abs(a[k]).max() for k in a}
    scale["zeta"] = np.abs(a["zeta"] + case.H).max()
    scale["ubar"] = scale["u"]          # the barotropic part of a velocity of that size
    err = {k: float(np.abs(a[k] - b[k]).max() / scale[k]) for k in a}
    print(f"[orientation] {name}: " + ", ".join(f"{k} {v:.2e}" for k, v in err.items()), flush=True)
    fp64 = case.params.precision == 0
    bound = {"u": 1e-12 if fp64 else 1e-5, "ubar": 1e-12 if fp64 else 1e-5, "h": 1e-12 if fp64 else 1e-9,
             "T": 1e-12 if fp64 else 1e-9, "zeta": 1e-13 if fp64 else 1e-11}
    for k, v in err.items():
        assert v <= bound[k], (name, k, v, bound[k])
