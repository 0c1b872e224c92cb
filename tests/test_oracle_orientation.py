"""Pin: the oracle's step does not depend on how the mesh orients its edges.

An edge's normal may point either way (TRiSK C-grid: cells_on_edge = (c1, c2)
puts it from c1 to c2, and vertices_on_edge orders the tangent k x n from v1
to v2); the normal velocity u_e is a component along that normal.  Describing
the same flow on the same mesh with some normals reversed -- c1 and c2 swapped,
v1 and v2 swapped, u_e negated, and every reconstruction weight that involves
a reversed edge negated (W = s(i,e) s(i,e') (...), with s the sign of the
normal seen from the cell) -- must give the same thicknesses, the same SSH and
the same velocities up to the reversed signs after any number of steps.  Any
term that treats the two cells or the two vertices of an edge unequally (a
one-sided average, a drag speed taken from one cell, a sign tied to the
numbering) breaks this.
"""
from dataclasses import replace

import numpy as np
import pytest

from oracle import ssprk_se as S
from synthetic import cases
from tests import parity_cases as P


def _reverse_normals(case, flip):
    m = case.mesh
    sgn = np.where(flip, -1.0, 1.0)
    coe = m.cellsOnEdge.copy()
    coe[flip] = coe[flip][:, ::-1]
    voe = m.verticesOnEdge.copy()
    voe[flip] = voe[flip][:, ::-1]
    valid = np.arange(m.edgesOnEdge.shape[1])[None, :] < m.nEdgesOnEdge[:, None]
    other = sgn[np.where(valid, m.edgesOnEdge, 0)]
    w = m.weightsOnEdge * sgn[:, None] * np.where(valid, other, 1.0)
    mesh = replace(m, cellsOnEdge=coe, verticesOnEdge=voe, weightsOnEdge=w,
                   normalEdge=m.normalEdge * sgn[:, None], tangentEdge=m.tangentEdge * sgn[:, None])
    return replace(case, mesh=mesh, u=case.u * sgn[:, None])


CASES = {
    "hex_ssprk3_drag": lambda: cases.c1(n=8, L=5, steps=3),
    "hex_ssprk2_vmix_del4": lambda: P.vmix(P.del4(cases.with_params(cases.c1(n=8, L=5, steps=3), scheme=2), 1e9)),
    "sphere_land_tracer": lambda: P.tracer(cases.sphere_case(3, 6, 31, substeps=4, dt_btr=200.0),
                                           kappa_h=20.0, kappa_v=1e-4),
    "sphere_land_isopycnal_literal": lambda: cases.with_params(cases.sphere_case(3, 6, 32, substeps=4, dt_btr=200.0),
                                                               vcoord=1, reconcile=2),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_step_does_not_depend_on_edge_orientation(name):
    case = CASES[name]()
    rng = np.random.default_rng(17)
    flip = rng.random(case.mesh.nEdges) < 0.4
    other = _reverse_normals(case, flip)
    steps = 3
    a = S.run(case, steps)
    b = S.run(other, steps)
    sgn = np.where(flip, -1.0, 1.0)
    names = ("u", "h", "zeta", "ubar", "T")
    for k, x, y in zip(names, a, b):
        if k == "u":
            y = y * sgn[:, None]
        elif k == "ubar":
            y = y * sgn
        scale = np.abs(x).max()
        assert scale > 0, k
        # the two runs add the same terms, in places in another order
        assert np.abs(x - y).max() <= 1e-12 * scale, (k, float(np.abs(x - y).max() / scale))
