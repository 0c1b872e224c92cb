"""A step at a size where the edge pass's arrays pass 4 GiB, checked by a
property that holds at any size: translation invariance on the periodic hex.

A 1200 x 1200 periodic hex (1.44 M cells, 4.32 M edges) with 128 layers
holds 4.4 GB per FP64 edge array, so the edge pass takes its 64-bit column
addresses, and every other kernel runs with byte offsets past 2^32.  Its
state is the 16 x 16 C1-recipe case tiled 75 x 75 times.  All mesh tables of
the hex are the same for every tile (checked below), no step operation mixes
columns beyond the stencils, and the barotropic patches compute the same
arithmetic per edge whatever the partition, so after two steps every cell and
edge of the big mesh must hold exactly the bits of its image in the small
case, which runs with 32-bit offsets (and which the parity tests compare with
the oracle)."""
from dataclasses import replace

import numpy as np
import pytest

from synthetic import cases
from synthetic.mesh import planar_hex

pytestmark = pytest.mark.gpu

SMALL, TILES, L, STEPS = 16, 75, 128, 2


@pytest.fixture(scope="module")
def dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2105_13484_amd import ssprkse
    ssprkse.load()
    return ssprkse


def tiled_case():
    small = cases.c1(n=SMALL, L=L, steps=STEPS)
    n = SMALL * TILES
    big = planar_hex(n, n, small.mesh.dc, f0=1.0e-4)
    jj, ii = np.divmod(np.arange(n * n), n)
    mc = (ii % SMALL) + SMALL * (jj % SMALL)
    me = (3 * mc[:, None] + np.arange(3)).ravel()
    mv = (2 * mc[:, None] + np.arange(2)).ravel()
    a = small.mesh
    assert np.array_equal(big.weightsOnEdge, a.weightsOnEdge[me])
    assert np.array_equal(big.kiteAreasOnVertex, a.kiteAreasOnVertex[mv])
    assert np.array_equal(mc[big.cellsOnEdge], a.cellsOnEdge[me])
    assert np.array_equal(3 * mc[big.edgesOnCell // 3] + big.edgesOnCell % 3, a.edgesOnCell[mc])
    eoe = np.where(big.edgesOnEdge >= 0, 3 * mc[big.edgesOnEdge // 3] + big.edgesOnEdge % 3, -1)
    assert np.array_equal(eoe, a.edgesOnEdge[me])
    assert np.array_equal(2 * mc[big.verticesOnEdge // 2] + big.verticesOnEdge % 2, a.verticesOnEdge[me])
    case = replace(small, name="c1_tiled", mesh=big, H=small.H[mc], h_ref=small.h_ref[mc], rho=small.rho[mc],
                   h=small.h[mc], u=small.u[me], cell_mask=small.cell_mask[mc],
                   temp=None if small.temp is None else small.temp[mc])
    return small, case, mc, me


@pytest.mark.timeout(600)
def test_tiled_mesh_past_4_gib_gives_the_small_case_bits(dev):
    small, case, mc, me = tiled_case()
    E = case.mesh.nEdges
    assert E * L * 8 > 2 ** 32            # the edge pass takes 64-bit column addresses
    print(f"[large] {case.mesh.nCells} cells, {E} edges, {L} layers, "
          f"{dev.footprint_bytes(case.mesh, case.params) / 2**30:.1f} GiB", flush=True)
    _, st = dev.state_from_case(small)
    assert st.step(STEPS) == 0, dev.last_error()
    ref = st.read()
    del st
    dm, st = dev.state_from_case(case)
    assert st.step(STEPS) == 0, dev.last_error()
    got = st.read()
    del st, dm
    assert np.array_equal(got["h"], ref["h"][mc])
    assert np.array_equal(got["zeta"], ref["zeta"][mc])
    assert np.array_equal(got["ubar"], ref["ubar"][me])
    for lo in range(0, E, 1 << 20):            # u in slices: 4.4 GB in all
        hi = min(E, lo + (1 << 20))
        assert np.array_equal(got["u"][lo:hi], ref["u"][me[lo:hi]]), lo
    assert np.abs(ref["u"]).max() > 0.0
