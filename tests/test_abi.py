"""The C ABI library loads, exports every symbol include/ssprkse.h declares,
and rejects broken meshes on the host (no GPU needed)."""
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ssprkse.h")


def _declared():
    text = open(HEADER).read()
    return sorted(set(re.findall(r"\b(sse_[a-z_0-9]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib():
    from paper_2105_13484_amd import ssprkse
    return ssprkse.load()


def test_exports_every_declared_symbol(lib):
    from paper_2105_13484_amd import ssprkse
    names = _declared()
    assert len(names) >= 19
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(ssprkse.EXPORTED)


def test_version_and_error(lib):
    assert b"gfx950" in lib.sse_version()
    assert isinstance(lib.sse_last_error(), bytes)


def test_mesh_validation_host_only():
    from paper_2105_13484_amd import ssprkse as S
    from synthetic import cases
    c = cases.c0()
    assert S.sse_mesh_validate(c.mesh, c.H, c.cell_mask) == S.SSE_OK
    for mutate, msg in [
        (lambda m: m.weightsOnEdge.__setitem__((3, 0), m.weightsOnEdge[3, 0] * 1.5), "antisymmetric"),
        (lambda m: m.cellsOnEdge.__setitem__((7, 1), 10 ** 6), "out of range"),
        (lambda m: m.dcEdge.__setitem__(5, -1.0), "length"),
        (lambda m: m.edgesOnCell.__setitem__((2, 3), 0), "does not touch"),
    ]:
        bad = cases.c0()
        mutate(bad.mesh)
        assert S.sse_mesh_validate(bad.mesh, bad.H, bad.cell_mask) == S.SSE_EINVAL
        assert msg in S.last_error()


def test_sphere_with_land_validates():
    from paper_2105_13484_amd import ssprkse as S
    from synthetic import cases
    c = cases.sphere_case(3, 4, 5, substeps=4, dt_btr=100.0)
    assert S.sse_mesh_validate(c.mesh, c.H, c.cell_mask) == S.SSE_OK
    H = c.H.copy()
    H[np.nonzero(c.cell_mask)[0][0]] = 0.0          # an ocean cell without depth
    assert S.sse_mesh_validate(c.mesh, H, c.cell_mask) == S.SSE_EINVAL
