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


def test_size_queries_validate_the_mesh_on_the_host():
    """The device-size and footprint queries read the cell-edge topology (the
    barotropic patch tables are sized from it): a counts-only or malformed
    description is rejected, a valid one sized, with no GPU involved."""
    import ctypes
    from paper_2105_13484_amd import ssprkse as S
    from synthetic import cases
    c = cases.c0()
    lib = S.load()
    d = S.sse_mesh_desc()
    d.n_cells, d.n_edges, d.n_vertices = c.mesh.nCells, c.mesh.nEdges, c.mesh.nVertices
    d.max_edges, d.max_edges2 = 6, 10
    n = ctypes.c_size_t()
    assert lib.sse_mesh_device_bytes(ctypes.byref(d), ctypes.byref(n)) == S.SSE_EINVAL
    p = S.make_params(c.params)
    assert lib.sse_footprint_bytes(ctypes.byref(d), ctypes.byref(p), ctypes.byref(n)) == S.SSE_EINVAL
    good, keep = S.mesh_desc(c.mesh, c.H, c.cell_mask)
    assert lib.sse_mesh_device_bytes(ctypes.byref(good), ctypes.byref(n)) == S.SSE_OK
    mesh_bytes = n.value
    fp = S.footprint_bytes(c.mesh, c.params)
    assert fp > mesh_bytes > 0
    bad = cases.c0()
    bad.mesh.cellsOnEdge[7, 1] = 10 ** 6
    bd, keep2 = S.mesh_desc(bad.mesh, bad.H, bad.cell_mask)
    assert lib.sse_mesh_device_bytes(ctypes.byref(bd), ctypes.byref(n)) == S.SSE_EINVAL


def test_params_struct_matches_the_header(tmp_path):
    """Field offsets and size of sse_params as the C compiler lays them out
    equal those of the ctypes mirror."""
    import ctypes
    import subprocess
    from paper_2105_13484_amd import ssprkse as S
    src = tmp_path / "lay.c"
    fields = [f for f, _ in S.sse_params._fields_]
    body = "".join(f'printf("%zu ", offsetof(sse_params, {f}));' for f in fields)
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "ssprkse.h"\n'
                   f'int main(void) {{ {body} printf("%zu\\n", sizeof(sse_params)); return 0; }}\n')
    exe = tmp_path / "lay"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = [int(x) for x in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    expect = [getattr(S.sse_params, f).offset for f in fields] + [ctypes.sizeof(S.sse_params)]
    assert out == expect
