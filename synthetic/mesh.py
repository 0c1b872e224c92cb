"""Seeded synthetic meshes: unstructured, locally orthogonal TRiSK C-grids.

This module only produces *inputs* (mesh connectivity and geometry).  It holds
none of the time-stepping arithmetic: both the FP64 oracle and the HIP library
consume its tables, exactly as an MPAS mesh file would be consumed.

Two generators:

* ``planar_hex(nx, ny, dc)``  -- a doubly periodic regular hexagonal mesh
  (``ny`` even), cells in row-major order.
* ``icosahedral(level, radius)`` -- the Voronoi dual of a recursively bisected
  icosahedron on a sphere (C = 10*4^n + 2, E = 30*4^n, V = 20*4^n).

Conventions (shared by every consumer; all indices 0-based, -1 = absent):

* ``cellsOnEdge[e] = (c1, c2)``; the unit normal ``n_e`` points from c1 to c2;
  ``dcEdge`` is the c1-c2 distance.
* ``verticesOnEdge[e] = (v1, v2)`` ordered so that the tangent
  ``t_e = k x n_e`` points from v1 to v2; ``dvEdge`` is the v1-v2 distance.
* ``edgesOnCell[i]`` lists the cell's edges counter-clockwise (seen from
  outside); ``verticesOnCell[i][m]`` is the vertex between edge slot m and
  edge slot m+1.  ``kiteAreasOnCell[i][m]`` is the area of the kite
  (x_i, mid(edge m), x_v, mid(edge m+1)).
* ``edgesOnVertex[v]`` / ``cellsOnVertex[v]`` / ``kiteAreasOnVertex[v]``:
  the three edges/cells around a vertex and the kite of each cell.
* ``edgesOnEdge[e]``: the other edges of c1 (walking counter-clockwise from e)
  followed by those of c2; ``weightsOnEdge`` are the TRiSK tangential
  reconstruction weights for them (Thuburn et al. 2009 / Ringler et al. 2010,
  the spatial scheme the paper delegates to in its Section 5 opening):
  ``v_e = sum_j W[e, j] u[edgesOnEdge[e, j]]`` approximates ``u . t_e``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

MAX_EDGES = 6
MAX_EDGES2 = 10
OMEGA_EARTH = 7.292e-5
R_EARTH = 6.371e6


@dataclass
class Mesh:
    nCells: int
    nEdges: int
    nVertices: int
    cellsOnEdge: np.ndarray        # (E, 2) int32
    edgesOnCell: np.ndarray        # (C, 6) int32
    nEdgesOnCell: np.ndarray       # (C,)   int32
    verticesOnCell: np.ndarray     # (C, 6) int32
    cellsOnCell: np.ndarray        # (C, 6) int32, neighbour across edge slot m
    verticesOnEdge: np.ndarray     # (E, 2) int32
    edgesOnVertex: np.ndarray      # (V, 3) int32
    cellsOnVertex: np.ndarray      # (V, 3) int32
    edgesOnEdge: np.ndarray        # (E, 10) int32
    nEdgesOnEdge: np.ndarray       # (E,)  int32
    weightsOnEdge: np.ndarray      # (E, 10) float64
    dcEdge: np.ndarray             # (E,)
    dvEdge: np.ndarray             # (E,)
    areaCell: np.ndarray           # (C,)
    areaTriangle: np.ndarray       # (V,)
    kiteAreasOnCell: np.ndarray    # (C, 6)
    kiteAreasOnVertex: np.ndarray  # (V, 3)
    fEdge: np.ndarray              # (E,)
    fVertex: np.ndarray            # (V,)
    fCell: np.ndarray              # (C,)
    # geometry for building initial states and analytic test fields
    xCell: np.ndarray              # (C, 3) planar (z=0) or unit-sphere * radius
    xEdge: np.ndarray              # (E, 3) edge midpoint
    xVertex: np.ndarray            # (V, 3)
    normalEdge: np.ndarray         # (E, 3) unit normal n_e
    tangentEdge: np.ndarray        # (E, 3) unit tangent t_e = k x n_e
    kind: str = "planar"
    radius: float = 0.0
    Lx: float = 0.0
    Ly: float = 0.0
    dc: float = 0.0
    extra: dict = field(default_factory=dict)

    @property
    def maxEdges(self) -> int:
        return MAX_EDGES

    @property
    def maxEdges2(self) -> int:
        return MAX_EDGES2


# ----------------------------------------------------------------------------
# Generic TRiSK tables from cell-ordered connectivity
# ----------------------------------------------------------------------------

def _edge_sign(cellsOnEdge: np.ndarray, cell: np.ndarray, edge: np.ndarray) -> np.ndarray:
    """+1 where the edge normal points out of ``cell`` (cell is c1), else -1."""
    return np.where(cellsOnEdge[edge, 0] == cell, 1.0, -1.0)


def build_edges_on_edge(cellsOnEdge, edgesOnCell, nEdgesOnCell, kiteAreasOnCell,
                        areaCell, dcEdge, dvEdge):
    """edgesOnEdge / weightsOnEdge from the TRiSK tangential reconstruction.

    For each cell i of edge e, walk the cell's edges counter-clockwise starting
    at e: e_0 = e, e_1, ..., e_{n-1}; v_m is the vertex between e_{m-1} and
    e_m, R_{i,v} the kite fraction A_{i,v}/A_i.  Then
    W[e, e_j] = s_{i,e} s_{i,e_j} (1/2 - sum_{m<=j} R_{i,v_m}) l_{e_j} / d_e.
    """
    E = cellsOnEdge.shape[0]
    eoe = np.full((E, MAX_EDGES2), -1, np.int32)
    w = np.zeros((E, MAX_EDGES2), np.float64)
    neoe = np.zeros(E, np.int32)
    # position of each edge inside each of its cells
    C = edgesOnCell.shape[0]
    for side in range(2):
        cells = cellsOnEdge[:, side]
        # slot p with edgesOnCell[cell, p] == e
        match = edgesOnCell[cells] == np.arange(E)[:, None]
        p = np.argmax(match, axis=1)
        assert match[np.arange(E), p].all(), "edge missing from its cell"
        n = nEdgesOnCell[cells]
        s_e = _edge_sign(cellsOnEdge, cells, np.arange(E))
        cum = np.zeros(E)
        for j in range(1, MAX_EDGES):
            valid = j < n
            slot_e = (p + j) % n
            slot_v = (p + j - 1) % n
            ej = edgesOnCell[cells, slot_e]
            R = kiteAreasOnCell[cells, slot_v] / areaCell[cells]
            cum = cum + np.where(valid, R, 0.0)
            s_j = _edge_sign(cellsOnEdge, cells, np.where(valid, ej, 0))
            wj = s_e * s_j * (0.5 - cum) * dvEdge[np.where(valid, ej, 0)] / dcEdge
            col = neoe
            rows = np.nonzero(valid)[0]
            eoe[rows, col[rows]] = ej[rows]
            w[rows, col[rows]] = wj[rows]
            neoe = neoe + valid.astype(np.int32)
    _ = C
    return eoe, neoe, w


def _vertex_tables_from_cells(nV, edgesOnCell, verticesOnCell, nEdgesOnCell,
                              kiteAreasOnCell):
    """cellsOnVertex / edgesOnVertex / kiteAreasOnVertex by scattering cell slots."""
    C = edgesOnCell.shape[0]
    cov = np.full((nV, 3), -1, np.int32)
    eov = np.full((nV, 3), -1, np.int32)
    kov = np.zeros((nV, 3))
    fill = np.zeros(nV, np.int64)
    for m in range(MAX_EDGES):
        valid = m < nEdgesOnCell
        cells = np.nonzero(valid)[0]
        v = verticesOnCell[cells, m]
        # edge slot m+1 of the cell leaves the vertex counter-clockwise
        nxt = edgesOnCell[cells, (m + 1) % nEdgesOnCell[cells]]
        # several cells may hold the same vertex in the same slot index m
        order = np.argsort(v, kind="stable")
        v, cells, nxt = v[order], cells[order], nxt[order]
        first = np.searchsorted(v, v, side="left")
        slot = fill[v] + (np.arange(len(v)) - first)
        assert (slot < 3).all()
        cov[v, slot] = cells
        eov[v, slot] = nxt
        kov[v, slot] = kiteAreasOnCell[cells, m]
        np.add.at(fill, v, 1)
    assert (fill == 3).all(), "every vertex must touch exactly three cells"
    _ = C
    return cov, eov, kov


# ----------------------------------------------------------------------------
# Planar doubly periodic hexagonal mesh
# ----------------------------------------------------------------------------

def planar_hex(nx: int, ny: int, dc: float, f0: float = 1.0e-4) -> Mesh:
    """Regular hexagons (pointy-top Voronoi cells), periodic in x and y.

    Cell (i, j) sits at x = (i + (j mod 2)/2) dc, y = j dc sqrt(3)/2; ``ny``
    must be even for the row offset to be periodic.  Each cell owns three
    edges (towards its E, NE, NW neighbours) and two vertices (at 30 and 90
    degrees), so E = 3C and V = 2C.
    """
    if ny % 2:
        raise ValueError("ny must be even for a periodic hex mesh")
    C = nx * ny
    E, V = 3 * C, 2 * C
    s3 = np.sqrt(3.0)
    Lx, Ly = nx * dc, ny * dc * s3 / 2.0
    jj, ii = np.divmod(np.arange(C), nx)
    odd = jj % 2

    def cid(i, j):
        return (i % nx) + nx * (j % ny)

    east = cid(ii + 1, jj)
    west = cid(ii - 1, jj)
    ne = cid(ii + odd, jj + 1)
    nw = cid(ii - 1 + odd, jj + 1)
    sw = cid(ii - 1 + odd, jj - 1)
    se = cid(ii + odd, jj - 1)

    c = np.arange(C)
    cellsOnEdge = np.empty((E, 2), np.int32)
    cellsOnEdge[0::3] = np.stack([c, east], 1)
    cellsOnEdge[1::3] = np.stack([c, ne], 1)
    cellsOnEdge[2::3] = np.stack([c, nw], 1)

    vA = 2 * c          # vertex at 30 degrees of cell c
    vB = 2 * c + 1      # vertex at 90 degrees
    edgesOnCell = np.stack([3 * c, 3 * c + 1, 3 * c + 2, 3 * west, 3 * sw + 1, 3 * se + 2], 1).astype(np.int32)
    cellsOnCell = np.stack([east, ne, nw, west, sw, se], 1).astype(np.int32)
    verticesOnCell = np.stack([vA, vB, 2 * west, 2 * sw + 1, 2 * sw, 2 * se + 1], 1).astype(np.int32)
    nEdgesOnCell = np.full(C, 6, np.int32)

    verticesOnEdge = np.empty((E, 2), np.int32)
    verticesOnEdge[0::3] = np.stack([2 * se + 1, vA], 1)
    verticesOnEdge[1::3] = np.stack([vA, vB], 1)
    verticesOnEdge[2::3] = np.stack([vB, 2 * west], 1)

    areaCell = np.full(C, s3 / 2.0 * dc * dc)
    areaTriangle = np.full(V, s3 / 4.0 * dc * dc)
    kiteAreasOnCell = np.full((C, 6), areaCell[0] / 6.0)
    dcEdge = np.full(E, dc)
    dvEdge = np.full(E, dc / s3)

    cellsOnVertex, edgesOnVertex, kiteAreasOnVertex = _vertex_tables_from_cells(
        V, edgesOnCell, verticesOnCell, nEdgesOnCell, kiteAreasOnCell)
    eoe, neoe, w = build_edges_on_edge(cellsOnEdge, edgesOnCell, nEdgesOnCell,
                                       kiteAreasOnCell, areaCell, dcEdge, dvEdge)

    xc = np.zeros((C, 3))
    xc[:, 0] = (ii + 0.5 * odd) * dc
    xc[:, 1] = jj * dc * s3 / 2.0
    ang = np.deg2rad(np.array([0.0, 60.0, 120.0]))
    nrm = np.zeros((E, 3))
    for k in range(3):
        nrm[k::3, 0] = np.cos(ang[k])
        nrm[k::3, 1] = np.sin(ang[k])
    tan = np.zeros((E, 3))
    tan[:, 0] = -nrm[:, 1]
    tan[:, 1] = nrm[:, 0]
    xe = np.repeat(xc, 3, axis=0) + 0.5 * dc * nrm
    xv = np.zeros((V, 3))
    r = dc / s3
    xv[0::2, 0] = xc[:, 0] + r * np.cos(np.pi / 6)
    xv[0::2, 1] = xc[:, 1] + r * np.sin(np.pi / 6)
    xv[1::2, 0] = xc[:, 0]
    xv[1::2, 1] = xc[:, 1] + r
    for arr in (xe, xv):
        arr[:, 0] %= Lx
        arr[:, 1] %= Ly

    return Mesh(
        nCells=C, nEdges=E, nVertices=V,
        cellsOnEdge=cellsOnEdge, edgesOnCell=edgesOnCell, nEdgesOnCell=nEdgesOnCell,
        verticesOnCell=verticesOnCell, cellsOnCell=cellsOnCell, verticesOnEdge=verticesOnEdge,
        edgesOnVertex=edgesOnVertex, cellsOnVertex=cellsOnVertex,
        edgesOnEdge=eoe, nEdgesOnEdge=neoe, weightsOnEdge=w,
        dcEdge=dcEdge, dvEdge=dvEdge, areaCell=areaCell, areaTriangle=areaTriangle,
        kiteAreasOnCell=kiteAreasOnCell, kiteAreasOnVertex=kiteAreasOnVertex,
        fEdge=np.full(E, f0), fVertex=np.full(V, f0), fCell=np.full(C, f0),
        xCell=xc, xEdge=xe, xVertex=xv, normalEdge=nrm, tangentEdge=tan,
        kind="planar", Lx=Lx, Ly=Ly, dc=dc,
    )


def periodic_delta(mesh: Mesh, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Minimum-image displacement b - a on the periodic plane (2 components)."""
    d = b[..., :2] - a[..., :2]
    d[..., 0] -= mesh.Lx * np.round(d[..., 0] / mesh.Lx)
    d[..., 1] -= mesh.Ly * np.round(d[..., 1] / mesh.Ly)
    return d


# ----------------------------------------------------------------------------
# Icosahedral geodesic Voronoi sphere
# ----------------------------------------------------------------------------

def _icosahedron():
    p = (1.0 + np.sqrt(5.0)) / 2.0
    v = np.array([
        [-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
        [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
        [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1]], float)
    f = np.array([
        [0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
        [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
        [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
        [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], np.int64)
    return v / np.linalg.norm(v, axis=1, keepdims=True), f


def _subdivide(v, f):
    e = np.sort(np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]]), axis=1)
    key = e[:, 0] * len(v) + e[:, 1]
    ukey, inv = np.unique(key, return_inverse=True)
    a, b = np.divmod(ukey, len(v))
    mid = v[a] + v[b]
    mid /= np.linalg.norm(mid, axis=1, keepdims=True)
    nf = len(f)
    m01 = len(v) + inv[:nf]
    m12 = len(v) + inv[nf:2 * nf]
    m20 = len(v) + inv[2 * nf:]
    v2 = np.concatenate([v, mid])
    f2 = np.concatenate([
        np.stack([f[:, 0], m01, m20], 1),
        np.stack([f[:, 1], m12, m01], 1),
        np.stack([f[:, 2], m20, m12], 1),
        np.stack([m01, m12, m20], 1)])
    return v2, f2


def _sph_tri_area(a, b, c):
    """Area of the geodesic triangle with unit-vector corners (unit sphere)."""
    num = np.abs(np.einsum("ij,ij->i", a, np.cross(b, c)))
    den = 1.0 + np.einsum("ij,ij->i", a, b) + np.einsum("ij,ij->i", b, c) + np.einsum("ij,ij->i", c, a)
    return 2.0 * np.arctan2(num, den)


def _arc(a, b):
    return np.arctan2(np.linalg.norm(np.cross(a, b), axis=1), np.einsum("ij,ij->i", a, b))


def icosahedral(level: int, radius: float = R_EARTH, omega: float = OMEGA_EARTH) -> Mesh:
    """Voronoi dual of a level-``level`` bisected icosahedron on a sphere."""
    v, f = _icosahedron()
    for _ in range(level):
        v, f = _subdivide(v, f)
    C, T = len(v), len(f)
    # orient every triangle counter-clockwise seen from outside
    nrm = np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]])
    flip = np.einsum("ij,ij->i", nrm, v[f].sum(1)) < 0
    f[flip] = f[flip][:, [0, 2, 1]]
    xv = np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]])
    xv /= np.linalg.norm(xv, axis=1, keepdims=True)

    # undirected edges
    de = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])      # directed, CCW in face
    dface = np.concatenate([np.arange(T)] * 3)
    und = np.sort(de, axis=1)
    key = und[:, 0] * C + und[:, 1]
    ukey, first, inv = np.unique(key, return_index=True, return_inverse=True)
    E = len(ukey)
    c1, c2 = np.divmod(ukey, C)
    cellsOnEdge = np.stack([c1, c2], 1).astype(np.int32)
    # v2 = face in which c1 -> c2 runs counter-clockwise (it lies left of n_e)
    fwd = de[:, 0] < de[:, 1]                 # directed edge runs min -> max = c1 -> c2
    verticesOnEdge = np.empty((E, 2), np.int32)
    verticesOnEdge[inv[fwd], 1] = dface[fwd]
    verticesOnEdge[inv[~fwd], 0] = dface[~fwd]

    # neighbours of each cell, sorted counter-clockwise around the local vertical
    nb_src = np.concatenate([c1, c2])
    nb_dst = np.concatenate([c2, c1])
    nb_edge = np.concatenate([np.arange(E), np.arange(E)])
    order = np.argsort(nb_src, kind="stable")
    nb_src, nb_dst, nb_edge = nb_src[order], nb_dst[order], nb_edge[order]
    counts = np.bincount(nb_src, minlength=C)
    nEdgesOnCell = counts.astype(np.int32)
    start = np.concatenate([[0], np.cumsum(counts)[:-1]])
    slot = np.arange(len(nb_src)) - start[nb_src]
    nbr = np.full((C, MAX_EDGES), -1, np.int64)
    nbe = np.full((C, MAX_EDGES), -1, np.int64)
    nbr[nb_src, slot] = nb_dst
    nbe[nb_src, slot] = nb_edge
    ref = np.where(np.abs(v[:, 0:1]) < 0.9, np.array([[1.0, 0, 0]]), np.array([[0, 1.0, 0]]))
    e1 = np.cross(ref, v)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(v, e1)
    d = v[np.where(nbr >= 0, nbr, 0)] - v[:, None, :]
    ang = np.arctan2(np.einsum("cmk,ck->cm", d, e2), np.einsum("cmk,ck->cm", d, e1))
    ang = np.where(nbr >= 0, ang, np.inf)
    srt = np.argsort(ang, axis=1)
    cellsOnCell = np.take_along_axis(nbr, srt, 1).astype(np.int32)
    edgesOnCell = np.take_along_axis(nbe, srt, 1).astype(np.int32)

    # vertex slot m = triangle {i, nb_m, nb_{m+1}}
    fs = np.sort(f, axis=1)
    fkey = (fs[:, 0] * C + fs[:, 1]) * C + fs[:, 2]
    forder = np.argsort(fkey)
    fkey_sorted = fkey[forder]
    verticesOnCell = np.full((C, MAX_EDGES), -1, np.int32)
    ci = np.arange(C)
    for m in range(MAX_EDGES):
        valid = m < nEdgesOnCell
        a = cellsOnCell[ci, m]
        b = cellsOnCell[ci, (m + 1) % nEdgesOnCell]
        tri = np.sort(np.stack([ci, a, b], 1), axis=1).astype(np.int64)
        k = (tri[:, 0] * C + tri[:, 1]) * C + tri[:, 2]
        pos = np.searchsorted(fkey_sorted, k)
        pos = np.minimum(pos, len(fkey_sorted) - 1)
        ok = fkey_sorted[pos] == k
        assert ok[valid].all(), "neighbour ring is not closed"
        verticesOnCell[valid, m] = forder[pos[valid]]

    # geometry on the unit sphere, scaled by radius at the end
    xe = v[c1] + v[c2]
    xe /= np.linalg.norm(xe, axis=1, keepdims=True)
    nrmE = v[c2] - v[c1]
    nrmE /= np.linalg.norm(nrmE, axis=1, keepdims=True)
    tanE = np.cross(xe, nrmE)
    dcEdge = _arc(v[c1], v[c2]) * radius
    dvEdge = _arc(xv[verticesOnEdge[:, 0]], xv[verticesOnEdge[:, 1]]) * radius
    areaTriangle = _sph_tri_area(v[f[:, 0]], v[f[:, 1]], v[f[:, 2]]) * radius ** 2

    kite = np.zeros((C, MAX_EDGES))
    for m in range(MAX_EDGES):
        valid = m < nEdgesOnCell
        cv = ci[valid]
        n = nEdgesOnCell[cv]
        vert = xv[verticesOnCell[cv, m]]
        ma = xe[edgesOnCell[cv, m]]
        mb = xe[edgesOnCell[cv, (m + 1) % n]]
        kite[cv, m] = (_sph_tri_area(v[cv], ma, vert) + _sph_tri_area(v[cv], vert, mb)) * radius ** 2
    areaCell = np.zeros(C)
    for m in range(MAX_EDGES):
        valid = m < nEdgesOnCell
        cv = ci[valid]
        n = nEdgesOnCell[cv]
        va = xv[verticesOnCell[cv, m]]
        vb = xv[verticesOnCell[cv, (m + 1) % n]]
        areaCell[cv] += _sph_tri_area(v[cv], va, vb) * radius ** 2

    cellsOnVertex, edgesOnVertex, kiteAreasOnVertex = _vertex_tables_from_cells(
        T, edgesOnCell, verticesOnCell, nEdgesOnCell, kite)
    eoe, neoe, w = build_edges_on_edge(cellsOnEdge, edgesOnCell, nEdgesOnCell,
                                       kite, areaCell, dcEdge, dvEdge)
    return Mesh(
        nCells=C, nEdges=E, nVertices=T,
        cellsOnEdge=cellsOnEdge, edgesOnCell=edgesOnCell, nEdgesOnCell=nEdgesOnCell,
        verticesOnCell=verticesOnCell, cellsOnCell=cellsOnCell, verticesOnEdge=verticesOnEdge,
        edgesOnVertex=edgesOnVertex, cellsOnVertex=cellsOnVertex,
        edgesOnEdge=eoe, nEdgesOnEdge=neoe, weightsOnEdge=w,
        dcEdge=dcEdge, dvEdge=dvEdge, areaCell=areaCell, areaTriangle=areaTriangle,
        kiteAreasOnCell=kite, kiteAreasOnVertex=kiteAreasOnVertex,
        fEdge=2 * omega * xe[:, 2], fVertex=2 * omega * xv[:, 2], fCell=2 * omega * v[:, 2],
        xCell=v * radius, xEdge=xe * radius, xVertex=xv * radius,
        normalEdge=nrmE, tangentEdge=tanE, kind="sphere", radius=radius,
    )
