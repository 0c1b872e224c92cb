"""TRiSK horizontal operators (oracle; test infrastructure only).

The paper discretizes the split system in space with the TRiSK scheme on
unstructured, locally orthogonal Voronoi/Delaunay meshes and delegates the
formulas to MPAS-Ocean (Section 5, opening paragraph; Thuburn et al. 2009,
Ringler et al. 2010).  The standard forms used here:

* gradient      (grad phi)_e = (phi_c2 - phi_c1) / d_e
* divergence    (div F)_i    = (1/A_i) sum_e s_{i,e} l_e F_e
* curl          zeta_v       = (1/A_v) sum_e r_{v,e} d_e u_e
* kinetic energy K_i         = (1/A_i) sum_e (l_e d_e / 4) u_e^2
* tangential    v_e          = sum_j W_{e,j} u_{e_j}
* Laplacian     (lap u)_e    = (grad div u)_e - (zeta_v2 - zeta_v1) / l_e

s_{i,e} = +1 when the edge normal points out of cell i; r_{v,e} = +1 when
v is the second vertex of the edge (the tangent points towards it).
Arrays may carry a trailing layer axis.
"""
from __future__ import annotations

import numpy as np


def _b(a: np.ndarray, x: np.ndarray) -> np.ndarray:
    """Broadcast a per-entity coefficient against a field with optional layers."""
    return a if x.ndim == 1 else a[:, None]


def cell_to_edge(phi: np.ndarray, mesh) -> np.ndarray:
    """Arithmetic mean of the two cells of each edge."""
    c1, c2 = mesh.cellsOnEdge[:, 0], mesh.cellsOnEdge[:, 1]
    return 0.5 * (phi[c1] + phi[c2])


def gradient(phi: np.ndarray, mesh) -> np.ndarray:
    c1, c2 = mesh.cellsOnEdge[:, 0], mesh.cellsOnEdge[:, 1]
    return (phi[c2] - phi[c1]) / _b(mesh.dcEdge, phi[c1])


def divergence(F: np.ndarray, mesh) -> np.ndarray:
    C = mesh.nCells
    out = np.zeros((C,) + F.shape[1:])
    cells = np.arange(C)
    for m in range(mesh.edgesOnCell.shape[1]):
        valid = m < mesh.nEdgesOnCell
        e = np.where(valid, mesh.edgesOnCell[:, m], 0)
        s = np.where(mesh.cellsOnEdge[e, 0] == cells, 1.0, -1.0)
        coef = np.where(valid, s * mesh.dvEdge[e], 0.0)
        out = out + _b(coef, F[e]) * F[e]
    return out / _b(mesh.areaCell, out)


def curl(u: np.ndarray, mesh) -> np.ndarray:
    V = mesh.nVertices
    out = np.zeros((V,) + u.shape[1:])
    verts = np.arange(V)
    for j in range(3):
        e = mesh.edgesOnVertex[:, j]
        r = np.where(mesh.verticesOnEdge[e, 1] == verts, 1.0, -1.0)
        coef = r * mesh.dcEdge[e]
        out = out + _b(coef, u[e]) * u[e]
    return out / _b(mesh.areaTriangle, out)


def kinetic_energy(u: np.ndarray, mesh) -> np.ndarray:
    C = mesh.nCells
    out = np.zeros((C,) + u.shape[1:])
    for m in range(mesh.edgesOnCell.shape[1]):
        valid = m < mesh.nEdgesOnCell
        e = np.where(valid, mesh.edgesOnCell[:, m], 0)
        coef = np.where(valid, 0.25 * mesh.dvEdge[e] * mesh.dcEdge[e], 0.0)
        out = out + _b(coef, u[e]) * u[e] ** 2
    return out / _b(mesh.areaCell, out)


def tangential_flux(coef: np.ndarray, u: np.ndarray, mesh) -> np.ndarray:
    """sum_j W_{e,j} * (coef_e + coef_{e_j}) / 2 * u_{e_j}.

    With coef = f this is the normal component of -f k x u (Coriolis); with
    coef = the edge-averaged relative vorticity it is the normal component of
    -(k . curl u) u^perp.  The symmetric edge average keeps both terms
    energy neutral (Ringler et al. 2010).
    """
    out = np.zeros_like(u)
    for j in range(mesh.edgesOnEdge.shape[1]):
        valid = j < mesh.nEdgesOnEdge
        ej = np.where(valid, mesh.edgesOnEdge[:, j], 0)
        w = np.where(valid, mesh.weightsOnEdge[:, j], 0.0)
        cbar = 0.5 * (coef + coef[ej])
        if cbar.ndim < u.ndim:
            cbar = cbar[:, None]
        out = out + _b(w, u) * cbar * u[ej]
    return out


def vorticity_on_edges(zeta_v: np.ndarray, mesh) -> np.ndarray:
    v1, v2 = mesh.verticesOnEdge[:, 0], mesh.verticesOnEdge[:, 1]
    return 0.5 * (zeta_v[v1] + zeta_v[v2])


def laplacian(u: np.ndarray, mesh) -> np.ndarray:
    """Vector Laplacian grad(div u) - k x grad(curl u), normal component."""
    v1, v2 = mesh.verticesOnEdge[:, 0], mesh.verticesOnEdge[:, 1]
    zv = curl(u, mesh)
    return gradient(divergence(u, mesh), mesh) - (zv[v2] - zv[v1]) / _b(mesh.dvEdge, u)
