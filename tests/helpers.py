"""Small builders of special-case inputs for the pin tests (inputs only)."""
from __future__ import annotations

import numpy as np

from synthetic.cases import Case, Params
from synthetic.mesh import Mesh, planar_hex


def uniform_case(L: int = 4, U=None, h_layers=None, rho_layers=None, f0: float = 1.0e-4,
                 scheme: int = 3, M: int = 4, dt: float = 600.0, nu_h: float = 10.0,
                 nu_v: float = 0.0, c_drag: float = 0.0, reconcile: int = 1, n: int = 8,
                 mesh: Mesh | None = None, vmix: int = 0, hdiff: int = 0) -> Case:
    """Horizontally uniform layers on a regular hex: u_{e,k} = U_k . n_e."""
    mesh = mesh if mesh is not None else planar_hex(n, n, 1.0e4, f0=f0)
    C, E = mesh.nCells, mesh.nEdges
    if h_layers is None:
        h_layers = np.linspace(100.0, 400.0, L)
    if rho_layers is None:
        rho_layers = 1025.0 + np.arange(L)
    if U is None:
        U = np.zeros((L, 2))
    H = np.full(C, float(np.sum(h_layers)))
    h = np.tile(np.asarray(h_layers, float), (C, 1))
    rho = np.tile(np.asarray(rho_layers, float), (C, 1))
    u = mesh.normalEdge[:, :2] @ np.asarray(U, float).T
    params = Params(n_layers=L, scheme=scheme, substeps=M, dt=dt, nu_h=nu_h, nu_v=nu_v,
                    c_drag=c_drag, reconcile=reconcile, vmix=vmix, hdiff=hdiff)
    return Case("uniform", mesh, params, H, h.copy(), rho, h, u, np.ones(C, np.uint8), 1, 0)


def smooth_case(n: int = 16, L: int = 4, scheme: int = 3, M: int = 4, dt: float = 240.0,
                reconcile: int = 1, seed: int = 7, bathymetry: bool = True, amp_u: float = 0.02) -> Case:
    """Smooth (no grid-scale noise) stratified case for convergence and invariants."""
    rng = np.random.default_rng(seed)
    mesh = planar_hex(n, n, 1.0e4, f0=1.0e-4)
    C = mesh.nCells
    x, y = mesh.xCell[:, 0], mesh.xCell[:, 1]
    kx, ky = 2 * np.pi / mesh.Lx, 2 * np.pi / mesh.Ly
    B = np.cos(kx * x + 0.3) * np.sin(ky * y + 1.1) if bathymetry else np.zeros(C)
    H = 1000.0 + 50.0 * B
    h_ref = np.repeat((H / L)[:, None], L, axis=1)
    zeta0 = 0.05 * np.sin(kx * x + 2.0) * np.cos(ky * y)
    h = h_ref * (1.0 + zeta0 / H)[:, None]
    rho = 1025.0 + np.arange(L)[None, :] + 0.2 * np.sin(kx * x + ky * y)[:, None]
    psi_amp = amp_u * rng.uniform(0.5, 1.0, size=L)
    xe, ye = mesh.xEdge[:, 0], mesh.xEdge[:, 1]
    vel = np.stack([np.cos(ky * ye), np.sin(kx * xe)], 1)
    u = (vel @ np.eye(2))[:, :, None] * psi_amp[None, None, :]
    u = np.einsum("ejk,ej->ek", u, mesh.normalEdge[:, :2])
    params = Params(n_layers=L, scheme=scheme, substeps=M, dt=dt, reconcile=reconcile)
    return Case("smooth", mesh, params, H, h_ref, rho, h, u, np.ones(C, np.uint8), 1, seed)


def rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
