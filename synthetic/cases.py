"""Seeded synthetic layered-ocean workloads.

These stand in for the paper's MPAS test cases (the baroclinic-eddies channel
and the QU240 / EC60to30 global meshes of Section 5), which are not available.
Every array is drawn from ``numpy.random.default_rng(seed)`` with
``seed = 2105_13484 + 100 * config + member``.  The module builds inputs only:
meshes, bottom depth, reference and initial layer thicknesses, density,
initial velocity, the land mask and the run parameters.  No time stepping.

Recipes
-------
* ``c0``: 16x16 periodic hex, dc = 10 km, 4 layers, rho = 1025..1028, flat
  1000 m, f = 1e-4, Gaussian SSH bump (0.1 m, e-folding radius 50 km) plus
  N(0, 1e-3) edge-velocity noise; SSPRK2-SE, dt = 300 s, M = 10, 100 steps.
* ``c1``: 512x512 periodic hex, dc = 5 km, 60 layers, bathymetry
  1000 m + 100 m * (8 seeded periodic Fourier modes, |k| <= 4, max 1),
  temperature 15 - 10 z/1000 m + 2 K front (wavelength Lx/13) -> linear EOS;
  at rest; SSPRK3-SE, dt = 300 s, M = 20 (dt_btr = 15 s), 200 steps.
* ``c2``: icosahedral level 7 on the Earth, 60 z-star layers, 30 % land from a
  seeded field of 20 Gaussian bumps, depth 500..5000 m, f = 2 Omega sin(lat),
  T = 25 - 23 z/5000 m + smoothed N(0, 0.5 K); SSPRK3-SE, dt = 1800 s, M = 30.
* ``c3_member``: ensemble member on a 64..256 square hex, 20/40/60 layers,
  M in [10, 30], dt_btr = 30 s, C1 front recipe with a seeded wavenumber.
* ``c4_request``: served request, icosahedral level 5..8, 16..100 layers,
  50..500 steps, FP64 or mixed, C2 recipe, dt_btr = 60 s * 2^(7 - level).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace

import numpy as np

from .mesh import Mesh, icosahedral, periodic_delta, planar_hex

SEED_BASE = 2105_13484

GRAVITY = 9.80616
RHO0 = 1025.0


@dataclass
class Params:
    """Run parameters; mirrors the library's ``sse_params``."""
    n_layers: int
    scheme: int = 3            # 2 = SSPRK2-SE, 3 = SSPRK3-SE
    substeps: int = 10         # M
    precision: int = 0         # 0 = FP64, 1 = mixed
    vcoord: int = 0            # 0 = z-star, 1 = isopycnal (w = 0)
    reconcile: int = 1         # 0 = off, 1 = exact (default), 2 = literal
    dt: float = 300.0
    gravity: float = GRAVITY
    rho0: float = RHO0
    nu_h: float = 10.0
    nu_v: float = 1.0e-4
    c_drag: float = 1.0e-3
    vmix: int = 0              # 1 = implicit vertical mixing (Algorithm 2)
    hdiff: int = 0             # 0 = nu_h lap u (m^2/s), 1 = -nu_h lap(lap u) (m^4/s)
    tracer: int = 0            # 1 = temperature evolves and rho follows the linear EOS
    kappa_h: float = 0.0       # tracer horizontal diffusivity (m^2/s)
    kappa_v: float = 0.0       # tracer vertical diffusivity (m^2/s)
    eos_alpha: float = 2.0e-4  # rho = rho0 (1 - eos_alpha (T - eos_tref))
    eos_tref: float = 10.0


@dataclass
class Case:
    name: str
    mesh: Mesh
    params: Params
    H: np.ndarray              # (C,)  bottom depth (0 on land)
    h_ref: np.ndarray          # (C, L) z-star reference thickness
    rho: np.ndarray            # (C, L) frozen density
    h: np.ndarray              # (C, L) initial layer thickness
    u: np.ndarray              # (E, L) initial normal velocity
    cell_mask: np.ndarray      # (C,)  uint8, 1 = ocean
    steps: int = 1
    seed: int = 0
    meta: dict = field(default_factory=dict)
    temp: np.ndarray | None = None  # (C, L) temperature the density was derived from

    @property
    def edge_mask(self) -> np.ndarray:
        c = self.mesh.cellsOnEdge
        return (self.cell_mask[c[:, 0]] & self.cell_mask[c[:, 1]]).astype(np.uint8)

    @property
    def active_cell_layers(self) -> int:
        return int(self.cell_mask.sum()) * self.params.n_layers


def linear_eos(T: np.ndarray) -> np.ndarray:
    return RHO0 * (1.0 - 2.0e-4 * (T - 10.0))


def _mid_depth(H: np.ndarray, L: int) -> np.ndarray:
    return H[:, None] * (np.arange(L) + 0.5)[None, :] / L


# ----------------------------------------------------------------------------

def c0(member: int = 0, nx: int = 16, ny: int = 16, steps: int = 100) -> Case:
    seed = SEED_BASE + member
    rng = np.random.default_rng(seed)
    mesh = planar_hex(nx, ny, 1.0e4, f0=1.0e-4)
    L = 4
    C, E = mesh.nCells, mesh.nEdges
    H = np.full(C, 1000.0)
    h_ref = np.full((C, L), 250.0)
    rho = np.tile(1025.0 + np.arange(L, dtype=float), (C, 1))
    centre = np.array([rng.uniform(0, mesh.Lx), rng.uniform(0, mesh.Ly), 0.0])
    r = np.linalg.norm(periodic_delta(mesh, np.broadcast_to(centre, mesh.xCell.shape), mesh.xCell), axis=1)
    zeta0 = 0.1 * np.exp(-(r / 5.0e4) ** 2)
    h = h_ref * (1.0 + zeta0 / H)[:, None]
    u = rng.normal(0.0, 1.0e-3, size=(E, L))
    params = Params(n_layers=L, scheme=2, substeps=10, dt=300.0)
    return Case("c0", mesh, params, H, h_ref, rho, h, u, np.ones(C, np.uint8), steps, seed)


def _front_temperature(x, depth, H, lam, phase, t_surf=15.0, grad=10.0, zscale=1000.0, amp=2.0):
    return t_surf - grad * depth / zscale + amp * np.sin(2 * np.pi * x / lam + phase)[:, None] * (1.0 - depth / H[:, None])


def c1(n: int = 512, L: int = 60, member: int = 0, steps: int = 200, dc: float = 5.0e3,
       substeps: int = 20, dt_btr: float = 15.0) -> Case:
    seed = SEED_BASE + 100 + member
    rng = np.random.default_rng(seed)
    mesh = planar_hex(n, n, dc, f0=1.0e-4)
    C, E = mesh.nCells, mesh.nEdges
    x, y = mesh.xCell[:, 0], mesh.xCell[:, 1]
    B = np.zeros(C)
    for _ in range(8):
        while True:
            kx, ky = rng.integers(-4, 5, size=2)
            if (kx, ky) != (0, 0) and kx * kx + ky * ky <= 16:
                break
        B += rng.uniform(0.5, 1.0) * np.cos(2 * np.pi * (kx * x / mesh.Lx + ky * y / mesh.Ly) + rng.uniform(0, 2 * np.pi))
    B /= np.abs(B).max()
    H = 1000.0 + 100.0 * B
    h_ref = np.repeat((H / L)[:, None], L, axis=1)
    depth = _mid_depth(H, L)
    lam = mesh.Lx / 13.0
    T = _front_temperature(x, depth, H, lam, rng.uniform(0, 2 * np.pi))
    rho = linear_eos(T)
    params = Params(n_layers=L, scheme=3, substeps=substeps, dt=substeps * dt_btr)
    return Case("c1", mesh, params, H, h_ref, rho, h_ref.copy(), np.zeros((E, L)),
                np.ones(C, np.uint8), steps, seed, meta={"n": n}, temp=T)


def _sphere_bumps(mesh: Mesh, rng, nb: int = 20) -> np.ndarray:
    R = mesh.radius
    xc = mesh.xCell / R
    s = np.zeros(mesh.nCells)
    for _ in range(nb):
        p = rng.normal(size=3)
        p /= np.linalg.norm(p)
        rb = rng.uniform(1.0e6, 3.0e6)
        a = rng.uniform(0.5, 1.5)
        d = R * np.arccos(np.clip(xc @ p, -1.0, 1.0))
        s += a * np.exp(-(d / rb) ** 2)
    return s


def _smooth_cells(mesh: Mesh, field_: np.ndarray, ocean: np.ndarray, passes: int) -> np.ndarray:
    out = field_.copy()
    nb = mesh.cellsOnCell
    valid = (np.arange(6)[None, :] < mesh.nEdgesOnCell[:, None]) & (nb >= 0)
    nbc = np.where(valid, nb, 0)
    w = (valid & ocean[nbc]).astype(float)
    for _ in range(passes):
        acc = out + (w[..., None] * out[nbc]).sum(1)
        out = acc / (1.0 + w.sum(1))[:, None]
    return out


def sphere_case(level: int, L: int, seed: int, substeps: int, dt_btr: float,
                name: str = "sphere", land_fraction: float = 0.3, mesh: Mesh | None = None) -> Case:
    rng = np.random.default_rng(seed)
    mesh = mesh if mesh is not None else icosahedral(level)
    C, E = mesh.nCells, mesh.nEdges
    s = _sphere_bumps(mesh, rng)
    q = np.quantile(s, 1.0 - land_fraction)
    ocean = s < q
    H = np.clip(500.0 + 4500.0 * (q - s) / (q - s.min()), 500.0, 5000.0)
    H = np.where(ocean, H, 0.0)
    h_ref = np.repeat((H / L)[:, None], L, axis=1)
    depth = _mid_depth(H, L)
    T = 25.0 - 23.0 * depth / 5000.0 + rng.normal(0.0, 0.5, size=(C, L))
    T = _smooth_cells(mesh, T, ocean, 2)
    rho = np.where(ocean[:, None], linear_eos(T), 0.0)
    T = np.where(ocean[:, None], T, 0.0)
    params = Params(n_layers=L, scheme=3, substeps=substeps, dt=substeps * dt_btr)
    return Case(name, mesh, params, H, h_ref, rho, h_ref.copy(), np.zeros((E, L)),
                ocean.astype(np.uint8), 1, seed, meta={"level": level}, temp=T)


def c2(level: int = 7, L: int = 60, member: int = 0, mixed: bool = True) -> Case:
    case = sphere_case(level, L, SEED_BASE + 200 + member, substeps=30, dt_btr=60.0, name="c2")
    case.params.precision = 1 if mixed else 0
    case.steps = 20
    return case


def c3_member(member: int) -> Case:
    seed = SEED_BASE + 300 + member
    rng = np.random.default_rng(seed)
    n = int(rng.choice([64, 128, 192, 256]))
    L = int(rng.choice([20, 40, 60]))
    M = int(rng.integers(10, 31))
    kfront = int(rng.integers(4, 13))
    mesh = planar_hex(n, n, 1.0e4, f0=1.0e-4)
    C, E = mesh.nCells, mesh.nEdges
    H = np.full(C, 1000.0)
    h_ref = np.repeat((H / L)[:, None], L, axis=1)
    T = _front_temperature(mesh.xCell[:, 0], _mid_depth(H, L), H, mesh.Lx / kfront, rng.uniform(0, 2 * np.pi))
    params = Params(n_layers=L, scheme=3, substeps=M, dt=30.0 * M, precision=1)
    return Case(f"c3[{member}]", mesh, params, H, h_ref, linear_eos(T), h_ref.copy(), np.zeros((E, L)),
                np.ones(C, np.uint8), 100, seed, meta={"n": n, "kfront": kfront}, temp=T)


def served_dt_btr(level: int) -> float:
    """Barotropic substep of a served request: 60 s at level 7, halved per finer
    level; coarser levels keep 60 s (dt = 1800 s with M = 30), since with
    dt of several hours the explicit bottom drag on thin bottom layers is
    unstable."""
    return 60.0 * 2.0 ** min(0, 7 - level)


def c4_request(i: int, max_level: int = 8, meshes: dict | None = None) -> Case:
    """Served request i.  ``meshes`` (level -> Mesh) lets many requests share
    one icosahedral mesh per level instead of generating it again."""
    seed = SEED_BASE + 400 + i
    rng = np.random.default_rng(seed)
    level = int(rng.integers(5, max_level + 1))
    L = int(rng.integers(16, 101))
    steps = int(rng.integers(50, 501))
    mixed = bool(rng.integers(0, 2))
    mesh = None
    if meshes is not None:
        if level not in meshes:
            meshes[level] = icosahedral(level)
        mesh = meshes[level]
    case = sphere_case(level, L, seed, substeps=30, dt_btr=served_dt_btr(level), name=f"c4[{i}]", mesh=mesh)
    case.params.precision = 1 if mixed else 0
    case.steps = steps
    return case


def with_params(case: Case, **kw) -> Case:
    return replace(case, params=replace(case.params, **kw))
