"""Layered primitive equations of Section 2 (oracle; test infrastructure only).

Layers k = 0 .. L-1 run from the surface down; layer interfaces i = 0 .. L,
interface i being the top of layer i.  Velocity and thickness sit at layer
mid-depth, the vertical velocity w at interfaces (Section 2, vertical
staggering).  Notation follows the paper:

* \\bar(phi)^m_k = (phi_k + phi_{k+1}) / 2            (interfaces -> layer)
* D_{z^m}(phi)_k = (phi_k - phi_{k+1}) / h_k            (interfaces -> layer)
* D_{z^t}(phi)_k = (phi_{k-1} - phi_k) / \\bar(h)^t_k    (layers -> interface)

Readings of what the paper leaves to MPAS (each stated where it is used):

* thickness at edges is the mean of the two cells (h_e);
* hydrostatic pressure (hydrocon) with zero surface pressure; the pressure
  gradient in tilted layers is [grad p + g rho_e grad z_mid] / rho0 with
  z_mid = -H + sum_{l>k} h_l + h_k/2, evaluated from the differences of the two
  columns (algebraically the difference of the two hydrostatic sums);
* z-star: the layer-thickness tendency is the column-total thickness-flux
  divergence distributed by the reference thickness fractions, and w follows
  from the thickness equation upwards from w_{L} = 0; isopycnal: w = 0;
* vertical boundary conditions: w = 0 at the surface and the bottom, no
  surface stress, bottom stress c_drag |u| u at the lowest layer (the drag
  condition of Section 5), with |u|^2 = K_c1 + K_c2 of the bottom layer;
* horizontal viscosity nu_h lap u, or the biharmonic -nu_h lap(lap u) with the
  inner Laplacian zeroed on coast edges;
* tracers (temperature, when params.tracer is set): the content h T follows
  the layered tracer equation with centred edge values and the thickness
  stages' own fluxes and w; the density follows the linear EOS;
* implicit vertical diffusion (Algorithm 2): the same operator with the drag
  speed |u| taken from the stage input and frozen, so that the solve is
  linear; the velocity multiplying c_drag |u| is the new one.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import trisk


@dataclass
class Setup:
    """Static inputs of a run: mesh, parameters and frozen column data."""
    mesh: object
    params: object
    H: np.ndarray          # (C,) bottom depth
    h_ref: np.ndarray      # (C, L)
    rho: np.ndarray        # (C, L)
    cell_mask: np.ndarray  # (C,) bool
    edge_mask: np.ndarray  # (E,) bool

    @classmethod
    def from_case(cls, case) -> "Setup":
        cm = case.cell_mask.astype(bool)
        c = case.mesh.cellsOnEdge
        return cls(case.mesh, case.params, case.H.astype(float), case.h_ref.astype(float),
                   case.rho.astype(float), cm, cm[c[:, 0]] & cm[c[:, 1]])

    @property
    def L(self) -> int:
        return self.h_ref.shape[1]


SUM_ORDERS = ("exact", "top_down", "bottom_up")
_sum_order = "exact"


def set_sum_order(order: str) -> str:
    """Selects how ``colsum`` adds the layers; returns the previous choice.

    "exact" (the default, and the only one the parity tests compare against)
    is the correctly rounded sum.  "top_down" and "bottom_up" add the layers
    one after the other from the surface or from the bottom; they exist only
    to measure how far the rounding of column sums alone moves a run, which is
    what sets the parity bounds of long windows.
    """
    global _sum_order
    if order not in SUM_ORDERS:
        raise ValueError(f"unknown summation order {order!r}")
    prev, _sum_order = _sum_order, order
    return prev


def colsum(x: np.ndarray) -> np.ndarray:
    """sum_{k=1}^{L} x_k of every row, the sums over the layers of a column
    (the split BBspl, G-bar of Algorithm 1, the fluxes F^h of Section 3.4,
    zeta = sum h - H, the z-star column totals).

    The paper fixes no summation order.  The default is the correctly rounded
    sum of the row (``math.fsum``, Shewchuk's exact partials), which no
    addition order can improve on, so that the oracle carries no particular
    association of its own.
    """
    N = x.shape[0]
    if _sum_order == "exact":
        return np.fromiter(map(math.fsum, x), float, count=N)
    cols = range(x.shape[1]) if _sum_order == "top_down" else range(x.shape[1] - 1, -1, -1)
    acc = np.zeros(N)
    for k in cols:
        acc = acc + x[:, k]
    return acc


def safe_ratio(num: np.ndarray, den: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """num / den on active entities, 0 elsewhere (dry edges have den = 0)."""
    out = np.zeros_like(num)
    np.divide(num, den, out=out, where=mask)
    return out


def mask_edges(x: np.ndarray, st: Setup) -> np.ndarray:
    m = st.edge_mask if x.ndim == 1 else st.edge_mask[:, None]
    return np.where(m, x, 0.0)


def D_zt(phi: np.ndarray, h: np.ndarray) -> np.ndarray:
    """D_{z^t}(phi) at interior interfaces 1..L-1; 0 at the surface and the bottom."""
    N, L = phi.shape
    out = np.zeros((N, L + 1))
    hbar_t = 0.5 * (h[:, :-1] + h[:, 1:])
    np.divide(phi[:, :-1] - phi[:, 1:], hbar_t, out=out[:, 1:L], where=hbar_t > 0)
    return out


def thickness_flux_divergence(h: np.ndarray, u: np.ndarray, st: Setup) -> np.ndarray:
    """div(h_k u_k) per layer, with h at edges the mean of the two cells."""
    flux = mask_edges(trisk.cell_to_edge(h, st.mesh) * u, st)
    return trisk.divergence(flux, st.mesh)


def vertical_velocity(h: np.ndarray, u: np.ndarray, st: Setup) -> np.ndarray:
    """w at the L+1 interfaces of every column (Section 2, z-star paragraph).

    z-star keeps each layer a fixed fraction of the column, so the thickness
    tendency of layer k is h_ref_k / sum h_ref times minus the column-total
    flux divergence; (layerthickness) then fixes w_k - w_{k+1}, integrated
    upwards from w = 0 at the bottom.  Isopycnal: w = 0.
    """
    C, L = h.shape
    w = np.zeros((C, L + 1))
    if st.params.vcoord == 1:
        return w
    div = thickness_flux_divergence(h, u, st)
    frac = safe_ratio(st.h_ref, colsum(st.h_ref)[:, None], st.cell_mask[:, None])
    th = -frac * colsum(div)[:, None]
    for k in range(L - 1, -1, -1):
        w[:, k] = w[:, k + 1] - div[:, k] - th[:, k]
    return np.where(st.cell_mask[:, None], w, 0.0)


def T_h(h: np.ndarray, u: np.ndarray, st: Setup) -> np.ndarray:
    """T^h_k(h, u) = -div(h_k u_k) - D_{z^m}(w)_k h_k  (Section 2, grouping T^h).

    z-star: with w from ``vertical_velocity`` this is exactly the distributed
    column-total divergence -frac_k sum_l div_l, which is evaluated directly
    (the difference form would cancel the baroclinic divergences in
    floating point).  Isopycnal: w = 0, T^h = -div(h u).
    """
    div = thickness_flux_divergence(h, u, st)
    if st.params.vcoord == 1:
        th = -div
    else:
        frac = safe_ratio(st.h_ref, colsum(st.h_ref)[:, None], st.cell_mask[:, None])
        th = -frac * colsum(div)[:, None]
    return np.where(st.cell_mask[:, None], th, 0.0)


def eos(T: np.ndarray, st: Setup) -> np.ndarray:
    """Linear equation of state (eqstate) with temperature only:
    rho = rho0 (1 - alpha (T - T_ref))."""
    p = st.params
    return p.rho0 * (1.0 - p.eos_alpha * (T - p.eos_tref))


def tracer_tendency(h: np.ndarray, T: np.ndarray, v: np.ndarray, st: Setup) -> np.ndarray:
    """Tendency of the tracer content h_k T_k in the layered tracer equation
    (tracer) of Section 2, for the layer thicknesses h and the velocity v that
    transport the thickness in the same stage:

        -div(h_e T_e v) - [Tbar^t w]_k + [Tbar^t w]_{k+1}
        + div(h_e kappa_h grad T) + h_k D_{z^m}(kappa_v D_{z^t} T)_k

    with T_e = (T_c1 + T_c2)/2 (centred), Tbar^t the mean of the two layers at
    an interface, w the vertical velocity of the thickness equation for the
    same h and v (z-star, zero for isopycnal), and no flux through the surface
    and the bottom.  With T = 1 this is exactly the thickness tendency, so a
    uniform tracer stays uniform.
    """
    m, p = st.mesh, st.params
    C, L = h.shape
    he = trisk.cell_to_edge(h, m)
    Te = trisk.cell_to_edge(T, m)
    adv = trisk.divergence(mask_edges(he * Te * v, st), m)
    w = vertical_velocity(h, v, st)
    Tt = np.zeros((C, L + 1))
    Tt[:, 1:L] = 0.5 * (T[:, :-1] + T[:, 1:])
    wT = Tt * w
    vert = wT[:, :L] - wT[:, 1:]
    tend = -adv - vert
    if p.kappa_h:
        tend = tend + trisk.divergence(mask_edges(he * p.kappa_h * trisk.gradient(T, m), st), m)
    if p.kappa_v:
        flux = p.kappa_v * D_zt(T, h)          # zero at the surface and the bottom
        tend = tend + (flux[:, :-1] - flux[:, 1:])
    return np.where(st.cell_mask[:, None], tend, 0.0)


def pressure_gradient_force(h: np.ndarray, st: Setup) -> np.ndarray:
    """-(1/rho0) grad p_k in z-star layers, normal component at edges.

    p_k = sum_{l<k} rho_l g h_l + rho_k g h_k / 2 (hydrocon, p^s = 0) and
    z_k = -H + sum_{l>k} h_l + h_k / 2; the force is
    -[(p_c2 - p_c1) + g rho_e (z_c2 - z_c1)] / (rho0 d_e), with both column
    differences summed from the per-layer differences.
    """
    m, p = st.mesh, st.params
    c1, c2 = m.cellsOnEdge[:, 0], m.cellsOnEdge[:, 1]
    E, L = m.nEdges, h.shape[1]
    drh = st.rho[c2] * h[c2] - st.rho[c1] * h[c1]
    dh = h[c2] - h[c1]
    dp = np.zeros((E, L))
    acc = np.zeros(E)
    for k in range(L):
        dp[:, k] = p.gravity * (acc + 0.5 * drh[:, k])
        acc = acc + drh[:, k]
    dz = np.zeros((E, L))
    acc = np.zeros(E)
    dH = st.H[c2] - st.H[c1]
    for k in range(L - 1, -1, -1):
        dz[:, k] = -dH + acc + 0.5 * dh[:, k]
        acc = acc + dh[:, k]
    rho_e = 0.5 * (st.rho[c1] + st.rho[c2])
    return -(dp + p.gravity * rho_e * dz) / (p.rho0 * m.dcEdge[:, None])


def T_u(u: np.ndarray, h: np.ndarray, st: Setup, w: np.ndarray | None = None) -> np.ndarray:
    """T^u_k(u) = -grad|u|^2/2 - (k.curl u) u^perp - \\bar(w D_{z^t} u)^m - grad p/rho0 + nu_h lap u.

    w (cells, L + 1) is the interface vertical velocity; by default the one
    the thickness equation gives for (h, u) (``vertical_velocity``).  At an
    edge it is the mean of the two cells, and zero at the surface and the
    bottom.
    """
    m, p = st.mesh, st.params
    he = trisk.cell_to_edge(h, m)
    K = trisk.kinetic_energy(u, m)
    q = trisk.vorticity_on_edges(trisk.curl(u, m), m)
    vort = trisk.tangential_flux(q, u, m)
    if w is None:
        w = vertical_velocity(h, u, st)
    w_e = trisk.cell_to_edge(w, m)
    w_e[:, 0] = 0.0
    w_e[:, -1] = 0.0
    wdz = w_e * D_zt(u, he)
    vadv = 0.5 * (wdz[:, :-1] + wdz[:, 1:])
    tu = -trisk.gradient(K, m) + vort - vadv + pressure_gradient_force(h, st) + horizontal_viscosity(u, st)
    return mask_edges(tu, st)


def horizontal_viscosity(u: np.ndarray, st: Setup) -> np.ndarray:
    """nu_h lap u (hdiff = 0), or the hyperviscosity -nu_h lap(lap u) that the
    remark of Section 2 puts in its place for global runs (hdiff = 1).  The
    inner Laplacian is a velocity-like edge field and, like u, is zero on
    coast edges before the outer one is taken."""
    m, p = st.mesh, st.params
    lap = trisk.laplacian(u, m)
    if getattr(p, "hdiff", 0) == 1:
        return -p.nu_h * trisk.laplacian(mask_edges(lap, st), m)
    return p.nu_h * lap


def bottom_speed(u: np.ndarray, st: Setup) -> np.ndarray:
    """|u| of the lowest layer at edges, sqrt(K_c1 + K_c2) of that layer (drag)."""
    m = st.mesh
    kb = trisk.kinetic_energy(u, m)[:, -1]
    return np.sqrt(kb[m.cellsOnEdge[:, 0]] + kb[m.cellsOnEdge[:, 1]])


def D_u(u: np.ndarray, h: np.ndarray, st: Setup, speed: np.ndarray | None = None) -> np.ndarray:
    """D^u_k(u) = D_{z^m}(nu_v D_{z^t}(u))_k with no surface stress and bottom drag.

    The drag speed is that of u itself unless ``speed`` is given (the
    linearised form whose implicit solve is ``vertical_diffusion_solve``).
    """
    m, p = st.mesh, st.params
    he = trisk.cell_to_edge(h, m)
    tau = p.nu_v * D_zt(u, he)
    if speed is None:
        speed = bottom_speed(u, st)
    tau[:, 0] = 0.0
    tau[:, -1] = p.c_drag * speed * u[:, -1]
    du = safe_ratio(tau[:, :-1] - tau[:, 1:], he, st.edge_mask[:, None])
    return mask_edges(du, st)


def thomas(a: np.ndarray, b: np.ndarray, c: np.ndarray, d: np.ndarray) -> np.ndarray:
    """Solves a_k x_{k-1} + b_k x_k + c_k x_{k+1} = d_k, k = 0 .. L-1, for every row
    of the (N, L) arrays (a_0 and c_{L-1} unused): Gaussian elimination
    without pivoting of a tridiagonal matrix, forward sweep then back
    substitution (Golub and Van Loan, the tridiagonal LU).  Stable for the
    diagonally dominant systems of implicit vertical diffusion."""
    N, L = d.shape
    cp = np.zeros((N, L))
    dp = np.zeros((N, L))
    cp[:, 0] = c[:, 0] / b[:, 0]
    dp[:, 0] = d[:, 0] / b[:, 0]
    for k in range(1, L):
        piv = b[:, k] - a[:, k] * cp[:, k - 1]
        cp[:, k] = c[:, k] / piv
        dp[:, k] = (d[:, k] - a[:, k] * dp[:, k - 1]) / piv
    x = np.zeros((N, L))
    x[:, L - 1] = dp[:, L - 1]
    for k in range(L - 2, -1, -1):
        x[:, k] = dp[:, k] - cp[:, k] * x[:, k + 1]
    return x


def vertical_diffusion_solve(r: np.ndarray, h: np.ndarray, speed: np.ndarray, dt: float,
                             st: Setup) -> np.ndarray:
    """The vertical diffusion solve of Algorithm 2: u with u - dt D^u(u) = r.

    D^u is the operator of ``D_u`` with the bottom-drag speed frozen at
    ``speed`` (the stage input's), which makes the system linear and
    tridiagonal in each edge column: with A_k = nu_v / hbar^t_k at the
    interior interfaces, A_0 = 0 (no surface stress) and A_L = c_drag |u|,

        -dt A_k / h_k u_{k-1} + (1 + dt (A_k + A_{k+1}) / h_k) u_k
            - dt A_{k+1} / h_k u_{k+1} = r_k.

    Dry edges return 0.
    """
    m, p = st.mesh, st.params
    he = trisk.cell_to_edge(h, m)
    N, L = r.shape
    wet = st.edge_mask
    hs = np.where(wet[:, None], he, 1.0)
    A = np.zeros((N, L + 1))
    hbar_t = 0.5 * (hs[:, :-1] + hs[:, 1:])
    A[:, 1:L] = p.nu_v / hbar_t
    A[:, L] = p.c_drag * np.where(wet, speed, 0.0)
    a = -dt * A[:, :L] / hs
    c = -dt * A[:, 1:] / hs
    b = 1.0 + dt * (A[:, :L] + A[:, 1:]) / hs
    a[:, 0] = 0.0
    c[:, L - 1] = 0.0
    return mask_edges(thomas(a, b, c, np.where(wet[:, None], r, 0.0)), st)
