"""SSPRK2-SE / SSPRK3-SE split-explicit steps (oracle; test infrastructure only).

Follows Section 3 of the paper:

* ``split``                       -- barotropic/baroclinic split (BBspl)
* ``baroclinic_feuler``           -- Algorithm 1 (Baroclinic_FEuler)
* ``baroclinic_feuler_mixing``    -- Algorithm 2 (Baroclinic_FEuler_Mixing), used
                                     in every stage instead of Algorithm 1 when
                                     ``params.vmix`` is set
* ``barotropic_ssprk2_substep``   -- Algorithm 3, with the accumulated flux F^zeta
                                     of the SSPRK2-SE reconciliation paragraph
* ``barotropic_ssprk3_substep``   -- Algorithm 4, with F^zeta of the SSPRK3-SE
                                     reconciliation paragraph
* ``interp2`` / ``interp3``       -- equations (force2) and (force3)
* ``ssprk2_se_step``              -- Section 3.2 steps 1-3 with the revised
                                     thickness updates of Section 3.4
* ``ssprk3_se_step``              -- Section 3.3 steps 1-3 with Section 3.4

Reconciliation modes (``params.reconcile``): 0 = off (u^A = 0); 1 = "exact":
the layer fluxes that enter F^h of the averaged final stage are the ones the
thickness actually received in the earlier stages (F^zeta_1, F^zeta_2), which
makes the layer SSH equal the barotropic SSH at every stage, the stated aim of
Section 3.4; 2 = "literal": the printed F^h_2 (SSPRK2-SE) and F^h_3
(SSPRK3-SE), which use the unadjusted stage fluxes.

Two-dimensional fields carry no layer axis; three-dimensional ones are
(entities, L).  h at edges is the mean of the two cells, the same h_e in the
split, in G-bar, in F^h and in the u^A denominators.
"""
from __future__ import annotations

import numpy as np

from . import trisk
from dataclasses import replace

from .layered import (Setup, T_h, T_u, D_u, bottom_speed, colsum, eos, mask_edges, safe_ratio,
                      tracer_tendency, vertical_diffusion_solve)


def split(u: np.ndarray, h: np.ndarray, st: Setup):
    """(BBspl): ubar = sum h_k u_k / sum h_k, ut_k = u_k - ubar."""
    he = trisk.cell_to_edge(h, st.mesh)
    ubar = safe_ratio(colsum(he * u), colsum(he), st.edge_mask)
    return ubar, mask_edges(u - ubar[:, None], st)


def baroclinic_feuler(u, ut, zeta, h, dt, st: Setup):
    """Algorithm 1: forward Euler for the baroclinic mode plus G-bar.

    ut1 = ut + dt(-f ut^perp + T^u(u) + D^u(u) + g grad zeta);
    G = (1/dt) sum h ut1 / sum h;  ut1 -= dt G.
    """
    m, p = st.mesh, st.params
    coriolis = trisk.tangential_flux(m.fEdge, ut, m)          # -f ut^perp
    rhs = coriolis + T_u(u, h, st) + D_u(u, h, st) + p.gravity * trisk.gradient(zeta, m)[:, None]
    ut1 = mask_edges(ut + dt * rhs, st)
    he = trisk.cell_to_edge(h, m)
    G = safe_ratio(colsum(he * ut1), colsum(he), st.edge_mask) / dt
    ut1 = mask_edges(ut1 - dt * G[:, None], st)
    return ut1, G


def baroclinic_feuler_mixing(u, ut, ubar, zeta, h, dt, st: Setup):
    """Algorithm 2: Algorithm 1 without D^u, then the implicit vertical
    diffusion of the whole velocity.

    ut1 = ut + dt(-f ut^perp + T^u(u) + g grad zeta);  G from ut1 as in
    Algorithm 1;  ut1 -= dt G;  u1 - dt D^u(u1) = ut1 + ubar;  ut1 = u1 - ubar.
    ubar is the barotropic velocity of the stage input (u = ubar + ut); the
    drag speed of D^u is the input's.  G is the one formed before the solve.
    """
    m, p = st.mesh, st.params
    coriolis = trisk.tangential_flux(m.fEdge, ut, m)
    rhs = coriolis + T_u(u, h, st) + p.gravity * trisk.gradient(zeta, m)[:, None]
    ut1 = mask_edges(ut + dt * rhs, st)
    he = trisk.cell_to_edge(h, m)
    G = safe_ratio(colsum(he * ut1), colsum(he), st.edge_mask) / dt
    ut1 = mask_edges(ut1 - dt * G[:, None], st)
    u1 = vertical_diffusion_solve(ut1 + ubar[:, None], h, bottom_speed(u, st), dt, st)
    return mask_edges(u1 - ubar[:, None], st), G


def bfe(u, ut, ubar, zeta, h, dt, st: Setup):
    """The stage's baroclinic forward Euler: Algorithm 2 when params.vmix is
    set (implicit vertical mixing), else Algorithm 1 (explicit D^u)."""
    if getattr(st.params, "vmix", 0):
        return baroclinic_feuler_mixing(u, ut, ubar, zeta, h, dt, st)
    return baroclinic_feuler(u, ut, zeta, h, dt, st)


def barotropic_rhs(ubar, zeta, G, st: Setup):
    """Right-hand side of the barotropic system (eqtropic) with G frozen."""
    m, p = st.mesh, st.params
    du = trisk.tangential_flux(m.fEdge, ubar, m) - p.gravity * trisk.gradient(zeta, m) + G
    dzeta = -trisk.divergence(barotropic_flux(ubar, zeta, st), m)
    return mask_edges(du, st), np.where(st.cell_mask, dzeta, 0.0)


def barotropic_flux(ubar, zeta, st: Setup):
    """ubar (zeta + H) at edges, (zeta + H) the mean of the two cells."""
    return mask_edges(ubar * trisk.cell_to_edge(zeta + st.H, st.mesh), st)


def barotropic_ssprk2_substep(ubar, zeta, G, dt, M, st: Setup):
    """Algorithm 3.  Returns (ubar^1, zeta^1, F^zeta)."""
    tau = dt / M
    F = np.zeros_like(ubar)
    for _ in range(M):
        du, dz = barotropic_rhs(ubar, zeta, G, st)
        u1, z1 = ubar + tau * du, zeta + tau * dz
        du, dz = barotropic_rhs(u1, z1, G, st)
        u2, z2 = u1 + tau * du, z1 + tau * dz
        F = F + (barotropic_flux(ubar, zeta, st) + barotropic_flux(u1, z1, st)) / (2 * M)
        ubar, zeta = 0.5 * (ubar + u2), 0.5 * (zeta + z2)
    return ubar, zeta, F


def barotropic_ssprk3_substep(ubar, zeta, G, dt, M, st: Setup):
    """Algorithm 4.  Returns (ubar^1, zeta^1, F^zeta)."""
    tau = dt / M
    F = np.zeros_like(ubar)
    for _ in range(M):
        du, dz = barotropic_rhs(ubar, zeta, G, st)
        u1, z1 = ubar + tau * du, zeta + tau * dz
        du, dz = barotropic_rhs(u1, z1, G, st)
        u2, z2 = u1 + tau * du, z1 + tau * dz
        uh, zh = 0.75 * ubar + 0.25 * u2, 0.75 * zeta + 0.25 * z2
        du, dz = barotropic_rhs(uh, zh, G, st)
        u3, z3 = uh + tau * du, zh + tau * dz
        F = F + ((barotropic_flux(ubar, zeta, st) + barotropic_flux(u1, z1, st)) / (6 * M)
                 + 2.0 * barotropic_flux(uh, zh, st) / (3 * M))
        ubar, zeta = ubar / 3.0 + 2.0 * u3 / 3.0, zeta / 3.0 + 2.0 * z3 / 3.0
    return ubar, zeta, F


def interp2(G1, G2):
    """(force2)."""
    return 0.5 * G1 + 0.5 * G2


def interp3(G1, G2, G3):
    """(force3)."""
    return G1 / 6.0 + G2 / 6.0 + 2.0 * G3 / 3.0


def thickness_stage(h_in, u_stage, uA, dt, st: Setup):
    """h_in + dt T^h(h_in, u_stage + u^A) (Section 3.4 revised thickness updates)."""
    return h_in + dt * T_h(h_in, mask_edges(u_stage + uA[:, None], st), st)


def tracer_stage(h_in, T_in, u_stage, uA, dt, st: Setup):
    """(h T)_in + dt T^T(h_in, T_in, u_stage + u^A): the tracer content moved by
    the same velocity and thickness fluxes as the matching thickness stage."""
    return h_in * T_in + dt * tracer_tendency(h_in, T_in, mask_edges(u_stage + uA[:, None], st), st)


def tracer_of(hT, h, st: Setup):
    """T = (h T) / h on ocean cells."""
    return safe_ratio(hT, h, st.cell_mask[:, None])


def with_density(st: Setup, T):
    """The setup with the density of temperature T (tracer runs); st itself otherwise."""
    return st if T is None else replace(st, rho=eos(T, st))


def ssh(h, st: Setup):
    """zeta = sum_k h_k - H (Section 2, definition of zeta)."""
    return np.where(st.cell_mask, colsum(h) - st.H, 0.0)


def _edge_sum(h, u, st: Setup):
    """sum_k h_{e,k} u_k and sum_k h_{e,k}."""
    he = trisk.cell_to_edge(h, st.mesh)
    return mask_edges(colsum(he * u), st), mask_edges(colsum(he), st)


def ssprk2_se_step(u, h, st: Setup, diag: dict | None = None, T=None):
    """One SSPRK2-SE step t_n -> t_{n+1} (Section 3.2 with Section 3.4).  With a
    temperature T (tracer runs) its content follows the thickness stages and
    every baroclinic stage sees the density of its stage temperature."""
    p = st.params
    dt, M, rec = p.dt, p.substeps, p.reconcile
    zeta = ssh(h, st)
    ubar, ut = split(u, h, st)
    # Step 1, stage 1
    ut1, G0 = bfe(u, ut, ubar, zeta, h, dt, with_density(st, T))
    ub1, zb1, Fz1 = barotropic_ssprk2_substep(ubar, zeta, G0, dt, M, st)
    u1 = mask_edges(ub1[:, None] + ut1, st)
    Fh1, S1 = _edge_sum(h, u, st)
    uA1 = safe_ratio(Fz1 - Fh1, S1, st.edge_mask) if rec else np.zeros_like(ubar)
    h1 = thickness_stage(h, u, uA1, dt, st)
    z1 = ssh(h1, st)
    T1 = None if T is None else tracer_of(tracer_stage(h, T, u, uA1, dt, st), h1, st)
    # Step 1, stage 2
    ut2, G1 = bfe(u1, ut1, ub1, z1, h1, dt, with_density(st, T1))
    ut_new = 0.5 * (ut + ut2)
    # Step 2
    ub_new, zb2, Fz2 = barotropic_ssprk2_substep(ubar, zeta, interp2(G0, G1), dt, M, st)
    u_new = mask_edges(ub_new[:, None] + ut_new, st)
    # Step 3, stage 2 of the thickness
    P, S2 = _edge_sum(h1, u_new, st)
    if rec == 0:
        uA2 = np.zeros_like(ubar)
    else:
        Fh2 = 0.5 * ((Fz1 if rec == 1 else Fh1) + P)
        uA2 = safe_ratio(2.0 * (Fz2 - Fh2), S2, st.edge_mask)
    h2 = thickness_stage(h1, u_new, uA2, dt, st)
    h_new = 0.5 * (h + h2)
    if T is not None:
        T_new = tracer_of(0.5 * (h * T + tracer_stage(h1, T1, u_new, uA2, dt, st)), h_new, st)
    if diag is not None:
        diag.update(ubar=ubar, ut=ut, zeta=zeta, ut1=ut1, G0=G0, ub1=ub1, zeta_bt1=zb1, Fz1=Fz1,
                    Fh1=Fh1, uA1=uA1, h1=h1, zeta1=z1, ut2=ut2, G1=G1, ub_new=ub_new, zeta_bt2=zb2,
                    Fz2=Fz2, P=P, uA2=uA2, h2=h2, zeta_new=ssh(h_new, st), T1=T1)
    if T is not None:
        return u_new, h_new, T_new
    return u_new, h_new


def ssprk3_se_step(u, h, st: Setup, diag: dict | None = None, T=None):
    """One SSPRK3-SE step t_n -> t_{n+1} (Section 3.3 with Section 3.4); T as in
    ssprk2_se_step."""
    p = st.params
    dt, M, rec = p.dt, p.substeps, p.reconcile
    zeta = ssh(h, st)
    ubar, ut = split(u, h, st)
    zero = np.zeros_like(ubar)
    # Step 1, stage 1
    ut1, G0 = bfe(u, ut, ubar, zeta, h, dt, with_density(st, T))
    ub1, zb1, Fz1 = barotropic_ssprk3_substep(ubar, zeta, G0, dt, M, st)
    u1 = mask_edges(ub1[:, None] + ut1, st)
    Fh1, S1 = _edge_sum(h, u, st)
    uA1 = safe_ratio(Fz1 - Fh1, S1, st.edge_mask) if rec else zero
    h1 = thickness_stage(h, u, uA1, dt, st)
    z1 = ssh(h1, st)
    T1 = None if T is None else tracer_of(tracer_stage(h, T, u, uA1, dt, st), h1, st)
    # Step 1, stage 2
    ut2, G1 = bfe(u1, ut1, ub1, z1, h1, dt, with_density(st, T1))
    ut_half = 0.75 * ut + 0.25 * ut2
    ub2, zb2, Fz2 = barotropic_ssprk3_substep(ub1, z1, G1, dt, M, st)
    ub_half = 0.75 * ubar + 0.25 * ub2
    u_half = mask_edges(ub_half[:, None] + ut_half, st)
    Fh2, S2 = _edge_sum(h1, u1, st)
    uA2 = safe_ratio(Fz2 - Fh2, S2, st.edge_mask) if rec else zero
    h2 = thickness_stage(h1, u1, uA2, dt, st)
    h_half = 0.75 * h + 0.25 * h2
    z_half = ssh(h_half, st)
    T_half = None
    if T is not None:
        T_half = tracer_of(0.75 * (h * T) + 0.25 * tracer_stage(h1, T1, u1, uA2, dt, st), h_half, st)
    # Step 1, stage 3
    ut3, G_half = bfe(u_half, ut_half, ub_half, z_half, h_half, dt, with_density(st, T_half))
    ut_new = ut / 3.0 + 2.0 * ut3 / 3.0
    # Step 2
    ub_new, zb3, Fz3 = barotropic_ssprk3_substep(ubar, zeta, interp3(G0, G1, G_half), dt, M, st)
    u_new = mask_edges(ub_new[:, None] + ut_new, st)
    # Step 3, stage 3 of the thickness
    P, S3 = _edge_sum(h_half, u + u_new, st)
    if rec == 0:
        uA3 = zero
    else:
        f1, f2 = (Fz1, Fz2) if rec == 1 else (Fh1, Fh2)
        Fh3 = (f1 + f2 + 2.0 * P) / 6.0
        uA3 = safe_ratio(1.5 * (Fz3 - Fh3), S3, st.edge_mask)
    h3 = thickness_stage(h_half, 0.5 * (u + u_new), uA3, dt, st)
    h_new = h / 3.0 + 2.0 * h3 / 3.0
    if T is not None:
        hT3 = tracer_stage(h_half, T_half, 0.5 * (u + u_new), uA3, dt, st)
        T_new = tracer_of((h * T) / 3.0 + 2.0 * hT3 / 3.0, h_new, st)
    if diag is not None:
        diag.update(ubar=ubar, ut=ut, zeta=zeta, ut1=ut1, G0=G0, ub1=ub1, zeta_bt1=zb1, Fz1=Fz1,
                    Fh1=Fh1, uA1=uA1, h1=h1, zeta1=z1, ut2=ut2, G1=G1, ub2=ub2, zeta_bt2=zb2,
                    Fz2=Fz2, Fh2=Fh2, uA2=uA2, h2=h2, h_half=h_half, zeta_half=z_half, ut3=ut3,
                    G_half=G_half, ub_new=ub_new, zeta_bt3=zb3, Fz3=Fz3, P=P, uA3=uA3, h3=h3,
                    zeta_new=ssh(h_new, st), T1=T1, T_half=T_half)
    if T is not None:
        return u_new, h_new, T_new
    return u_new, h_new


def step(u, h, st: Setup, diag: dict | None = None, T=None):
    """One step; returns (u, h), or (u, h, T) when a temperature is carried."""
    if st.params.scheme == 2:
        return ssprk2_se_step(u, h, st, diag, T)
    return ssprk3_se_step(u, h, st, diag, T)


def run(case, steps: int | None = None):
    """Advance a synthetic case; returns (u, h, zeta, ubar) at the end, and the
    temperature as a fifth value when the case carries a tracer."""
    st = Setup.from_case(case)
    u, h = case.u.astype(float).copy(), case.h.astype(float).copy()
    u = mask_edges(u, st)
    T = None
    if getattr(case.params, "tracer", 0):
        T = np.where(st.cell_mask[:, None], case.temp.astype(float), 0.0)
    for _ in range(case.steps if steps is None else steps):
        if T is None:
            u, h = step(u, h, st)
        else:
            u, h, T = step(u, h, st, T=T)
    ubar, _ = split(u, h, st)
    if T is not None:
        return u, h, ssh(h, st), ubar, T
    return u, h, ssh(h, st), ubar
