"""Mutation check of the oracle's pins (CPU only; not collected by pytest).

Plants one mistake at a time -- a flipped sign, a dropped or swapped term, a
wrong weight or index, a stage fed the wrong state -- in a copy of the oracle
(``oracle/layered.py``, ``oracle/trisk.py``, ``oracle/ssprk_se.py``) and runs
the CPU suite (``-m "not gpu"``, the ABI tests left out) against each copy.
Every mistake must make at least one test fail; the script prints one line per
mutation and exits with status 1 if one survives that is not listed as
equivalent (a change that cannot alter any result).

    python tests/oracle_mutations.py [index ...]      # all by default, ~4 min on 6 workers

Nothing in the library or the GPU tests uses this file.
"""
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

L, T, S = "oracle/layered.py", "oracle/trisk.py", "oracle/ssprk_se.py"
MUT = [
    (L, "np.divide(phi[:, :-1] - phi[:, 1:], hbar_t", "np.divide(phi[:, 1:] - phi[:, :-1], hbar_t"),
    (L, "w[:, k] = w[:, k + 1] - div[:, k] - th[:, k]", "w[:, k] = w[:, k + 1] + div[:, k] - th[:, k]"),
    (L, "        th = -frac * colsum(div)[:, None]\n    return np.where(st.cell_mask[:, None], th, 0.0)", "        th = frac * colsum(div)[:, None]\n    return np.where(st.cell_mask[:, None], th, 0.0)"),
    (L, "        th = -div\n", "        th = div\n"),
    (L, "(1.0 - p.eos_alpha", "(1.0 + p.eos_alpha"),
    (L, "vert = wT[:, :L] - wT[:, 1:]", "vert = wT[:, 1:] - wT[:, :L]"),
    (L, "tend = tend + trisk.divergence(mask_edges(he * p.kappa_h", "tend = tend - trisk.divergence(mask_edges(he * p.kappa_h"),
    (L, "tend = tend + (flux[:, :-1] - flux[:, 1:])", "tend = tend + (flux[:, 1:] - flux[:, :-1])"),
    (L, "tend = -adv - vert", "tend = adv - vert"),
    (L, "dp[:, k] = p.gravity * (acc + 0.5 * drh[:, k])", "dp[:, k] = p.gravity * (acc - 0.5 * drh[:, k])"),
    (L, "dz[:, k] = -dH + acc + 0.5 * dh[:, k]", "dz[:, k] = dH + acc + 0.5 * dh[:, k]"),
    (L, "rho_e = 0.5 * (st.rho[c1] + st.rho[c2])", "rho_e = st.rho[c1]"),
    (L, "tu = -trisk.gradient(K, m) + vort", "tu = trisk.gradient(K, m) + vort"),
    (L, "+ vort - vadv +", "- vort - vadv +"),
    (L, "+ vort - vadv +", "+ vort + vadv +"),
    (L, "- vadv + pressure_gradient_force(h, st)", "- vadv - pressure_gradient_force(h, st)"),
    (L, "    return p.nu_h * lap", "    return -p.nu_h * lap"),
    (L, "return -p.nu_h * trisk.laplacian(mask_edges(lap, st), m)", "return p.nu_h * trisk.laplacian(mask_edges(lap, st), m)"),
    (L, "tau[:, -1] = p.c_drag * speed * u[:, -1]", "tau[:, -1] = -p.c_drag * speed * u[:, -1]"),
    (L, "du = safe_ratio(tau[:, :-1] - tau[:, 1:], he", "du = safe_ratio(tau[:, 1:] - tau[:, :-1], he"),
    (L, "piv = b[:, k] - a[:, k] * cp[:, k - 1]", "piv = b[:, k] + a[:, k] * cp[:, k - 1]"),
    (L, "b = 1.0 + dt * (A[:, :L] + A[:, 1:]) / hs", "b = 1.0 + dt * (A[:, :L]) / hs"),
    (L, "vadv = 0.5 * (wdz[:, :-1] + wdz[:, 1:])", "vadv = wdz[:, :-1]"),
    (L, "A[:, L] = p.c_drag * np.where(wet, speed, 0.0)", "A[:, L] = 0.0"),
    (T, "return (phi[c2] - phi[c1]) / _b(", "return (phi[c1] - phi[c2]) / _b("),
    (T, "s = np.where(mesh.cellsOnEdge[e, 0] == cells, 1.0, -1.0)", "s = np.where(mesh.cellsOnEdge[e, 0] == cells, -1.0, 1.0)"),
    (T, "r = np.where(mesh.verticesOnEdge[e, 1] == verts, 1.0, -1.0)", "r = np.where(mesh.verticesOnEdge[e, 1] == verts, -1.0, 1.0)"),
    (T, "coef = np.where(valid, 0.25 * mesh.dvEdge[e]", "coef = np.where(valid, 0.5 * mesh.dvEdge[e]"),
    (T, "cbar = 0.5 * (coef + coef[ej])", "cbar = coef"),
    (T, "- (zv[v2] - zv[v1]) / _b(mesh.dvEdge, u)", "+ (zv[v2] - zv[v1]) / _b(mesh.dvEdge, u)"),
    (T, "return 0.5 * (zeta_v[v1] + zeta_v[v2])", "return zeta_v[v1]"),
    (S, "return ubar, mask_edges(u - ubar[:, None], st)", "return ubar, mask_edges(u + ubar[:, None], st)"),
    (S, "rhs = coriolis + T_u(u, h, st) + D_u(u, h, st) + p.gravity", "rhs = coriolis + T_u(u, h, st) + D_u(u, h, st) - p.gravity"),
    (S, "rhs = coriolis + T_u(u, h, st) + D_u(u, h, st) + p.gravity", "rhs = coriolis + T_u(u, h, st) + p.gravity"),
    (S, "rhs = coriolis + T_u(u, h, st) + D_u(u, h, st) + p.gravity", "rhs = -coriolis + T_u(u, h, st) + D_u(u, h, st) + p.gravity"),
    (S, "    ut1 = mask_edges(ut1 - dt * G[:, None], st)\n    return ut1, G", "    ut1 = mask_edges(ut1 + dt * G[:, None], st)\n    return ut1, G"),
    (S, "- p.gravity * trisk.gradient(zeta, m) + G", "+ p.gravity * trisk.gradient(zeta, m) + G"),
    (S, "- p.gravity * trisk.gradient(zeta, m) + G", "- p.gravity * trisk.gradient(zeta, m) - G"),
    (S, "du = trisk.tangential_flux(m.fEdge, ubar, m) -", "du = -trisk.tangential_flux(m.fEdge, ubar, m) -"),
    (S, "trisk.cell_to_edge(zeta + st.H, st.mesh)", "trisk.cell_to_edge(zeta, st.mesh)"),
    (S, "F = F + (barotropic_flux(ubar, zeta, st) + barotropic_flux(u1, z1, st)) / (2 * M)", "F = F + (barotropic_flux(ubar, zeta, st) + barotropic_flux(u1, z1, st)) / M"),
    (S, "uh, zh = 0.75 * ubar + 0.25 * u2, 0.75 * zeta + 0.25 * z2", "uh, zh = 0.5 * ubar + 0.5 * u2, 0.5 * zeta + 0.5 * z2"),
    (S, "+ 2.0 * barotropic_flux(uh, zh, st) / (3 * M))", "+ 2.0 * barotropic_flux(uh, zh, st) / (6 * M))"),
    (S, "return G1 / 6.0 + G2 / 6.0 + 2.0 * G3 / 3.0", "return G1 / 3.0 + G2 / 3.0 + G3 / 3.0"),
    (S, "return 0.5 * G1 + 0.5 * G2", "return G2"),
    (S, "Fh3 = (f1 + f2 + 2.0 * P) / 6.0", "Fh3 = (f1 + f2 + P) / 6.0"),
    (S, "uA3 = safe_ratio(1.5 * (Fz3 - Fh3), S3", "uA3 = safe_ratio((Fz3 - Fh3), S3"),
    (S, "uA2 = safe_ratio(2.0 * (Fz2 - Fh2), S2", "uA2 = safe_ratio((Fz2 - Fh2), S2"),
    (S, "ut_half = 0.75 * ut + 0.25 * ut2", "ut_half = 0.5 * ut + 0.5 * ut2"),
    (S, "h_new = h / 3.0 + 2.0 * h3 / 3.0", "h_new = 0.5 * h + 0.5 * h3"),
    (S, "return mask_edges(u1 - ubar[:, None], st), G", "return mask_edges(u1, st), G"),
    (S, "return h_in * T_in + dt * tracer_tendency", "return T_in + dt * tracer_tendency"),
    (S, "barotropic_ssprk2_substep(ubar, zeta, interp2(G0, G1), dt, M, st)", "barotropic_ssprk2_substep(ubar, zeta, G1, dt, M, st)"),
    (S, "barotropic_ssprk3_substep(ub1, z1, G1, dt, M, st)", "barotropic_ssprk3_substep(ubar, zeta, G1, dt, M, st)"),
    (S, "uA1 = safe_ratio(Fz1 - Fh1, S1, st.edge_mask) if rec else zero", "uA1 = safe_ratio(Fh1 - Fz1, S1, st.edge_mask) if rec else zero"),
    (S, "h_half = 0.75 * h + 0.25 * h2", "h_half = 0.75 * h1 + 0.25 * h2"),
    (S, "ut_new = 0.5 * (ut + ut2)", "ut_new = ut2"),
    (S, "h_new = 0.5 * (h + h2)", "h_new = h2"),
    (S, "ub_half = 0.75 * ubar + 0.25 * ub2", "ub_half = ub2"),
    (S, "h3 = thickness_stage(h_half, 0.5 * (u + u_new), uA3, dt, st)", "h3 = thickness_stage(h_half, u_new, uA3, dt, st)"),
    (S, "ubar, zeta = ubar / 3.0 + 2.0 * u3 / 3.0, zeta / 3.0 + 2.0 * z3 / 3.0", "ubar, zeta = u3, z3"),
    (S, "ubar, zeta = 0.5 * (ubar + u2), 0.5 * (zeta + z2)", "ubar, zeta = u2, z2"),
]

MUT += [
    (L, "    frac = safe_ratio(st.h_ref, colsum(st.h_ref)[:, None], st.cell_mask[:, None])\n    th = -frac * colsum(div)[:, None]\n    for k", "    frac = safe_ratio(h, colsum(h)[:, None], st.cell_mask[:, None])\n    th = -frac * colsum(div)[:, None]\n    for k"),
    (L, "        frac = safe_ratio(st.h_ref, colsum(st.h_ref)[:, None], st.cell_mask[:, None])\n        th = -frac", "        frac = safe_ratio(h, colsum(h)[:, None], st.cell_mask[:, None])\n        th = -frac"),
    (L, "hbar_t = 0.5 * (h[:, :-1] + h[:, 1:])\n    np.divide", "hbar_t = h[:, :-1]\n    np.divide"),
    (L, "return np.sqrt(kb[m.cellsOnEdge[:, 0]] + kb[m.cellsOnEdge[:, 1]])", "return np.sqrt(2.0 * kb[m.cellsOnEdge[:, 0]])"),
    (L, "c = -dt * A[:, 1:] / hs", "c = -dt * A[:, :L] / hs"),
    (L, "Tt[:, 1:L] = 0.5 * (T[:, :-1] + T[:, 1:])", "Tt[:, 1:L] = T[:, :-1]"),
    (L, "adv = trisk.divergence(mask_edges(he * Te * v, st), m)", "adv = trisk.divergence(mask_edges(he * v, st), m) * T"),
    (L, "(T - p.eos_tref))", "(T + p.eos_tref))"),
    (L, "flux = p.kappa_v * D_zt(T, h)", "flux = p.kappa_v * D_zt(T, np.ones_like(h))"),
    (L, "he * p.kappa_h * trisk.gradient(T, m)", "p.kappa_h * trisk.gradient(T, m)"),
    (S, "ubar = safe_ratio(colsum(he * u), colsum(he), st.edge_mask)", "ubar = safe_ratio(colsum(u), colsum(np.ones_like(he)), st.edge_mask)"),
    (S, "Fh2, S2 = _edge_sum(h1, u1, st)", "Fh2, S2 = _edge_sum(h, u1, st)"),
    (S, "P, S3 = _edge_sum(h_half, u + u_new, st)", "P, S3 = _edge_sum(h_half, u_new, st)"),
    (S, "P, S2 = _edge_sum(h1, u_new, st)", "P, S2 = _edge_sum(h, u_new, st)"),
    (S, "Fh2 = 0.5 * ((Fz1 if rec == 1 else Fh1) + P)", "Fh2 = 0.5 * (Fh1 + P)"),
    (S, "f1, f2 = (Fz1, Fz2) if rec == 1 else (Fh1, Fh2)", "f1, f2 = (Fh1, Fh2)"),
    (S, "z_half = ssh(h_half, st)", "z_half = ssh(h1, st)"),
    (S, "ut3, G_half = bfe(u_half, ut_half, ub_half, z_half, h_half, dt", "ut3, G_half = bfe(u_half, ut_half, ub_half, z_half, h1, dt"),
    (S, "ut2, G1 = bfe(u1, ut1, ub1, z1, h1, dt, with_density(st, T1))\n    ut_new", "ut2, G1 = bfe(u1, ut1, ub1, zeta, h1, dt, with_density(st, T1))\n    ut_new"),
    (S, "ut2, G1 = bfe(u1, ut1, ub1, z1, h1, dt, with_density(st, T1))\n    ut_half", "ut2, G1 = bfe(u1, ut1, ub1, z1, h1, dt, with_density(st, T))\n    ut_half"),
    (S, "T_new = tracer_of(0.5 * (h * T + tracer_stage(h1, T1, u_new, uA2, dt, st)), h_new, st)", "T_new = tracer_of(0.5 * (h * T + tracer_stage(h1, T1, u_new, uA2, dt, st)), h2, st)"),
    (S, "u3, z3 = uh + tau * du, zh + tau * dz", "u3, z3 = ubar + tau * du, zeta + tau * dz"),
    (S, "        u2, z2 = u1 + tau * du, z1 + tau * dz\n        F = F + (barotropic_flux(ubar, zeta, st) + barotropic_flux(u1, z1, st)) / (2 * M)", "        u2, z2 = ubar + tau * du, zeta + tau * dz\n        F = F + (barotropic_flux(ubar, zeta, st) + barotropic_flux(u1, z1, st)) / (2 * M)"),
    (S, "u1 = vertical_diffusion_solve(ut1 + ubar[:, None], h, bottom_speed(u, st), dt, st)", "u1 = vertical_diffusion_solve(ut1 + ubar[:, None], h, bottom_speed(ut1, st), dt, st)"),
    (S, "tracer_of(tracer_stage(h, T, u, uA1, dt, st), h1, st)", "tracer_of(tracer_stage(h, T, u, 0.0 * uA1, dt, st), h1, st)"),
    (T, "return out / _b(mesh.areaCell, out)\n\n\ndef curl", "return out\n\n\ndef curl"),
    (T, "out = out + _b(w, u) * cbar * u[ej]", "out = out + _b(w, u) * cbar * u"),
    (T, "return gradient(divergence(u, mesh), mesh) -", "return -gradient(divergence(u, mesh), mesh) -"),
    (S, "    ut1 = mask_edges(ut + dt * rhs, st)\n    he = trisk.cell_to_edge(h, m)\n    G = safe_ratio(colsum(he * ut1), colsum(he), st.edge_mask) / dt\n    ut1 = mask_edges(ut1 - dt * G[:, None], st)\n    return ut1, G", "    ut1 = ut + dt * rhs\n    he = trisk.cell_to_edge(h, m)\n    G = safe_ratio(colsum(he * ut1), colsum(he), st.edge_mask) / dt\n    ut1 = mask_edges(ut1 - dt * G[:, None], st)\n    return ut1, G"),
    (S, "return mask_edges(du, st), np.where(st.cell_mask, dzeta, 0.0)", "return du, dzeta"),
    (S, "return h_in + dt * T_h(h_in, mask_edges(u_stage + uA[:, None], st), st)", "return h_in + dt * T_h(h_in, mask_edges(u_stage, st), st)"),
]


# Mutations that cannot change any result, with the reason.
EQUIVALENT = {
    next(i for i, m in enumerate(MUT) if m[2].startswith("    ut1 = ut + dt * rhs")):
        "Algorithm 1 without the first mask: G-bar of a land edge is zeroed by its own mask and "
        "ut1 is masked again after the G-bar subtraction, so land values never reach a result",
}


def run(i):
    f, old, new = MUT[i]
    src = open(os.path.join(ROOT, f)).read()
    if src.count(old) < 1:
        return i, "NOT FOUND", ""
    d = tempfile.mkdtemp(prefix=f"oracle_mut{i}_")
    try:
        for sub in ("oracle", "tests", "synthetic", "paper_2105_13484_amd"):
            shutil.copytree(os.path.join(ROOT, sub), os.path.join(d, sub),
                            ignore=shutil.ignore_patterns("__pycache__", "csrc"))
        for fn in ("pytest.ini", "__graft_entry__.py"):
            shutil.copy(os.path.join(ROOT, fn), d)
        with open(os.path.join(d, f), "w") as fh:
            fh.write(src.replace(old, new, 1))
        r = subprocess.run([sys.executable, "-m", "pytest", "tests", "-q", "-m", "not gpu", "-p", "no:cacheprovider",
                            "-x", "--ignore=tests/test_abi.py"], cwd=d, capture_output=True, text=True, timeout=900,
                           env=dict(os.environ, OMP_NUM_THREADS="1", OPENBLAS_NUM_THREADS="1"))
    finally:
        shutil.rmtree(d, ignore_errors=True)
    failed = [ln for ln in r.stdout.splitlines() if ln.startswith(("FAILED", "ERROR"))]
    last = r.stdout.strip().splitlines()[-1] if r.stdout.strip() else ""
    return i, ("killed" if r.returncode != 0 else "SURVIVED"), (failed[0] if failed else last)


def main() -> int:
    sel = range(len(MUT)) if len(sys.argv) < 2 else [int(x) for x in sys.argv[1:]]
    bad = 0
    with ThreadPoolExecutor(6) as ex:
        for i, status, info in ex.map(run, sel):
            f, old, new = MUT[i]
            note = ""
            if status != "killed":
                if i in EQUIVALENT:
                    note = " (equivalent: " + EQUIVALENT[i] + ")"
                else:
                    bad += 1
            print(f"{i:2d} {status:9s} {os.path.basename(f):12s} {new[:60]!r} :: {info[:100]}{note}", flush=True)
    print(f"{len(sel)} mutations, {bad} surviving that are not equivalent", flush=True)
    return 1 if bad else 0


if __name__ == "__main__":
    sys.exit(main())
