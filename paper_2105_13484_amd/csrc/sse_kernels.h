// Kernel argument blocks and host-side launchers (defined in sse_kernels.hip).
#pragma once

#include "sse_internal.h"

namespace sse {

// Convex combinations used by the SSPRK stages, written exactly as the
// stage formulas: out = x, 3/4 b + 1/4 x, b/3 + 2x/3, (b + x)/2.
enum Combine { COMB_NONE = 0, COMB_34 = 1, COMB_THIRD = 2, COMB_HALF = 3 };

// Baroclinic forward Euler, cell pass: K - nu_h div u, z-star w at layer tops,
// bottom-layer K.  Velocity u = X + ubar_add (ubar_add may be null).
struct FECellArgs {
    DevMesh m;
    int L;
    const double *X;
    const double *ubar_add;
    const double *h;
    const double *frac;      // h_ref / sum h_ref (z-star), null for isopycnal
    double nu_h;
    double *B;               // [C][L]
    double *Wtop;            // [C][L]
    double *Kbot;            // [C]
};

// Baroclinic forward Euler, vertex pass: relative vorticity of u = X + ubar_add.
struct FEVertexArgs {
    DevMesh m;
    int L;
    const double *X;
    const double *ubar_add;
    double *Z;               // [V][L]
};

// Baroclinic forward Euler, edge pass (Algorithm 1 with the stage combination).
struct FEEdgeArgs {
    DevMesh m;
    int L;
    const double *X;          // stage velocity storage
    const double *ubar_add;   // u  = X + ubar_add
    const double *ubar_sub;   // ut = X - ubar_sub
    const double *h;
    const double *rho;
    const double *B;
    const double *Wtop;
    const double *Kbot;
    const double *Z;
    const double *zeta;
    const double *Un;         // ut^n = Un - ubar_n (used when comb != NONE or psum_a != 0)
    const double *ubar_n;
    int comb;                 // out = combine(comb, ut^n, ut1)
    double *out;              // [E][L]
    double *G;                // [E]
    double *sum_h;            // [E] sum_k h_e
    double *sum_hu;           // [E] sum_k h_e u_k (input u), nullable
    double *sum_hp;           // [E] sum_k h_e (psum_a ut^n_k + psum_b out_k), nullable
    double psum_a, psum_b;
    double *Gi;               // [E] gi0 Ga + gi1 Gb + gi2 G, nullable
    const double *Ga, *Gb;
    int interp;               // 2: (Ga + G)/2 form; 3: Ga/6 + Gb/6 + 2G/3
    double dt, g, rho0, nu_h, nu_v, c_drag;
};

// One forward-Euler evaluation of the barotropic system with frozen forcing,
// fused with the SSPRK stage combination and the F^zeta accumulation.
struct BTEvalArgs {
    DevMesh m;
    const double *ua, *za;    // stage input (ubar, zeta)
    const double *ub, *zb;    // base of the combination
    double *uo, *zo;          // output
    const double *G;          // frozen forcing
    double *F;                // accumulated flux (edges), nullable
    double wF;                // weight of this stage's flux
    int zeroF;                // overwrite F instead of accumulating
    int comb;
    double tau, g;
};

// Thickness stage with the z-star distribution of a 2D total flux.
struct THArgs {
    DevMesh m;
    int L;
    const double *h_in;
    const double *h_n;        // base of the combination
    const double *frac;
    const double *Ftot;       // [E] sum_k h_e (u_k + u^A)
    int comb;
    double dt;
    double *h_out;
    double *zeta_out;
    int *nonfinite;
};

// Thickness stage, isopycnal: per-layer flux h_e (X + ubar_add + uA).
struct THIsoArgs {
    DevMesh m;
    int L;
    const double *h_in, *h_n;
    const double *X1, *X2;    // stage velocity = c1 X1 + c2 X2 + a_e
    double c1, c2;
    const double *a1, *a2;    // a_e = ca1 a1 + ca2 a2 + uA (nullable parts)
    double ca1, ca2;
    const double *uA;
    int comb;
    double dt;
    double *h_out, *zeta_out;
    int *nonfinite;
};

// Reconciliation deficits (Section 3.4) on edges.
struct ReconArgs {
    DevMesh m;
    int mode;                 // 0: stage with F^h = sum_hu; 1: SSPRK3 stage 3; 2: SSPRK2 stage 2
    int rec;                  // SSE_RECONCILE_*
    const double *Fz, *Fh, *Sh, *Pp;
    const double *ub_n, *ub_new;
    const double *Fz1, *Fz2, *Fh1, *Fh2;
    double *Ftot, *uA;
    const double *ub2;        // optional: ub_half = 3/4 ub_n + 1/4 ub2
    double *ub_half;
};

// u = ubar_bt + X on every layer, then the split (BBspl) of u with h.
struct AssembleArgs {
    DevMesh m;
    int L;
    const double *X;          // ut^{n+1} (or u itself when ubar_bt is null)
    const double *ubar_bt;
    const double *h;
    double *U;                // [E][L] output (may alias X when ubar_bt is null)
    double *ubar;             // [E] split barotropic velocity
    int *nonfinite;
};

// LDS bytes the tiled edge pass needs for tile set t and L layers.
size_t fe_edge_tiled_lds(const DevTiles &t, int L);
void launch_fe_edge_tiled(const FEEdgeArgs &a, const DevTiles &t, hipStream_t s);
void set_tiled_lds_limit(size_t bytes);
void launch_fe_cell(const FECellArgs &a, hipStream_t s);
void launch_fe_vertex(const FEVertexArgs &a, hipStream_t s);
void launch_fe_edge(const FEEdgeArgs &a, hipStream_t s);
void launch_bt_eval(const BTEvalArgs &a, hipStream_t s);
void launch_thickness(const THArgs &a, hipStream_t s);
void launch_thickness_iso(const THIsoArgs &a, hipStream_t s);
void launch_recon(const ReconArgs &a, hipStream_t s);
void launch_assemble(const AssembleArgs &a, hipStream_t s);
void launch_zeta_from_h(const DevMesh &m, int L, const double *h, double *zeta, hipStream_t s);
void launch_edge_flux_sum(const DevMesh &m, int L, const double *h, const double *X, const double *uA,
                          double *F, hipStream_t s);
void launch_copy(const double *src, double *dst, size_t n, hipStream_t s);

}  // namespace sse
