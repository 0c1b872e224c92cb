// Kernel argument blocks and host-side launchers (defined in sse_kernels.hip).
//
// R is the storage and arithmetic type of the velocity-like 3D fields, of the
// tendency arithmetic and of the barotropic substep state: double in FP64
// mode, float in mixed mode.  Layer thicknesses, density, SSH, the pressure
// gradient (its two terms cancel to the density anomaly), the column sums that
// feed the barotropic forcing and the reconciliation, the accumulated
// barotropic transport and every 2D field handed between stages are double in
// both modes.
#pragma once

#include "sse_internal.h"

namespace sse {

// Convex combinations used by the SSPRK stages, written exactly as the
// stage formulas: out = x, 3/4 b + 1/4 x, b/3 + 2x/3, (b + x)/2.
enum Combine { COMB_NONE = 0, COMB_34 = 1, COMB_THIRD = 2, COMB_HALF = 3 };

// Baroclinic forward Euler, cell pass: K - nu_h div u, z-star w at layer tops,
// bottom-layer K.  Velocity u = X + ubar_add (ubar_add may be null).
template <typename R>
struct FECellArgs {
    DevMesh m;
    int L;
    const R *X;
    const double *ubar_add;
    const double *h;
    const double *frac;      // h_ref / sum h_ref (z-star), null for isopycnal
    double nu_h;
    R *B;                    // [C][L]
    R *D1;                   // [C][L] div u (biharmonic runs), nullable
    R *Wtop;                 // [C][L]
    double *Kbot;            // [C]
};

// Baroclinic forward Euler, vertex pass: relative vorticity of u = X + ubar_add.
template <typename R>
struct FEVertexArgs {
    DevMesh m;
    int L;
    const R *X;
    const double *ubar_add;
    R *Z;                    // [V][L]
};

// Baroclinic forward Euler, edge pass (Algorithm 1 with the stage combination).
template <typename R>
struct FEEdgeArgs {
    DevMesh m;
    int L;
    const R *X;               // stage velocity storage
    const double *ubar_add;   // u  = X + ubar_add
    const double *ubar_sub;   // ut = X - ubar_sub
    const double *h;
    const double *rho;        // FP64 in both modes (see the pressure gradient)
    const R *B;
    const R *Wtop;
    const double *Kbot;
    const R *Z;
    const double *zeta;
    const R *Un;              // ut^n = Un - ubar_n (used when comb != NONE or psum_a != 0)
    const double *ubar_n;
    int comb;                 // out = combine(comb, ut^n, ut1)
    R *out;                   // [E][L]
    double *G;                // [E]
    double *sum_h;            // [E] sum_k h_e
    double *sum_hu;           // [E] sum_k h_e u_k (input u), nullable
    double *sum_hp;           // [E] sum_k h_e (psum_a ut^n_k + psum_b out_k), nullable
    double psum_a, psum_b;
    double *Gi;               // [E] interpolated forcing, nullable
    const double *Ga, *Gb;
    int interp;               // 2: Ga/2 + G/2; 3: Ga/6 + Gb/6 + 2G/3
    int vmix;                 // 1: D^u by the implicit column solve (Algorithm 2)
    const R *D2, *Z2;         // div and curl of lap u (biharmonic runs), nullable
    double nu4;               // biharmonic coefficient (m^4/s); nu_h is 0 then
    double dt, g, rho0, nu_h, nu_v, c_drag;
};

// The FP32 pass also takes the barotropic velocity it uses rounded to FP32
// once per pass.  The FP64 pass keeps the layout above: where the pointer
// sits in the argument block moves the compiler's scalar-register spills, and
// these two layouts measured fastest for each precision (C1 edge pass: FP64
// 1.078 ms as before, FP32 0.753 ms; with one shared layout one of the two
// lost 2-3%).
template <>
struct FEEdgeArgs<float> {
    DevMesh m;
    int L;
    const float *X;           // stage velocity storage
    const double *ubar_add;   // u  = X + ubar_add
    const double *ubar_sub;   // ut = X - ubar_sub
    const float *ubar_r;      // ubar_add or ubar_sub, the one the pass uses, rounded to FP32
    const double *h;
    const double *rho;        // FP64 in both modes (see the pressure gradient)
    const float *B;
    const float *Wtop;
    const double *Kbot;
    const float *Z;
    const double *zeta;
    const float *Un;          // ut^n = Un - ubar_n (used when comb != NONE or psum_a != 0)
    const double *ubar_n;
    int comb;                 // out = combine(comb, ut^n, ut1)
    float *out;               // [E][L]
    double *G;                // [E]
    double *sum_h;            // [E] sum_k h_e
    double *sum_hu;           // [E] sum_k h_e u_k (input u), nullable
    double *sum_hp;           // [E] sum_k h_e (psum_a ut^n_k + psum_b out_k), nullable
    double psum_a, psum_b;
    double *Gi;               // [E] interpolated forcing, nullable
    const double *Ga, *Gb;
    int interp;               // 2: Ga/2 + G/2; 3: Ga/6 + Gb/6 + 2G/3
    int vmix;                 // 1: D^u by the implicit column solve (Algorithm 2)
    const float *D2, *Z2;     // div and curl of lap u (biharmonic runs), nullable
    double nu4;               // biharmonic coefficient (m^4/s); nu_h is 0 then
    double dt, g, rho0, nu_h, nu_v, c_drag;
};

// Vector Laplacian of u at edges from div u at cells and curl u at vertices:
// out = (D_c2 - D_c1) / d_e - (Z_v2 - Z_v1) / l_e, zero on coast edges.
template <typename R>
struct LapArgs {
    DevMesh m;
    int L;
    const R *D, *Z;
    R *out;                   // [E][L]
};

// Divergence of an edge field at cells: out_i = sum_j (s l / A)_ij X_ej.
template <typename R>
struct DivArgs {
    DevMesh m;
    int L;
    const R *X;
    R *out;                   // [C][L]
};

// One forward-Euler evaluation of the barotropic system with frozen forcing,
// fused with the SSPRK stage combination and the F^zeta accumulation.
template <typename R>
struct BTEvalArgs {
    DevMesh m;
    const R *ua, *za;         // stage input (ubar, zeta)
    const R *ub, *zb;         // base of the combination
    R *uo, *zo;               // output
    const double *G;          // frozen forcing
    double *F;                // accumulated flux (edges), nullable
    double wF;                // weight of this stage's flux
    int zeroF;                // overwrite F instead of accumulating
    int comb;
    double tau, g;
};

// One whole barotropic substep of every patch (tiled kernel): input (ua, za)
// is also the combination base; output (uo, zo) must not alias the input.
template <typename R>
struct BTTileArgs {
    DevBtTiles t;
    const R *ua, *za;
    R *uo, *zo;
    const double *G;
    double *F;                // nullable
    int zeroF;
    double tau, g;
    double w1, w3;            // flux weights: SSPRK3 w1, w1, w3; SSPRK2 w1, w1
};

// Buffers and barrier of the persistent barotropic loop: all M substeps in
// one cooperative launch, one workgroup per patch.
template <typename R>
struct BtLoop {
    int M;
    const R *u_in, *z_in;     // loop input (not modified)
    R *bu0, *bu1, *bz0, *bz1; // outputs of the substeps before the last, alternating
    R *u_out, *z_out;         // the last substep's output
    unsigned *bar, *gen;      // arrival counter and generation of the grid barriers (reset by the launch)
    int *err;                 // set when a barrier wait runs out
    unsigned spins;           // polls before a barrier wait runs out
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

// Thickness stage, isopycnal: per-layer flux h_e (c1 X1 + c2 X2 + a_e).
template <typename R>
struct THIsoArgs {
    DevMesh m;
    int L;
    const double *h_in, *h_n;
    const R *X1, *X2;
    double c1, c2;
    const double *a1;         // a_e = ca1 a1 + uA (nullable parts)
    double ca1;
    const double *uA;
    int comb;
    double dt;
    double *h_out, *zeta_out;
    int *nonfinite;
};

// Thickness stage fused with the tracer (temperature) stage: the per-layer
// fluxes h_e v and h_e T_e v of the stage velocity v = c1 X1 + c2 X2 + ca1 a1
// + u^A give the new thickness (z-star: the distributed column total;
// isopycnal: per layer), the stage's w, and the new tracer content; T = hT/h,
// rho = rho0 (1 - alpha (T - T_ref)), zeta = sum h - H.
template <typename R>
struct TracerArgs {
    DevMesh m;
    int L;
    const double *h_in, *h_n;      // stage input thickness, base of the combination
    const double *T_in, *T_n;      // stage input temperature, base of the combination
    const R *X1, *X2;
    double c1, c2;
    const double *a1;
    double ca1;
    const double *uA;
    const double *frac;            // z-star fractions; null for isopycnal
    int comb;
    double dt, kappa_h, kappa_v, rho0, alpha, tref;
    double *h_out, *zeta_out, *T_out, *rho_out;
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
template <typename R>
struct AssembleArgs {
    DevMesh m;
    int L;
    const R *X;               // ut^{n+1} (or u itself when ubar_bt is null)
    const double *ubar_bt;
    const double *h;
    R *U;                     // [E][L] output (may alias X when ubar_bt is null)
    double *ubar;             // [E] split barotropic velocity
    int *nonfinite;
};

// Element-wise type conversion dst[i] = src[i], i < n.
template <typename Tin, typename Tout>
struct ConvArgs {
    const Tin *src;
    Tout *dst;
    size_t n;
};

// Launch geometry: wavefronts (= columns) per workgroup of the column kernels
// and threads per workgroup of the 2D kernels.  The autotuner picks them.
struct Geom {
    int cols_per_block = 4;   // 1, 2, 4, 8 or 16
    int block_2d = 256;       // 64 .. 1024, a multiple of 64
};
bool geom_valid(const Geom &g);

// Workgroups of a column kernel over n columns, and of a 2D kernel over n
// entities (bt_eval: edge blocks, then cell blocks).
int col_blocks(int n, const Geom &g);

// Columns per wavefront of the light streaming column kernels (vertex,
// thickness, assembly, Laplacian and divergence passes), in single-state and
// batched launches alike; their grids count groups of that many columns.
constexpr int kVertexCols = 4, kThickCols = 2, kAssembleCols = 4, kLapCols = 2, kDivCols = 2;
template <int Q>
__host__ __device__ constexpr int wave_groups(int n) { return (n + Q - 1) / Q; }
int flat_blocks(size_t n, const Geom &g);
int bt_blocks(int E, int C, const Geom &g);

// Single-state launches.  The column kernels take NK from a.L and the velocity
// form from whether ubar_add is non-null.
template <typename R> void launch_fe_cell(const FECellArgs<R> &a, const Geom &g, hipStream_t s);
template <typename R> void launch_fe_vertex(const FEVertexArgs<R> &a, const Geom &g, hipStream_t s);
template <typename R> void launch_lap(const LapArgs<R> &a, const Geom &g, hipStream_t s);
template <typename R> void launch_tracer(const TracerArgs<R> &a, const Geom &g, hipStream_t s);
template <typename R> void launch_div(const DivArgs<R> &a, const Geom &g, hipStream_t s);
// wide: 64-bit column addressing whatever the array sizes (edge variant -2)
template <typename R> void launch_fe_edge(const FEEdgeArgs<R> &a, const Geom &g, hipStream_t s, bool wide = false);
// LDS bytes the tiled edge pass needs for tile set t, L layers and type R.
template <typename R> size_t fe_edge_tiled_lds(const DevTiles &t, int L);
template <typename R> void launch_fe_edge_tiled(const FEEdgeArgs<R> &a, const DevTiles &t, hipStream_t s);
template <typename R> void launch_edge_gathers(const FEEdgeArgs<R> &a, const Geom &g, hipStream_t s);
void set_tiled_lds_limit(size_t bytes);
template <typename R> void launch_bt_eval(const BTEvalArgs<R> &a, const Geom &g, hipStream_t s);
// scheme 2 or 3; requires a.t.nP > 0 and the LDS limit set (set_tiled_lds_limit).
template <typename R> void launch_bt_substep(const BTTileArgs<R> &a, int scheme, hipStream_t s);
// Polls before a grid barrier of the persistent loop gives up (about 0.3 s).
constexpr unsigned kBarrierSpins = 1u << 22;
// Workgroups of the persistent loop kernel the device holds at once for this
// tile set, precision and scheme (0 if it cannot launch cooperatively).
template <typename R> int bt_loop_capacity(const DevBtTiles &t, int scheme);
// The whole loop (a: tables, G, F, tau, g and flux weights; the per-substep
// pointers of a are unused); returns the launch's HIP error.
template <typename R> hipError_t launch_bt_loop(const BTTileArgs<R> &a, const BtLoop<R> &l, int scheme, hipStream_t s);
template <typename R> void launch_thickness_iso(const THIsoArgs<R> &a, const Geom &g, hipStream_t s);
template <typename R> void launch_assemble(const AssembleArgs<R> &a, const Geom &g, hipStream_t s);
template <typename R>
void launch_edge_flux_sum(const DevMesh &m, int L, const double *h, const R *X, const double *uA, double *F,
                          hipStream_t s);
template <typename Tin, typename Tout>
void launch_convert(const ConvArgs<Tin, Tout> &a, const Geom &g, hipStream_t s);
void launch_thickness(const THArgs &a, const Geom &g, hipStream_t s);
void launch_recon(const ReconArgs &a, const Geom &g, hipStream_t s);
void launch_zeta_from_h(const DevMesh &m, int L, const double *h, double *zeta, hipStream_t s);
// dst[i] = src[idx[i]] (scatter false) or dst[idx[i]] = src[i] (scatter true), i < n;
// idx is a permutation of 0 .. n-1 and dst does not alias src.
void launch_permute(const double *src, const int32_t *idx, double *dst, int n, bool scatter, const Geom &g,
                    hipStream_t s);

// Batched launches: one kernel launch over the blocks of several states.
// table[b] = (member index into args, that member's block index) for the
// b-th of `blocks` workgroups, in member order; args and table live in
// device memory.  nk and add select the template instance (all members of
// one batched launch share them).
template <typename A>
struct BatchLaunch {
    const A *args;
    const int2 *table;
    int blocks;
};
template <typename R> void launch_fe_cell_batch(const BatchLaunch<FECellArgs<R>> &b, int nk, bool add, const Geom &g, hipStream_t s);
template <typename R> void launch_fe_vertex_batch(const BatchLaunch<FEVertexArgs<R>> &b, int nk, bool add, const Geom &g, hipStream_t s);
template <typename R> void launch_lap_batch(const BatchLaunch<LapArgs<R>> &b, int nk, const Geom &g, hipStream_t s);
template <typename R> void launch_tracer_batch(const BatchLaunch<TracerArgs<R>> &b, int nk, const Geom &g, hipStream_t s);
template <typename R> void launch_div_batch(const BatchLaunch<DivArgs<R>> &b, int nk, const Geom &g, hipStream_t s);
// Geometry of the edge pass over nk register chunks: the two-chunk pass runs
// workgroups of at most kEdge2MaxCols wavefronts (its launch bound); record
// and launch both take their block counts and sizes from it.
constexpr int kEdge2MaxCols = 4;
constexpr int kEdge2Waves = 3;   // waves per SIMD requested for the two-chunk pass
Geom edge_geom(const Geom &g, int nk);
// Template variant of the edge pass: bit 0 canonical stencils with vertex
// chains (mesh), bit 1 implicit vertical mixing, bit 2 biharmonic viscosity
// (parameters), bit 3 64-bit column addressing (some array of L layers per
// entity reaches 4 GiB).
int fe_edge_variant(const DevMesh &m, int L, int vmix, bool del4);
template <typename R> void launch_fe_edge_batch(const BatchLaunch<FEEdgeArgs<R>> &b, int nk, bool add, int var, const Geom &g, hipStream_t s);
template <typename R> void launch_bt_eval_batch(const BatchLaunch<BTEvalArgs<R>> &b, bool delta16, const Geom &g, hipStream_t s);
// table entries (member, patch); ks and lds: the largest over the members
template <typename R>
void launch_bt_substep_batch(const BatchLaunch<BTTileArgs<R>> &b, int scheme, int ks, size_t lds, hipStream_t s);
template <typename R> void launch_thickness_iso_batch(const BatchLaunch<THIsoArgs<R>> &b, int nk, const Geom &g, hipStream_t s);
template <typename R> void launch_assemble_batch(const BatchLaunch<AssembleArgs<R>> &b, int nk, const Geom &g, hipStream_t s);
template <typename Tin, typename Tout>
void launch_convert_batch(const BatchLaunch<ConvArgs<Tin, Tout>> &b, const Geom &g, hipStream_t s);
void launch_thickness_batch(const BatchLaunch<THArgs> &b, int nk, const Geom &g, hipStream_t s);
void launch_recon_batch(const BatchLaunch<ReconArgs> &b, const Geom &g, hipStream_t s);

}  // namespace sse
