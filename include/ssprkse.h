/*
 * ssprkse.h -- C ABI of the MI355X (gfx950) split-explicit ocean step.
 *
 * Implements one step of the SSPRK2-SE / SSPRK3-SE multirate schemes of
 * Lan, Ju, Wang, Gunzburger & Jones, "High-Order Multirate Explicit
 * Time-Stepping Schemes for the Baroclinic-Barotropic Split Dynamics in
 * Primitive Equations" (arXiv 2105.13484), on an unstructured TRiSK C-grid:
 *
 *   - the baroclinic forward-Euler stages (Algorithm 1, Section 3.1) over all
 *     layers at the large step dt,
 *   - the barotropic SSPRK2 / SSPRK3 substep loops (Algorithms 3 and 4) at
 *     dt / M with the interpolated forcing Interp_2 / Interp_3 (force2,
 *     force3),
 *   - the layer-thickness stages with the flux-form SSH reconciliation of
 *     Section 3.4.
 *
 * Memory model: the library never allocates device memory.  The caller
 * provides one device buffer for each mesh and one for each state (sizes
 * from sse_mesh_device_bytes / sse_state_workspace_bytes) and a HIP stream;
 * all kernels run on that stream.  Host-side handles are malloc'd by the
 * library and freed by the *_destroy calls.
 *
 * Numbering: all host arrays passed in or out use the caller's entity
 * numbering; indices are 0-based int32, -1 marks an absent neighbour.
 * 3D arrays are row-major [entity][layer], layer 0 at the surface.
 *
 * Errors: every call returns an sse_status; on failure sse_last_error()
 * returns a thread-local message.  No call throws.  Calls on one handle are
 * not thread-safe; different handles may be used from different threads.
 */
#ifndef SSPRKSE_H
#define SSPRKSE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SSE_OK = 0,
    SSE_EINVAL = 1,      /* invalid argument, mesh table or parameter        */
    SSE_ENOMEM = 2,      /* caller buffer smaller than the size required      */
    SSE_EDEVICE = 3,     /* a HIP runtime call failed                         */
    SSE_ENONFINITE = 4,  /* NaN/Inf in the input or produced by a step        */
    SSE_ESTATE = 5       /* handle used in the wrong state (e.g. not initialised) */
} sse_status;

enum { SSE_SCHEME_SSPRK2 = 2, SSE_SCHEME_SSPRK3 = 3 };
/* Precision (Section 3.4 keeps the conservation in the thickness and
 * reconciliation updates): FP64 runs everything in double.  MIXED stores the
 * velocity-like 3D fields and runs the tendency arithmetic and the barotropic
 * substep state in float, keeping h, rho, zeta, the column sums that form
 * G-bar and F^h, the accumulated transport F^zeta, u^A and D^e in double.
 * MIXED_BT64 is MIXED with the barotropic substep loop (Algorithms 3 and 4)
 * in double, so that zeta is not limited by float rounding inside the loop;
 * its 3D part is MIXED's. */
enum { SSE_FP64 = 0, SSE_MIXED = 1, SSE_MIXED_BT64 = 2 };
enum { SSE_ZSTAR = 0, SSE_ISOPYCNAL = 1 };
/* Reconciliation of Section 3.4: OFF sets u^A = 0; EXACT uses the fluxes the
 * thickness actually received in earlier stages (F^zeta_1, F^zeta_2) inside
 * F^h of the averaged final stage, so the layer SSH equals the barotropic
 * SSH at every stage; LITERAL uses the printed F^h_2 (SSPRK2-SE) and F^h_3
 * (SSPRK3-SE). */
enum { SSE_RECONCILE_OFF = 0, SSE_RECONCILE_EXACT = 1, SSE_RECONCILE_LITERAL = 2 };
/* Vertical viscosity and bottom drag D^u (Section 3.1): EXPLICIT adds them to
 * the forward-Euler tendency of every baroclinic stage (Algorithm 1);
 * IMPLICIT leaves them out of the tendency and applies them afterwards to
 * the whole velocity by a backward-Euler solve, one tridiagonal system per
 * edge column (Algorithm 2, "vertical mixing").  The implicit solve freezes
 * the drag speed |u| at the stage input's; G-bar is the one formed before
 * the solve. */
enum { SSE_VMIX_EXPLICIT = 0, SSE_VMIX_IMPLICIT = 1 };
/* Horizontal viscosity (Section 2 and its remark on hyperviscosity): DEL2 is
 * nu_h lap u with nu_h in m^2/s; DEL4 is the scale-selective -nu_h lap(lap u)
 * with nu_h in m^4/s that replaces it in global runs.  lap is the TRiSK
 * vector Laplacian grad(div u) - k x grad(curl u); the inner Laplacian is
 * zero on coast edges.  DEL4 adds three column passes per stage and
 * workspace for four more 3D fields, and runs the direct edge pass only. */
enum { SSE_HDIFF_DEL2 = 0, SSE_HDIFF_DEL4 = 1 };
/* Tracers (Section 2, equations tracer and eqstate): NONE keeps the density
 * of sse_state_init frozen.  TEMPERATURE carries the layer temperature T: its
 * content h T goes through every thickness stage of the scheme with the
 * stage's own fluxes (centred edge values T_e = (T_c1 + T_c2)/2, the same
 * velocity, u^A included, and the same z-star w as the thickness), with
 * horizontal and vertical diffusion kappa_h, kappa_v, no flux through the
 * surface, the bottom or coasts, and the same convex combinations, so a
 * uniform T stays uniform; after every stage rho = rho0 (1 - eos_alpha
 * (T - eos_tref)) feeds the next baroclinic stage.  T and rho are FP64 in
 * both precisions. */
enum { SSE_TRACER_NONE = 0, SSE_TRACER_TEMPERATURE = 1 };

/*
 * Mesh description (host memory, caller numbering; copied by
 * sse_mesh_create, so the caller may free it afterwards).  Conventions of
 * the TRiSK C-grid (Section 5 opening; Thuburn et al. 2009):
 *   cells_on_edge[e] = (c1, c2), the edge normal points from c1 to c2;
 *   vertices_on_edge[e] = (v1, v2), the tangent k x n points from v1 to v2;
 *   edges_on_cell[i][0..n_edges_on_cell[i]) counter-clockwise;
 *   edges_on_edge / weights_on_edge: v_e = sum_j W[e][j] u[edges_on_edge[e][j]]
 *   reconstructs the tangential velocity; missing entries -1 with weight 0.
 * Lengths in metres, areas in m^2, Coriolis parameter in s^-1.
 */
typedef struct {
    int32_t n_cells, n_edges, n_vertices;
    int32_t max_edges;            /* columns of edges_on_cell (<= 6)          */
    int32_t max_edges2;           /* columns of edges_on_edge (<= 10)         */
    const int32_t *cells_on_edge;     /* [E][2]                               */
    const int32_t *edges_on_cell;     /* [C][max_edges]                       */
    const int32_t *n_edges_on_cell;   /* [C]                                  */
    const int32_t *vertices_on_edge;  /* [E][2]                               */
    const int32_t *edges_on_vertex;   /* [V][3]                               */
    const int32_t *edges_on_edge;     /* [E][max_edges2]                      */
    const int32_t *n_edges_on_edge;   /* [E]                                  */
    const double *weights_on_edge;    /* [E][max_edges2]                      */
    const double *dc_edge;            /* [E] cell-centre distance d_e         */
    const double *dv_edge;            /* [E] vertex distance l_e              */
    const double *f_edge;             /* [E] Coriolis parameter at edges      */
    const double *area_cell;          /* [C]                                  */
    const double *bottom_depth;       /* [C] H (total column height at rest)  */
    const double *area_triangle;      /* [V]                                  */
    const uint8_t *cell_mask;         /* [C] 1 = ocean, 0 = land              */
} sse_mesh_desc;

/*
 * Run parameters.  Every physical constant is explicit:
 *   n_layers L (1..128); scheme SSE_SCHEME_SSPRK2 | SSE_SCHEME_SSPRK3;
 *   substeps M >= 1 (barotropic step dt / M); precision SSE_FP64 |
 *   SSE_MIXED | SSE_MIXED_BT64;
 *   vcoord SSE_ZSTAR | SSE_ISOPYCNAL (Section 2, vertical coordinate);
 *   reconcile SSE_RECONCILE_*; vmix SSE_VMIX_*; hdiff SSE_HDIFF_*; tracer
 *   SSE_TRACER_*; dt > 0 (s); gravity g; rho0 (Boussinesq reference
 *   density); nu_h (horizontal viscosity, m^2/s for DEL2, m^4/s for DEL4);
 *   nu_v (vertical viscosity, m^2/s); c_drag (bottom drag of Section 5,
 *   dimensionless); kappa_h, kappa_v (tracer diffusivities, m^2/s) and
 *   eos_alpha (1/K), eos_tref (deg C) of the linear EOS, read in tracer runs
 *   only.
 */
typedef struct {
    int32_t n_layers, scheme, substeps, precision, vcoord, reconcile, vmix, hdiff, tracer;
    double dt, gravity, rho0, nu_h, nu_v, c_drag;
    double kappa_h, kappa_v, eos_alpha, eos_tref;
} sse_params;

typedef struct sse_mesh sse_mesh;
typedef struct sse_state sse_state;

/* Thread-local description of the last failure ("" if none). */
const char *sse_last_error(void);

/* Library version string. */
const char *sse_version(void);

/* Host-only check of a mesh description: index ranges, the two-cell and
 * two-vertex structure of every edge, positive lengths and areas, and the
 * antisymmetry l_e d_e W[e][e'] = -l_e' d_e' W[e'][e] that makes the Coriolis
 * term energy neutral.  Touches no GPU.  SSE_EINVAL on the first violation. */
int sse_mesh_validate(const sse_mesh_desc *d);

/* Device bytes a mesh occupies (for the caller's allocation).  The size of
 * the barotropic patch tables depends on the cell-edge topology, so the call
 * reads cells_on_edge, edges_on_cell and n_edges_on_cell (SSE_EINVAL if they
 * are NULL or out of range; sse_mesh_create validates everything).  The
 * partition is cached by a hash of those tables. */
int sse_mesh_device_bytes(const sse_mesh_desc *d, size_t *bytes);

/* Validate, lay out and upload a mesh into dev_buf (>= sse_mesh_device_bytes,
 * 256-byte aligned, owned by the caller and kept alive until destroy).
 * stream: hipStream_t used for the upload (NULL = default stream); the call
 * returns after the upload completed. */
int sse_mesh_create(const sse_mesh_desc *d, void *dev_buf, size_t bytes, void *stream,
                    sse_mesh **out);
int sse_mesh_destroy(sse_mesh *m);

/* Device workspace of one state (prognostic fields, stage buffers, the 2D
 * accumulators of the reconciliation and the barotropic loop). */
int sse_state_workspace_bytes(const sse_mesh *m, const sse_params *p, size_t *bytes);

/* Create a state on mesh m in the caller's device workspace (>= the size
 * above, 256-byte aligned); all kernels of this state run on `stream`
 * (a hipStream_t, NULL = default stream).  SSE_ENOMEM if bytes is too small,
 * SSE_EINVAL on bad parameters. */
int sse_state_create(const sse_mesh *m, const sse_params *p, void *dev_workspace, size_t bytes,
                     void *stream, sse_state **out);
int sse_state_destroy(sse_state *s);

/* Set the initial state from host arrays in the caller's numbering:
 * h [C][L] layer thicknesses, u [E][L] normal velocities, rho [C][L] frozen
 * layer densities (EOS evaluated by the caller), h_ref [C][L] z-star
 * reference thicknesses (may be NULL for isopycnal).  zeta is derived as
 * sum_k h_k - H (Section 2, definition of zeta); velocities on edges next to
 * land are forced to 0.  SSE_ENONFINITE if any input is NaN/Inf. */
int sse_state_init(sse_state *s, const double *h, const double *u, const double *rho,
                   const double *h_ref);

/* Tracer runs: the layer temperature T [C][L] (host, row-major, caller
 * numbering; land cells are ignored), required once after sse_state_init and
 * before the first step; it also sets rho from the EOS.  sse_read_tracer
 * copies the state's temperature out.  SSE_EINVAL / SSE_ESTATE when the
 * state carries no tracer; SSE_ENONFINITE for non-finite input. */
int sse_state_set_tracer(sse_state *s, const double *T);
int sse_read_tracer(const sse_state *s, double *T);

/* Enqueue n steps t -> t + n dt on the state's stream, wait, and check the
 * state for NaN/Inf.  SSE_ENONFINITE after a blow-up (the state keeps the
 * values of the last step, for inspection). */
int sse_step(sse_state *s, int32_t n);

/* Enqueue n steps and return immediately; sse_sync waits and reports
 * SSE_ENONFINITE like sse_step. */
int sse_step_async(sse_state *s, int32_t n);
int sse_sync(sse_state *s);

/* Copy the state to host arrays in the caller's numbering; any pointer may be
 * NULL.  h [C][L], u [E][L], zeta [C] = sum h - H, ubar [E] = the barotropic
 * velocity of (BBspl) for the current u and h.  Waits for the stream. */
int sse_read_state(const sse_state *s, double *h, double *u, double *zeta, double *ubar);

/* Per-kernel-class timing with HIP events on the state's stream.
 * class_mask: bit c set = record an event pair around every launch of class c
 * during subsequent steps (0 disables timing).  sse_profile_read returns, per
 * class, the number of launches and the summed milliseconds, then resets.
 * Classes: 0 baroclinic edge pass, 1 baroclinic cell pass, 2 vertex pass,
 * 3 barotropic substep evaluation, 4 thickness stage, 5 other 2D/assembly. */
enum { SSE_PROF_FE_EDGE = 0, SSE_PROF_FE_CELL = 1, SSE_PROF_FE_VERTEX = 2,
       SSE_PROF_BT_EVAL = 3, SSE_PROF_THICKNESS = 4, SSE_PROF_OTHER = 5, SSE_PROF_NCLASS = 6 };
int sse_profile_enable(sse_state *s, int class_mask);
int sse_profile_read(sse_state *s, int32_t *launches, double *milliseconds);

/* Kernel variant of the baroclinic edge pass (results are identical up to
 * the order of FP64 rounding in no operation: every variant performs the same
 * arithmetic on the same operands).  variant -1: direct gathers from global
 * memory, addressing each column by a 32-bit offset into its array while the
 * largest per-layer array (entities x L x 8 bytes) stays below 4 GiB and by a
 * 64-bit address otherwise; -2: direct gathers with 64-bit addresses always;
 * 0, 1, 2: the operands of tiles of 8, 16 or 32 consecutive edges are
 * first staged in LDS.  SSE_EINVAL if the variant is unknown or does not fit
 * this mesh (a tile list longer than 255 columns) or the device's LDS for the
 * state's layer count and precision.  The default is -1.  The first
 * selection of a tiled variant on a mesh builds its gather lists on the host
 * and uploads them (on the state's stream, synchronously) into space the
 * mesh buffer reserves for them.  Applies to subsequent steps; the autotuner
 * in the Python package calls it. */
int sse_state_set_edge_variant(sse_state *s, int variant);
int sse_state_get_edge_variant(const sse_state *s, int *variant);

/* Kernel layout of the barotropic substep loops (Algorithms 3 and 4); the
 * results are bitwise the same.  0: one launch per forward-Euler evaluation
 * (3M per SSPRK3 loop, 2M per SSPRK2 loop).  1: one launch per substep: the
 * mesh is cut into patches of a few hundred cells, and one workgroup carries
 * its patch, extended by the halo rings the substep's evaluations read,
 * through all evaluations of the substep in LDS.  2: one cooperative launch
 * per loop (persistent): every patch has its own workgroup for all M
 * substeps, keeps its stencil tables, frozen forcing and F^zeta sums in
 * registers, and waits at a grid barrier between substeps; available when
 * the device holds a workgroup for every patch at once (small meshes: a few
 * hundred patches).  A barrier wait is bounded: if one runs out, the step
 * call reports SSE_EDEVICE and the state is not valid.  Steps captured in a
 * HIP graph, and batch members, run variant 1 in place of 2.  The default is
 * 1 when the mesh has such patches (sse_mesh_create builds them when every
 * patch's halo region fits a workgroup and every reconstruction stencil stays
 * within the two cells of its edge) and they fit the device's LDS, else 0.
 * SSE_EINVAL for 1 or 2 where they do not apply.  Each member of a batch uses
 * its own variant. */
int sse_state_set_bt_variant(sse_state *s, int variant);
int sse_state_get_bt_variant(const sse_state *s, int *variant);

/* Device bytes one state of these parameters on this mesh needs in total:
 * the mesh image (sse_mesh_device_bytes, with its topology checks) plus the
 * workspace (sse_state_workspace_bytes).  Host only; allocates nothing.  For
 * admission control by a device-memory budget. */
int sse_footprint_bytes(const sse_mesh_desc *d, const sse_params *p, size_t *bytes);

/* Launch geometry of the state's kernels; results do not depend on it.
 * cols_per_block: wavefronts per workgroup of the column kernels (one
 * wavefront per vertical column), 1, 2, 4, 8 or 16 (the edge pass over more
 * than 64 layers takes at most 4, to keep its operands in registers);
 * block_2d: threads per workgroup of the 2D kernels (barotropic evaluations,
 * reconciliation), a multiple of 64 in [64, 1024].  Defaults 4 and 256.
 * SSE_EINVAL otherwise. */
int sse_state_set_geometry(sse_state *s, int cols_per_block, int block_2d);

/* enable != 0: the next sse_step / sse_step_async captures the launches of one
 * step on the state's stream into a HIP graph and every step then replays
 * it (one graph launch per step).  The stream must not be the null stream
 * (SSE_EINVAL).  Changing the geometry, the edge variant or this flag drops the
 * graph.  Per-class profiling does not apply to graph replays. */
int sse_state_use_graph(sse_state *s, int enable);

/*
 * Batched ensembles (many independent states advanced together).
 *
 * A batch advances its member states by whole SSPRK-SE steps with one kernel
 * launch per phase of the step across all members: the launch sequence of
 * one step (Sections 3.2 / 3.3; the barotropic loops of Algorithms 3 / 4 run
 * max M substeps, a member with a smaller M taking part in its first M) is
 * recorded for every member and equal launches are merged.  Members keep
 * their own mesh, parameters (L, M, dt, ...) and workspace, and produce
 * bit-for-bit the results they produce alone.  They must share precision,
 * scheme and vertical coordinate and have been created on the batch's
 * stream.  Batched launches use the direct-gather edge pass and the batch's
 * geometry.  The library allocates nothing: sse_batch_program_bytes gives
 * the size of the device buffer that sse_batch_compile fills with the
 * merged argument blocks and workgroup tables (256-byte aligned; the caller
 * owns it and keeps it alive while the batch steps).  Adding or removing a
 * member, or changing the geometry, invalidates the compiled program; these
 * calls touch host state only, so without HIP graphs they may be made while
 * launches enqueued by sse_batch_step_async run, provided the buffer those
 * launches read stays allocated until sse_batch_sync returns.  A member must not be stepped on
 * its own while the batch runs.
 */
typedef struct sse_batch sse_batch;
int sse_batch_create(void *hip_stream, sse_batch **out);
int sse_batch_destroy(sse_batch *b);
int sse_batch_add(sse_batch *b, sse_state *s);
int sse_batch_remove(sse_batch *b, sse_state *s);
int sse_batch_size(const sse_batch *b, int32_t *n);
int sse_batch_set_geometry(sse_batch *b, int cols_per_block, int block_2d);
int sse_batch_program_bytes(sse_batch *b, size_t *bytes);
int sse_batch_compile(sse_batch *b, void *dev_buf, size_t bytes);
/* Number of batched launches in one step of the compiled program. */
int sse_batch_launches_per_step(sse_batch *b, int32_t *n);
/* enable != 0: one step of the batch is captured into a HIP graph on first
 * use and replayed (non-null stream required). */
int sse_batch_use_graph(sse_batch *b, int enable);
/* Enqueue n steps of every member / wait and check every member's
 * non-finite flag (SSE_ENONFINITE if any member blew up; sse_sync on a
 * member tells which). */
int sse_batch_step_async(sse_batch *b, int32_t n);
int sse_batch_sync(sse_batch *b);
int sse_batch_step(sse_batch *b, int32_t n);

/*
 * Per-kernel debug entry points (host arrays, caller numbering).  They use
 * the state's stage buffers as scratch and leave its prognostic fields
 * untouched.
 */

/* Algorithm 1, Baroclinic_FEuler(u, ut = u - ubar, zeta, h, dt):
 * inputs u [E][L], ubar [E], zeta [C], h [C][L]; outputs ut1 [E][L] (after the
 * G-bar subtraction) and G [E]. */
int sse_debug_baroclinic_feuler(sse_state *s, const double *u, const double *ubar,
                                const double *zeta, const double *h, double dt,
                                double *ut1, double *G);

/* Algorithm 3 (scheme 2) or 4 (scheme 3) with M substeps over dt and G frozen:
 * inputs ubar [E], zeta [C], G [E]; outputs ubar1 [E], zeta1 [C] and the
 * accumulated flux F^zeta [E] of Section 3.4. */
int sse_debug_barotropic_substep(sse_state *s, int32_t scheme, int32_t M, double dt,
                                 const double *ubar, const double *zeta, const double *G,
                                 double *ubar1, double *zeta1, double *Fzeta);

/* Measurement aid for callers that compare the baroclinic edge pass with
 * the cost of its memory accesses alone: enqueues on the state's stream (and
 * returns without waiting) one launch that gathers, for every edge, the same
 * layer columns the direct edge pass reads (u and u^n at the edge, h, rho,
 * K - nu_h div u and w at its two cells, its 10 stencil edges and the
 * vorticity of the 10 vertices of their chains; Algorithm 1's operands) from
 * the state's current arrays and writes their sum into a stage buffer that
 * every step overwrites before reading.  The state steps on unchanged.
 * SSE_EINVAL without canonical stencils, above 64 layers or with arrays of
 * 4 GiB or more; SSE_ESTATE before sse_state_init or while the state is being
 * recorded into a batch; SSE_EDEVICE if the launch fails. */
int sse_debug_edge_gathers(sse_state *s);

/* Polls a grid barrier of the persistent barotropic loop (variant 2) makes
 * before it gives up, reports the timeout and lets every workgroup finish;
 * 0 restores the default (about 0.3 s of waiting).  For tests of that error
 * path: with 1, the first workgroup to reach a barrier finds it closed and
 * gives up at once (whenever the launch has more than one workgroup), the
 * step call returns SSE_EDEVICE and the state must be initialised again.
 * SSE_EINVAL for a NULL state. */
int sse_debug_set_barrier_spins(sse_state *s, uint32_t spins);

/* One thickness stage h_out = h_in + dt T^h(h_in, u + uA) (Section 3.4 revised
 * thickness updates) with the state's vertical coordinate: inputs h_in [C][L],
 * u [E][L], uA [E]; outputs h_out [C][L] and zeta_out [C] = sum h_out - H. */
int sse_debug_thickness_stage(sse_state *s, const double *h_in, const double *u, const double *uA,
                              double dt, double *h_out, double *zeta_out);

/*
 * Allocation-free barotropic loop, for callers that cannot allocate device
 * memory or pass a workspace (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc).  Same operation as
 * sse_debug_barotropic_substep (Algorithm 3 for scheme 2, Algorithm 4 for
 * scheme 3: M substeps over dt with G frozen, accumulating F^zeta of Section
 * 3.4), in the state's barotropic precision (FP32 for SSE_MIXED, else FP64),
 * but on DEVICE arrays in the caller's numbering: inputs ubar [E], zeta [C],
 * G [E]; outputs ubar1 [E], zeta1 [C], Fzeta [E] (outputs may alias inputs:
 * every input is read before any output is written).  The state supplies the
 * mesh, gravity, the barotropic kernel variant (variant 2, the persistent
 * loop kernel, runs as variant 1 here) and the stream; its own fields and
 * workspace are not touched.  The loop's stages live in a static
 * device array of 64 MiB per device, reserved when the library's code is
 * loaded on that device and held until the process ends; its address is
 * resolved by sse_state_create.  The call allocates nothing, enqueues its
 * kernels on the state's stream and returns without waiting.  All calls on
 * one device share that array, which keeps the last call's contents: calls
 * that overlap in time on one device race.  SSE_ENOMEM if the mesh needs more
 * than the array ((6 E + 4 C) x 8 bytes plus alignment); SSE_EINVAL for NULL
 * arguments, scheme not 2 or 3, M < 1, dt <= 0, or a current device other
 * than the state's; SSE_EDEVICE if a launch fails or the array's address is
 * unavailable.
 */
int sse_barotropic_substep_noalloc(sse_state *s, int32_t scheme, int32_t M, double dt,
                                   const double *ubar, const double *zeta, const double *G,
                                   double *ubar1, double *zeta1, double *Fzeta);

#ifdef __cplusplus
}
#endif

#endif /* SSPRKSE_H */
