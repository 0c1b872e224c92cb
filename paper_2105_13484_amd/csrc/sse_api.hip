// C ABI: mesh upload, state workspace, the SSPRK2-SE / SSPRK3-SE step
// orchestration, state init/read, debug entry points and per-class timing.
//
// Step structure (Section 3 of the paper; the reconciliation of Section 3.4):
//   SSPRK3-SE  FE1 -> BT1 -> TH1 -> FE2 -> BT2 -> TH2 -> FE3 -> BT3 -> TH3 -> assemble
//   SSPRK2-SE  FE1 -> BT1 -> TH1 -> FE2 -> BT2 -> TH2 -> assemble
// FE = baroclinic forward Euler (Algorithm 1: cell, vertex and edge passes),
// BT = barotropic substep loop (Algorithm 3 or 4), TH = thickness stage with
// the reconciliation deficits.  Everything is enqueued on the state's stream.
//
// Precision: the orchestration is a template over the real type R of the
// velocity-like 3D fields (double for SSE_FP64, float for SSE_MIXED and
// SSE_MIXED_BT64); the barotropic substep state is R, except that
// SSE_MIXED_BT64 keeps it double; thickness, density, SSH and all 2D fields
// handed between stages are double in every mode.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <map>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <string>
#include <type_traits>
#include <vector>

#include "sse_kernels.h"

using namespace sse;

// Scratch of the allocation-free barotropic entry point
// (sse_barotropic_substep_noalloc): one array per device, held until the
// process ends and shared by every call on that device.  Host code never
// passes the symbol itself: its device address comes from
// hipGetSymbolAddress once per device (scratch_address) and only that
// address reaches kernels.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) double scratch[kStaticScratchBytes / sizeof(double)];

namespace {

constexpr int kMaxDevices = 64;
std::atomic<void *> g_scratch[kMaxDevices];

// Resolves (once per device, with that device current) the address of this
// device's scratch array; nullptr if the runtime cannot give it.
void *scratch_address(int dev) {
    if (dev < 0 || dev >= kMaxDevices) return nullptr;
    void *p = g_scratch[dev].load(std::memory_order_acquire);
    if (p) return p;
    void *q = nullptr;
    if (hipGetSymbolAddress(&q, HIP_SYMBOL(scratch)) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    g_scratch[dev].store(q, std::memory_order_release);
    return q;
}

// Device workspace of one state.  Arrays marked R hold the mode's real type.
struct Work {
    void *U, *T1, *T2;                       // R [E][L]: u^n and two stage buffers
    void *B, *Wt;                            // R [C][L]: K - nu_h div u, w at layer tops
    void *Z;                                 // R [V][L]: relative vorticity
    void *bt_u1, *bt_uh, *bt_ua, *bt_uo;     // [E] substep stages, loop input / output, in the loop's type
    void *bt_z1, *bt_zh, *bt_za, *bt_zo;     // [C]
    double *Hs, *H1, *H2, *frac, *rho;       // [C][L]
    double *ubar_n, *ub1, *ub2, *ub_half, *ubar_new, *G0, *G1, *Gh, *Gi, *Fz1, *Fz2, *Fz3, *Sh1, *Fh1, *Sh2,
        *Fh2, *Sh3, *Pp, *Ftot, *uA;         // [E]
    double *zeta_n, *z1, *z_half, *Kbot, *bt_zout;  // [C]
    int *flag;                               // [0]: non-finite flag; [16], [48]: barrier counter and
                                             // generation, [32]: barrier error of the persistent
                                             // barotropic loop
    void *D1, *L1, *D2, *Z2;                 // R, biharmonic runs only: div u [C][L], lap u [E][L],
                                             // div(lap u) [C][L], curl(lap u) [V][L]
    double *Tn, *T1s, *Th;                   // [C][L], tracer runs only: temperature of the state,
                                             // of the first stage and of the n+1/2 stage
    void *ubar_r;                            // R [E]: the barotropic velocity an edge pass adds or
                                             // subtracts, rounded to R (mixed precision)
};

constexpr int kR3E = 3, kR3C = 2, kR3V = 1, kR2E = 4, kR2C = 4;  // arrays of type R
constexpr int kD3C = 5, kD2E = 20, kD2C = 5;                    // arrays of type double

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

size_t real_size(int precision) { return precision == SSE_FP64 ? sizeof(double) : sizeof(float); }

// Bytes of the barotropic loop's real type: FP32 only in SSE_MIXED.
size_t bt_size(int precision) { return precision == SSE_MIXED ? sizeof(float) : sizeof(double); }

size_t workspace_bytes(int C, int E, int V, int L, size_t rs, size_t bs, int hdiff, int tracer) {
    size_t b = 0;
    if (tracer) b += 3 * align_up((size_t)C * L * 8);
    b += align_up((size_t)E * rs);  // ubar_r, last
    if (hdiff == SSE_HDIFF_DEL4)
        b += align_up((size_t)E * L * rs) + 2 * align_up((size_t)C * L * rs) + align_up((size_t)V * L * rs);
    b += kR3E * align_up((size_t)E * L * rs);
    b += kR3C * align_up((size_t)C * L * rs);
    b += kR3V * align_up((size_t)V * L * rs);
    b += kR2E * align_up((size_t)E * bs);
    b += kR2C * align_up((size_t)C * bs);
    b += kD3C * align_up((size_t)C * L * 8);
    b += kD2E * align_up((size_t)E * 8);
    b += kD2C * align_up((size_t)C * 8);
    b += kAlign;  // flag
    return b;
}

Work carve(void *buf, int C, int E, int V, int L, size_t rs, size_t bs, int hdiff, int tracer) {
    char *p = static_cast<char *>(buf);
    auto take = [&](size_t n) {
        void *r = p;
        p += align_up(n);
        return r;
    };
    Work w{};
    void **r3e[] = {&w.U, &w.T1, &w.T2};
    for (auto q : r3e) *q = take((size_t)E * L * rs);
    void **r3c[] = {&w.B, &w.Wt};
    for (auto q : r3c) *q = take((size_t)C * L * rs);
    w.Z = take((size_t)V * L * rs);
    void **r2e[] = {&w.bt_u1, &w.bt_uh, &w.bt_ua, &w.bt_uo};
    for (auto q : r2e) *q = take((size_t)E * bs);
    void **r2c[] = {&w.bt_z1, &w.bt_zh, &w.bt_za, &w.bt_zo};
    for (auto q : r2c) *q = take((size_t)C * bs);
    double **d3c[] = {&w.Hs, &w.H1, &w.H2, &w.frac, &w.rho};
    for (auto q : d3c) *q = static_cast<double *>(take((size_t)C * L * 8));
    double **d2e[] = {&w.ubar_n, &w.ub1, &w.ub2, &w.ub_half, &w.ubar_new, &w.G0, &w.G1, &w.Gh, &w.Gi, &w.Fz1,
                      &w.Fz2, &w.Fz3, &w.Sh1, &w.Fh1, &w.Sh2, &w.Fh2, &w.Sh3, &w.Pp, &w.Ftot, &w.uA};
    for (auto q : d2e) *q = static_cast<double *>(take((size_t)E * 8));
    double **d2c[] = {&w.zeta_n, &w.z1, &w.z_half, &w.Kbot, &w.bt_zout};
    for (auto q : d2c) *q = static_cast<double *>(take((size_t)C * 8));
    w.flag = reinterpret_cast<int *>(p);
    p += kAlign;
    w.D1 = w.L1 = w.D2 = w.Z2 = nullptr;
    if (hdiff == SSE_HDIFF_DEL4) {
        w.D1 = take((size_t)C * L * rs);
        w.L1 = take((size_t)E * L * rs);
        w.D2 = take((size_t)C * L * rs);
        w.Z2 = take((size_t)V * L * rs);
    }
    w.Tn = w.T1s = w.Th = nullptr;
    if (tracer) {
        w.Tn = static_cast<double *>(take((size_t)C * L * 8));
        w.T1s = static_cast<double *>(take((size_t)C * L * 8));
        w.Th = static_cast<double *>(take((size_t)C * L * 8));
    }
    w.ubar_r = take((size_t)E * rs);
    return w;
}

template <typename R>
R *rp(void *p) { return static_cast<R *>(p); }

constexpr int kPatchCells = 512;  // cells per locality patch of the internal numbering
constexpr int kLocalSpan = 1024;  // index distance below which two cells count as near

// Share of edges whose two cells are at most kLocalSpan apart in a numbering
// (the caller's if o is null).
double local_share(const sse_mesh_desc *d, const MeshOrder *o) {
    long near = 0;
    for (int e = 0; e < d->n_edges; ++e) {
        int a = d->cells_on_edge[2 * (size_t)e], b = d->cells_on_edge[2 * (size_t)e + 1];
        if (a < 0 || b < 0) continue;
        if (o) { a = o->cell_new[a]; b = o->cell_new[b]; }
        near += std::abs(a - b) <= kLocalSpan;
    }
    return d->n_edges ? (double)near / d->n_edges : 1.0;
}

void identity_order(const sse_mesh_desc *d, MeshOrder &o) {
    auto iota = [](std::vector<int32_t> &v, int n) {
        v.resize(n);
        for (int i = 0; i < n; ++i) v[i] = i;
    };
    iota(o.cell_old, d->n_cells);
    iota(o.cell_new, d->n_cells);
    iota(o.edge_old, d->n_edges);
    iota(o.edge_new, d->n_edges);
    iota(o.vert_old, d->n_vertices);
    iota(o.vert_new, d->n_vertices);
}

// Rows of a host array between the caller's numbering and the internal one
// (old_of_new[i] = caller index of internal entity i).
template <typename T>
void rows_to_internal(const T *user, T *internal, const std::vector<int32_t> &old_of_new, size_t row) {
    for (size_t i = 0; i < old_of_new.size(); ++i)
        std::memcpy(internal + i * row, user + (size_t)old_of_new[i] * row, row * sizeof(T));
}
template <typename T>
void rows_to_user(const T *internal, T *user, const std::vector<int32_t> &old_of_new, size_t row) {
    for (size_t i = 0; i < old_of_new.size(); ++i)
        std::memcpy(user + (size_t)old_of_new[i] * row, internal + i * row, row * sizeof(T));
}

int hip_fail(hipError_t e, const char *what) {
    set_error(std::string(what) + ": " + hipGetErrorString(e));
    return SSE_EDEVICE;
}

#define SSE_HIP(call)                                   \
    do {                                                \
        hipError_t _e = (call);                         \
        if (_e != hipSuccess) return hip_fail(_e, #call); \
    } while (0)

bool all_finite(const double *x, size_t n) {
    for (size_t i = 0; i < n; ++i)
        if (!std::isfinite(x[i])) return false;
    return true;
}

// Launch recording.  While a batch compiles its program, the building blocks
// below do not launch: they append their argument block under a structural
// key (seq = launch site in step order; j = substep evaluation inside a
// barotropic loop), so that the same launch of every member can be merged
// into one batched launch.
enum class Kind : int { FE_CELL, FE_VERTEX, FE_EDGE, BT_EVAL, BT_TILE, THICK, THICK_ISO, RECON, ASSEMBLE, CONV_DF, CONV_FD, LAP, DIV, TRACER };

struct RecEntry {
    Kind kind;
    int seq, j;
    int nk;
    int var;      // kernel variant flag that must match within a batched launch
    bool add;
    int blocks;
    size_t lds = 0;   // dynamic LDS bytes the launch needs (tiled substeps)
    std::vector<uint8_t> args;
};

struct Recorder {
    int seq = 0;
    int loop_seq = -1;
    std::vector<RecEntry> entries;
};

}  // namespace

struct sse_state {
    const sse_mesh *mesh = nullptr;
    sse_params p{};
    hipStream_t stream = nullptr;
    Work w{};
    size_t bytes = 0;
    int device = 0;          // the device current at creation
    size_t rs = 8;           // bytes of the real type R
    bool bt64 = true;        // the barotropic loop runs in FP64 (SSE_FP64, SSE_MIXED_BT64)
    bool initialized = false;
    bool tracer_set = false; // tracer runs: the temperature has been given
    Geom geom{};             // launch geometry (autotuner knob)
    int edge_variant = -1;   // -1: direct gathers (-2: with 64-bit column addresses); 0 / 1 / 2: LDS tiles of 8 / 16 / 32 edges
    int bt_variant = 0;      // 0: one launch per barotropic evaluation; 1: one per substep (patches);
                             // 2: one cooperative launch per loop, one workgroup per patch
    int bt_capacity[2] = {0, 0};  // workgroups of the persistent loop kernel the device holds at once
                                  // (SSPRK2, SSPRK3 forms)
    bool capturing = false;  // a HIP graph capture of the step is in progress
    hipError_t launch_error = hipSuccess;  // the last failed cooperative launch, reported by the step call
    unsigned barrier_spins = kBarrierSpins;  // polls before a barrier of the persistent loop gives up
    size_t lds_max = 0;      // LDS bytes per workgroup on the state's device
    Recorder *rec = nullptr; // non-null while a batch records this state's step
    sse_batch *batch = nullptr;
    // single-state step captured as a HIP graph
    bool use_graph = false;
    hipGraphExec_t graph_exec = nullptr;
    // profiling
    bool prof = false;
    int prof_mask = 0;
    std::vector<hipEvent_t> events;
    std::vector<int> rec_class;
    size_t ev_used = 0;
    long nlaunch[SSE_PROF_NCLASS] = {};
    double ms[SSE_PROF_NCLASS] = {};
};

namespace {

// ---- per-class event timing ------------------------------------------------
void prof_flush(sse_state *s) {
    if (s->ev_used == 0) return;
    (void)hipStreamSynchronize(s->stream);
    for (size_t i = 0; i < s->ev_used / 2; ++i) {
        float t = 0.f;
        if (hipEventElapsedTime(&t, s->events[2 * i], s->events[2 * i + 1]) == hipSuccess) {
            s->ms[s->rec_class[i]] += t;
            s->nlaunch[s->rec_class[i]] += 1;
        }
    }
    s->ev_used = 0;
    s->rec_class.clear();
}

struct ProfScope {
    sse_state *s;
    int cls;
    bool active;
    ProfScope(sse_state *st, int c)
        : s(st), cls(c),
          active(st->prof && !st->rec && !st->events.empty() && ((st->prof_mask >> c) & 1)) {
        if (!active) return;
        if (s->ev_used + 2 > s->events.size()) prof_flush(s);
        (void)hipEventRecord(s->events[s->ev_used], s->stream);
    }
    ~ProfScope() {
        if (!active) return;
        (void)hipEventRecord(s->events[s->ev_used + 1], s->stream);
        s->ev_used += 2;
        s->rec_class.push_back(cls);
    }
};

template <typename A>
void record(sse_state *s, Kind kind, const A &a, int nk, bool add, int blocks, int j = -1, int var = 0) {
    Recorder &r = *s->rec;
    RecEntry e;
    e.kind = kind;
    e.j = j;
    e.seq = j >= 0 ? r.loop_seq : r.seq++;
    e.nk = nk;
    e.var = var;
    e.add = add;
    e.blocks = blocks;
    e.args.assign(reinterpret_cast<const uint8_t *>(&a), reinterpret_cast<const uint8_t *>(&a) + sizeof(A));
    r.entries.push_back(std::move(e));
}

int nk_of(int L) { return L <= kWave ? 1 : 2; }

// The tiled barotropic substep kernel is usable: the mesh has patches and
// the largest patch's LDS fits the device.
bool bt_tiles_fit(const sse_state *s) {
    const DevBtTiles &t = s->mesh->bt;
    return t.nP > 0 && (s->bt64 ? t.lds_d : t.lds_f) <= s->lds_max;
}

// The persistent loop kernel can give every patch its own workgroup at once
// (a cooperative launch of the XCD-padded patch count) for this scheme.
bool bt_loop_fits(const sse_state *s, int scheme) {
    const int nP = s->mesh->bt.nP;
    return bt_tiles_fit(s) && kXcd * ((nP + kXcd - 1) / kXcd) <= s->bt_capacity[scheme == SSE_SCHEME_SSPRK3 ? 1 : 0];
}

// ---- building blocks -------------------------------------------------------
template <typename Tin, typename Tout>
void convert(sse_state *s, const Tin *src, Tout *dst, size_t n);

template <typename R>
void fe_pass(sse_state *s, const R *X, const double *add, const double *sub, const double *h, const double *zeta,
             int comb, R *out, double *G, double *sum_h, double *sum_hu, double *sum_hp, double pa, double pb,
             double *Gi, const double *Ga, const double *Gb, int interp) {
    const DevMesh &m = s->mesh->d;
    const sse_params &p = s->p;
    Work &w = s->w;
    const bool zstar = p.vcoord == SSE_ZSTAR;
    const int nk = nk_of(p.n_layers);
    const bool del4 = p.hdiff == SSE_HDIFF_DEL4;
    // the FP32 edge pass reads the barotropic velocity of every stencil edge:
    // rounded to FP32 once here instead of in every gather
    if constexpr (sizeof(R) == 4) convert<double, float>(s, add ? add : sub, rp<float>(w.ubar_r), (size_t)m.E);
    {
        ProfScope ps(s, SSE_PROF_FE_CELL);
        FECellArgs<R> a{m, p.n_layers, X, add, h, zstar ? w.frac : nullptr, del4 ? 0.0 : p.nu_h, rp<R>(w.B),
                        del4 ? rp<R>(w.D1) : nullptr, rp<R>(w.Wt), w.Kbot};
        if (s->rec) record(s, Kind::FE_CELL, a, nk, add != nullptr, col_blocks(m.C, s->geom));
        else launch_fe_cell<R>(a, s->geom, s->stream);
    }
    {
        ProfScope ps(s, SSE_PROF_FE_VERTEX);
        FEVertexArgs<R> a{m, p.n_layers, X, add, rp<R>(w.Z)};
        if (s->rec) record(s, Kind::FE_VERTEX, a, nk, add != nullptr, col_blocks(wave_groups<kVertexCols>(m.V), s->geom));
        else launch_fe_vertex<R>(a, s->geom, s->stream);
    }
    if (!del4 && s->rec) {
        // keep the launch sequence aligned with members that run the three
        // biharmonic passes, so that batches merge the later phases
        s->rec->seq += 3;
    } else if (del4) {
        // lap u at edges, then its divergence at cells and its curl at vertices
        ProfScope ps(s, SSE_PROF_OTHER);
        LapArgs<R> la{m, p.n_layers, rp<R>(w.D1), rp<R>(w.Z), rp<R>(w.L1)};
        if (s->rec) record(s, Kind::LAP, la, nk, false, col_blocks(wave_groups<kLapCols>(m.E), s->geom));
        else launch_lap<R>(la, s->geom, s->stream);
        DivArgs<R> da{m, p.n_layers, rp<R>(w.L1), rp<R>(w.D2)};
        if (s->rec) record(s, Kind::DIV, da, nk, false, col_blocks(wave_groups<kDivCols>(m.C), s->geom));
        else launch_div<R>(da, s->geom, s->stream);
        FEVertexArgs<R> va{m, p.n_layers, rp<R>(w.L1), nullptr, rp<R>(w.Z2)};
        if (s->rec) record(s, Kind::FE_VERTEX, va, nk, false, col_blocks(wave_groups<kVertexCols>(m.V), s->geom));
        else launch_fe_vertex<R>(va, s->geom, s->stream);
    }
    {
        ProfScope ps(s, SSE_PROF_FE_EDGE);
        FEEdgeArgs<R> a{};
        a.m = m;
        a.L = p.n_layers;
        a.X = X;
        a.ubar_add = add;
        a.ubar_sub = sub;
        if constexpr (sizeof(R) == 4) a.ubar_r = rp<R>(w.ubar_r);
        a.h = h;
        a.rho = w.rho;
        a.B = rp<R>(w.B);
        a.Wtop = rp<R>(w.Wt);
        a.Kbot = w.Kbot;
        a.Z = rp<R>(w.Z);
        a.zeta = zeta;
        a.Un = (comb != COMB_NONE || (sum_hp && pa != 0.0)) ? rp<R>(w.U) : nullptr;
        a.ubar_n = w.ubar_n;
        a.comb = comb;
        a.out = out;
        a.G = G;
        a.sum_h = sum_h;
        a.sum_hu = sum_hu;
        a.sum_hp = sum_hp;
        a.psum_a = pa;
        a.psum_b = pb;
        a.Gi = Gi;
        a.Ga = Ga;
        a.Gb = Gb;
        a.interp = interp;
        a.dt = p.dt;
        a.g = p.gravity;
        a.rho0 = p.rho0;
        a.nu_h = p.nu_h;
        a.nu_v = p.nu_v;
        a.c_drag = p.c_drag;
        a.vmix = p.vmix;
        if (del4) {
            a.nu_h = 0.0;
            a.nu4 = p.nu_h;
            a.D2 = rp<R>(w.D2);
            a.Z2 = rp<R>(w.Z2);
        }
        if (s->rec)
            record(s, Kind::FE_EDGE, a, nk, add != nullptr, col_blocks(m.E, edge_geom(s->geom, nk)), -1,
                   fe_edge_variant(m, p.n_layers, p.vmix, del4) | (s->edge_variant == -2 ? 8 : 0));
        else if (s->edge_variant >= 0)
            launch_fe_edge_tiled<R>(a, s->mesh->tiles[s->edge_variant], s->stream);
        else
            launch_fe_edge<R>(a, s->geom, s->stream, s->edge_variant == -2);
    }
}

template <typename Tin, typename Tout>
void convert(sse_state *s, const Tin *src, Tout *dst, size_t n) {
    ProfScope ps(s, SSE_PROF_OTHER);
    ConvArgs<Tin, Tout> a{src, dst, n};
    if (s->rec)
        record(s, std::is_same<Tin, double>::value ? Kind::CONV_DF : Kind::CONV_FD, a, 1, false, flat_blocks(n, s->geom));
    else
        launch_convert<Tin, Tout>(a, s->geom, s->stream);
}

// Stage buffers of one barotropic loop, in the loop's real type: the stages
// (u1, uh, z1, zh) and, for the FP32 loop, its rounded input and its output
// before widening (ua, za, uo, zo).
struct BtBufs {
    void *u1, *uh, *z1, *zh, *ua, *za, *uo, *zo;
};

BtBufs bt_bufs(const Work &w) { return {w.bt_u1, w.bt_uh, w.bt_z1, w.bt_zh, w.bt_ua, w.bt_za, w.bt_uo, w.bt_zo}; }

// Algorithm 3 (scheme 2) / Algorithm 4 (scheme 3): M substeps of dt / M with
// G frozen, accumulating F^zeta in FP64.  The inputs are not modified.  In
// mixed precision the loop state is FP32: the FP64 inputs are rounded once on
// entry and the result widened once on exit.
template <typename R>
void bt_loop(sse_state *s, int scheme, int M, double dt, const double *in_u, const double *in_z, const double *G,
             double *out_u, double *out_z, double *F, const BtBufs &w) {
    const DevMesh &m = s->mesh->d;
    const R *iu;
    const R *iz;
    R *ou;
    R *oz;
    if constexpr (std::is_same<R, double>::value) {
        iu = in_u;
        iz = in_z;
        ou = out_u;
        oz = out_z;
    } else {
        convert<double, R>(s, in_u, rp<R>(w.ua), m.E);
        convert<double, R>(s, in_z, rp<R>(w.za), m.C);
        iu = rp<R>(w.ua);
        iz = rp<R>(w.za);
        ou = rp<R>(w.uo);
        oz = rp<R>(w.zo);
    }
    R *u1 = rp<R>(w.u1), *uh = rp<R>(w.uh), *z1 = rp<R>(w.z1), *zh = rp<R>(w.zh);
    if (s->bt_variant == 2 && !s->rec && !s->capturing && bt_loop_fits(s, scheme)) {
        // one cooperative launch: every patch in its own workgroup for all M
        // substeps, grid barriers between them
        BTTileArgs<R> a{};
        a.t = s->mesh->bt;
        a.G = G;
        a.F = F;
        a.zeroF = 1;
        a.tau = dt / M;
        a.g = s->p.gravity;
        a.w1 = scheme == SSE_SCHEME_SSPRK3 ? 1.0 / (6.0 * M) : 1.0 / (2.0 * M);
        a.w3 = scheme == SSE_SCHEME_SSPRK3 ? 2.0 / (3.0 * M) : 0.0;
        BtLoop<R> l{};
        l.M = M;
        l.u_in = iu;
        l.z_in = iz;
        l.bu0 = u1;
        l.bu1 = uh;
        l.bz0 = z1;
        l.bz1 = zh;
        l.u_out = ou;
        l.z_out = oz;
        l.bar = reinterpret_cast<unsigned *>(s->w.flag + 16);
        l.gen = reinterpret_cast<unsigned *>(s->w.flag + 48);
        l.err = s->w.flag + 32;
        l.spins = s->barrier_spins;
        {
            ProfScope ps(s, SSE_PROF_BT_EVAL);
            const hipError_t e = launch_bt_loop<R>(a, l, scheme, s->stream);
            if (e != hipSuccess) s->launch_error = e;
        }
        if constexpr (!std::is_same<R, double>::value) {
            convert<R, double>(s, ou, out_u, m.E);
            convert<R, double>(s, oz, out_z, m.C);
        }
        return;
    }
    if (s->bt_variant >= 1) {
        // one launch per substep; outputs alternate between the loop's
        // output and a scratch pair so that no launch reads what another
        // workgroup of the same launch writes, ending in the output
        BTTileArgs<R> a{};
        a.t = s->mesh->bt;
        a.G = G;
        a.F = F;
        a.tau = dt / M;
        a.g = s->p.gravity;
        a.w1 = scheme == SSE_SCHEME_SSPRK3 ? 1.0 / (6.0 * M) : 1.0 / (2.0 * M);
        a.w3 = scheme == SSE_SCHEME_SSPRK3 ? 2.0 / (3.0 * M) : 0.0;
        const R *pu = iu, *pz = iz;
        if (s->rec) s->rec->loop_seq = s->rec->seq++;
        for (int sub = 0; sub < M; ++sub) {
            const bool to_out = (M - 1 - sub) % 2 == 0;
            R *tu = to_out ? ou : u1, *tz = to_out ? oz : z1;
            a.ua = pu;
            a.za = pz;
            a.uo = tu;
            a.zo = tz;
            a.zeroF = sub == 0;
            if (s->rec) {
                record(s, Kind::BT_TILE, a, 1, false, a.t.nP, sub, a.t.ks);
                s->rec->entries.back().lds = std::is_same<R, double>::value ? a.t.lds_d : a.t.lds_f;
            } else {
                ProfScope ps(s, SSE_PROF_BT_EVAL);
                launch_bt_substep<R>(a, scheme, s->stream);
            }
            pu = tu;
            pz = tz;
        }
        if constexpr (!std::is_same<R, double>::value) {
            convert<R, double>(s, ou, out_u, m.E);
            convert<R, double>(s, oz, out_z, m.C);
        }
        return;
    }
    if (s->rec) s->rec->loop_seq = s->rec->seq++;
    const int nblk = bt_blocks(m.E, m.C, s->geom);
    BTEvalArgs<R> a{};
    a.m = m;
    a.G = G;
    a.F = F;
    a.tau = dt / M;
    a.g = s->p.gravity;
    int j = 0;
    auto eval = [&]() {
        ProfScope ps(s, SSE_PROF_BT_EVAL);
        if (s->rec) record(s, Kind::BT_EVAL, a, 1, false, nblk, j++, m.delta16);
        else launch_bt_eval<R>(a, s->geom, s->stream);
    };
    for (int sub = 0; sub < M; ++sub) {
        const R *bu = sub == 0 ? iu : ou;
        const R *bz = sub == 0 ? iz : oz;
        if (scheme == SSE_SCHEME_SSPRK3) {
            const double w1 = 1.0 / (6.0 * M), w3 = 2.0 / (3.0 * M);
            a.ua = bu; a.za = bz; a.ub = bu; a.zb = bz; a.uo = u1; a.zo = z1;
            a.wF = w1; a.zeroF = (sub == 0); a.comb = COMB_NONE; eval();
            a.ua = u1; a.za = z1; a.ub = bu; a.zb = bz; a.uo = uh; a.zo = zh;
            a.wF = w1; a.zeroF = 0; a.comb = COMB_34; eval();
            a.ua = uh; a.za = zh; a.ub = bu; a.zb = bz; a.uo = ou; a.zo = oz;
            a.wF = w3; a.zeroF = 0; a.comb = COMB_THIRD; eval();
        } else {
            const double w1 = 1.0 / (2.0 * M);
            a.ua = bu; a.za = bz; a.ub = bu; a.zb = bz; a.uo = u1; a.zo = z1;
            a.wF = w1; a.zeroF = (sub == 0); a.comb = COMB_NONE; eval();
            a.ua = u1; a.za = z1; a.ub = bu; a.zb = bz; a.uo = ou; a.zo = oz;
            a.wF = w1; a.zeroF = 0; a.comb = COMB_HALF; eval();
        }
    }
    if constexpr (!std::is_same<R, double>::value) {
        convert<R, double>(s, ou, out_u, m.E);
        convert<R, double>(s, oz, out_z, m.C);
    }
}

void recon(sse_state *s, int mode, const double *Fz, const double *Fh, const double *Sh, const double *Pp,
           const double *ub_new, const double *ub2, double *ub_half) {
    ProfScope ps(s, SSE_PROF_OTHER);
    Work &w = s->w;
    ReconArgs a{};
    a.m = s->mesh->d;
    a.mode = mode;
    a.rec = s->p.reconcile;
    a.Fz = Fz;
    a.Fh = Fh;
    a.Sh = Sh;
    a.Pp = Pp;
    a.ub_n = w.ubar_n;
    a.ub_new = ub_new;
    a.Fz1 = w.Fz1;
    a.Fz2 = w.Fz2;
    a.Fh1 = w.Fh1;
    a.Fh2 = w.Fh2;
    a.Ftot = w.Ftot;
    a.uA = w.uA;
    a.ub2 = ub2;
    a.ub_half = ub_half;
    if (s->rec) record(s, Kind::RECON, a, 1, false, flat_blocks(a.m.E, s->geom));
    else launch_recon(a, s->geom, s->stream);
}

// Thickness stage.  z-star uses the 2D total flux w.Ftot; isopycnal rebuilds
// the per-layer velocity c1 X1 + c2 X2 + ca1 a1 + u^A.
// Thickness stage, fused with the temperature stage in tracer runs: T_in and
// T_out are the stage's input and output temperature (base T^n when comb is
// set); the density is updated in place.
template <typename R>
void thickness(sse_state *s, const double *h_in, const double *h_n, int comb, double *h_out, double *zeta_out,
               const R *X1, double c1, const R *X2, double c2, const double *a1, double ca1, double dt,
               const double *T_in = nullptr, double *T_out = nullptr) {
    ProfScope ps(s, SSE_PROF_THICKNESS);
    Work &w = s->w;
    const int nk = nk_of(s->p.n_layers), nb = col_blocks(s->mesh->d.C, s->geom);
    if (s->p.tracer) {
        const sse_params &p = s->p;
        TracerArgs<R> a{};
        a.m = s->mesh->d;
        a.L = p.n_layers;
        a.h_in = h_in;
        a.h_n = h_n;
        a.T_in = T_in;
        a.T_n = w.Tn;
        a.X1 = X1;
        a.X2 = X2;
        a.c1 = c1;
        a.c2 = c2;
        a.a1 = a1;
        a.ca1 = ca1;
        a.uA = w.uA;
        a.frac = p.vcoord == SSE_ZSTAR ? w.frac : nullptr;
        a.comb = comb;
        a.dt = dt;
        a.kappa_h = p.kappa_h;
        a.kappa_v = p.kappa_v;
        a.rho0 = p.rho0;
        a.alpha = p.eos_alpha;
        a.tref = p.eos_tref;
        a.h_out = h_out;
        a.zeta_out = zeta_out;
        a.T_out = T_out;
        a.rho_out = w.rho;
        a.nonfinite = w.flag;
        if (s->rec) record(s, Kind::TRACER, a, nk, false, nb);
        else launch_tracer<R>(a, s->geom, s->stream);
        return;
    }
    if (s->p.vcoord == SSE_ZSTAR) {
        THArgs a{s->mesh->d, s->p.n_layers, h_in, h_n, w.frac, w.Ftot, comb, dt, h_out, zeta_out, w.flag};
        if (s->rec) record(s, Kind::THICK, a, nk, false, col_blocks(wave_groups<kThickCols>(s->mesh->d.C), s->geom));
        else launch_thickness(a, s->geom, s->stream);
    } else {
        THIsoArgs<R> a{};
        a.m = s->mesh->d;
        a.L = s->p.n_layers;
        a.h_in = h_in;
        a.h_n = h_n;
        a.X1 = X1;
        a.X2 = X2;
        a.c1 = c1;
        a.c2 = c2;
        a.a1 = a1;
        a.ca1 = ca1;
        a.uA = w.uA;
        a.comb = comb;
        a.dt = dt;
        a.h_out = h_out;
        a.zeta_out = zeta_out;
        a.nonfinite = w.flag;
        if (s->rec) record(s, Kind::THICK_ISO, a, nk, false, nb);
        else launch_thickness_iso<R>(a, s->geom, s->stream);
    }
}

template <typename R>
void assemble(sse_state *s, const R *X, const double *ubar_bt) {
    ProfScope ps(s, SSE_PROF_OTHER);
    Work &w = s->w;
    AssembleArgs<R> a{s->mesh->d, s->p.n_layers, X, ubar_bt, w.Hs, rp<R>(w.U), w.ubar_n, w.flag};
    if (s->rec)
        record(s, Kind::ASSEMBLE, a, nk_of(s->p.n_layers), false, col_blocks(wave_groups<kAssembleCols>(a.m.E), s->geom));
    else launch_assemble<R>(a, s->geom, s->stream);
}

// The step's barotropic loop: FP32 state in SSE_MIXED, FP64 otherwise.
template <typename R>
void bt_loop_of(sse_state *s, int scheme, int M, double dt, const double *in_u, const double *in_z,
                const double *G, double *out_u, double *out_z, double *F) {
    if (s->bt64)
        bt_loop<double>(s, scheme, M, dt, in_u, in_z, G, out_u, out_z, F, bt_bufs(s->w));
    else
        bt_loop<float>(s, scheme, M, dt, in_u, in_z, G, out_u, out_z, F, bt_bufs(s->w));
}

template <typename R>
void step_ssprk3(sse_state *s) {
    Work &w = s->w;
    const int M = s->p.substeps;
    const double dt = s->p.dt;
    R *U = rp<R>(w.U), *T1 = rp<R>(w.T1), *T2 = rp<R>(w.T2);
    const R *none = nullptr;
    // Stage 1: baroclinic FE from (u^n, ut^n, zeta^n, h^n); predictor loop; thickness.
    fe_pass<R>(s, U, nullptr, w.ubar_n, w.Hs, w.zeta_n, COMB_NONE, T1, w.G0, w.Sh1, w.Fh1, nullptr, 0, 0,
               nullptr, nullptr, nullptr, 0);
    bt_loop_of<R>(s, 3, M, dt, w.ubar_n, w.zeta_n, w.G0, w.ub1, w.bt_zout, w.Fz1);
    recon(s, 0, w.Fz1, w.Fh1, w.Sh1, nullptr, nullptr, nullptr, nullptr);
    thickness<R>(s, w.Hs, nullptr, COMB_NONE, w.H1, w.z1, U, 1.0, none, 0.0, nullptr, 0.0, dt, w.Tn, w.T1s);
    // Stage 2: FE from (u-hat^{n+1}, ut-hat^{n+1}, zeta-hat^{n+1}, h-hat^{n+1}); second loop; thickness.
    fe_pass<R>(s, T1, w.ub1, nullptr, w.H1, w.z1, COMB_34, T2, w.G1, w.Sh2, w.Fh2, nullptr, 0, 0, nullptr,
               nullptr, nullptr, 0);
    bt_loop_of<R>(s, 3, M, dt, w.ub1, w.z1, w.G1, w.ub2, w.bt_zout, w.Fz2);
    recon(s, 0, w.Fz2, w.Fh2, w.Sh2, nullptr, nullptr, w.ub2, w.ub_half);
    thickness<R>(s, w.H1, w.Hs, COMB_34, w.H2, w.z_half, T1, 1.0, none, 0.0, w.ub1, 1.0, dt, w.T1s, w.Th);
    // Stage 3: FE from the n+1/2 stage -> ut^{n+1}; G interpolated by Interp_3.
    fe_pass<R>(s, T2, w.ub_half, nullptr, w.H2, w.z_half, COMB_THIRD, T1, w.Gh, w.Sh3, nullptr, w.Pp, 1.0, 1.0,
               w.Gi, w.G0, w.G1, 3);
    // Step 2: corrector loop from (ubar^n, zeta^n).
    bt_loop_of<R>(s, 3, M, dt, w.ubar_n, w.zeta_n, w.Gi, w.ubar_new, w.bt_zout, w.Fz3);
    // Step 3: last thickness stage with u^A_3, then u^{n+1} and its split.
    recon(s, 1, w.Fz3, nullptr, w.Sh3, w.Pp, w.ubar_new, nullptr, nullptr);
    thickness<R>(s, w.H2, w.Hs, COMB_THIRD, w.Hs, w.zeta_n, U, 0.5, T1, 0.5, w.ubar_new, 0.5, dt, w.Th, w.Tn);
    assemble<R>(s, T1, w.ubar_new);
}

template <typename R>
void step_ssprk2(sse_state *s) {
    Work &w = s->w;
    const int M = s->p.substeps;
    const double dt = s->p.dt;
    R *U = rp<R>(w.U), *T1 = rp<R>(w.T1), *T2 = rp<R>(w.T2);
    const R *none = nullptr;
    fe_pass<R>(s, U, nullptr, w.ubar_n, w.Hs, w.zeta_n, COMB_NONE, T1, w.G0, w.Sh1, w.Fh1, nullptr, 0, 0,
               nullptr, nullptr, nullptr, 0);
    bt_loop_of<R>(s, 2, M, dt, w.ubar_n, w.zeta_n, w.G0, w.ub1, w.bt_zout, w.Fz1);
    recon(s, 0, w.Fz1, w.Fh1, w.Sh1, nullptr, nullptr, nullptr, nullptr);
    thickness<R>(s, w.Hs, nullptr, COMB_NONE, w.H1, w.z1, U, 1.0, none, 0.0, nullptr, 0.0, dt, w.Tn, w.T1s);
    fe_pass<R>(s, T1, w.ub1, nullptr, w.H1, w.z1, COMB_HALF, T2, w.G1, w.Sh2, nullptr, w.Pp, 0.0, 1.0, w.Gi,
               w.G0, nullptr, 2);
    bt_loop_of<R>(s, 2, M, dt, w.ubar_n, w.zeta_n, w.Gi, w.ubar_new, w.bt_zout, w.Fz2);
    recon(s, 2, w.Fz2, nullptr, w.Sh2, w.Pp, w.ubar_new, nullptr, nullptr);
    thickness<R>(s, w.H1, w.Hs, COMB_HALF, w.Hs, w.zeta_n, T2, 1.0, none, 0.0, w.ubar_new, 1.0, dt, w.T1s, w.Tn);
    assemble<R>(s, T2, w.ubar_new);
}

template <typename R>
void step_one(sse_state *s) {
    if (s->p.scheme == SSE_SCHEME_SSPRK3)
        step_ssprk3<R>(s);
    else
        step_ssprk2<R>(s);
}

int check_params(const sse_params *p) {
    if (!p) { set_error("params is NULL"); return SSE_EINVAL; }
    if (p->n_layers < 1 || p->n_layers > 2 * kWave) { set_error("n_layers must be in [1, 128]"); return SSE_EINVAL; }
    if (p->scheme != SSE_SCHEME_SSPRK2 && p->scheme != SSE_SCHEME_SSPRK3) { set_error("scheme must be 2 or 3"); return SSE_EINVAL; }
    if (p->substeps < 1) { set_error("substeps must be >= 1"); return SSE_EINVAL; }
    if (p->precision != SSE_FP64 && p->precision != SSE_MIXED && p->precision != SSE_MIXED_BT64) {
        set_error("precision must be SSE_FP64, SSE_MIXED or SSE_MIXED_BT64");
        return SSE_EINVAL;
    }
    if (p->vcoord != SSE_ZSTAR && p->vcoord != SSE_ISOPYCNAL) { set_error("vcoord must be ZSTAR or ISOPYCNAL"); return SSE_EINVAL; }
    if (p->reconcile < SSE_RECONCILE_OFF || p->reconcile > SSE_RECONCILE_LITERAL) { set_error("invalid reconcile mode"); return SSE_EINVAL; }
    if (p->vmix != SSE_VMIX_EXPLICIT && p->vmix != SSE_VMIX_IMPLICIT) { set_error("vmix must be SSE_VMIX_EXPLICIT or SSE_VMIX_IMPLICIT"); return SSE_EINVAL; }
    if (p->hdiff != SSE_HDIFF_DEL2 && p->hdiff != SSE_HDIFF_DEL4) { set_error("hdiff must be SSE_HDIFF_DEL2 or SSE_HDIFF_DEL4"); return SSE_EINVAL; }
    if (p->tracer != SSE_TRACER_NONE && p->tracer != SSE_TRACER_TEMPERATURE) { set_error("tracer must be SSE_TRACER_NONE or SSE_TRACER_TEMPERATURE"); return SSE_EINVAL; }
    if (p->tracer) {
        if (!(p->kappa_h >= 0) || !(p->kappa_v >= 0) || !std::isfinite(p->kappa_h) || !std::isfinite(p->kappa_v) ||
            !std::isfinite(p->eos_alpha) || !std::isfinite(p->eos_tref)) {
            set_error("kappa_h, kappa_v must be >= 0 and the EOS coefficients finite");
            return SSE_EINVAL;
        }
    }
    const double v[] = {p->dt, p->gravity, p->rho0};
    for (double x : v)
        if (!(x > 0) || !std::isfinite(x)) { set_error("dt, gravity and rho0 must be positive"); return SSE_EINVAL; }
    const double nn[] = {p->nu_h, p->nu_v, p->c_drag};
    for (double x : nn)
        if (!(x >= 0) || !std::isfinite(x)) { set_error("nu_h, nu_v and c_drag must be >= 0"); return SSE_EINVAL; }
    return SSE_OK;
}

int read_flag(sse_state *s) {
    int flag[33] = {};
    SSE_HIP(hipMemcpyAsync(flag, s->w.flag, sizeof(flag), hipMemcpyDeviceToHost, s->stream));
    SSE_HIP(hipStreamSynchronize(s->stream));
    if (s->prof) prof_flush(s);
    if (flag[32]) {
        set_error("a grid barrier of the persistent barotropic loop timed out; the state is not valid");
        return SSE_EDEVICE;
    }
    if (flag[0]) { set_error("non-finite value in the state (the step blew up)"); return SSE_ENONFINITE; }
    return SSE_OK;
}

// A cooperative launch that failed while steps were enqueued.
int take_launch_error(sse_state *s) {
    const hipError_t e = s->launch_error;
    s->launch_error = hipSuccess;
    return e == hipSuccess ? SSE_OK : hip_fail(e, "hipLaunchCooperativeKernel");
}

// Host <-> device copies of an array of the state's real type from / to FP64
// host memory (the conversion is done on the host).
int upload_real(sse_state *s, void *dst, const double *src, size_t n) {
    if (s->rs == sizeof(double)) {
        SSE_HIP(hipMemcpyAsync(dst, src, n * 8, hipMemcpyHostToDevice, s->stream));
        return SSE_OK;
    }
    std::vector<float> tmp(src, src + n);
    SSE_HIP(hipMemcpyAsync(dst, tmp.data(), n * 4, hipMemcpyHostToDevice, s->stream));
    SSE_HIP(hipStreamSynchronize(s->stream));  // tmp dies at return
    return SSE_OK;
}

int download_real(const sse_state *s, double *dst, const void *src, size_t n) {
    if (s->rs == sizeof(double)) {
        SSE_HIP(hipMemcpyAsync(dst, src, n * 8, hipMemcpyDeviceToHost, s->stream));
        return SSE_OK;
    }
    std::vector<float> tmp(n);
    SSE_HIP(hipMemcpyAsync(tmp.data(), src, n * 4, hipMemcpyDeviceToHost, s->stream));
    SSE_HIP(hipStreamSynchronize(s->stream));
    std::copy(tmp.begin(), tmp.end(), dst);
    return SSE_OK;
}

#define SSE_TRY(call)               \
    do {                            \
        int _rc = (call);           \
        if (_rc != SSE_OK) return _rc; \
    } while (0)

}  // namespace

// ===========================================================================
// Mesh
// ===========================================================================
extern "C" int sse_mesh_create(const sse_mesh_desc *d, void *dev_buf, size_t bytes, void *stream, sse_mesh **out) {
    if (!out) { set_error("out is NULL"); return SSE_EINVAL; }
    *out = nullptr;
    std::string err;
    int rc = validate_desc(d, err);
    if (rc != SSE_OK) { set_error(err); return rc; }
    // Renumber for locality: cells in compact patches, edges and vertices
    // after their cells.  Every table below is built in the new numbering;
    // the host-side state I/O translates at the boundary.
    // The caller's numbering is kept when it is already at least as local
    // (share of edges whose two cells lie within kLocalSpan indices).
    const sse_mesh_desc *d0 = d;  // the caller's numbering
    MeshOrder ord;
    locality_order(d, kPatchCells, ord);
    if (local_share(d, nullptr) >= local_share(d, &ord)) identity_order(d, ord);
    PermutedDesc pd;
    permute_desc(d, ord, pd);
    // Reconstruction stencils in canonical two-cell order when the mesh
    // allows it (the edge pass then gathers 10 vertex columns, not 20).
    std::vector<int32_t> chain;
    const bool canonical = canonical_stencils(pd, chain);
    d = &pd.d;
    MeshLayout lay = mesh_layout(d->n_cells, d->n_edges, d->n_vertices);
    size_t need = lay.total;
    for (int q = 0; q < kTileVariants; ++q) need += tiles_bytes(d, kTileSizes[q]);
    need += bt_tiles_bytes(d0);
    need += wpair_f_bytes(d);
    if (!dev_buf || bytes < need) { set_error("mesh device buffer too small"); return SSE_ENOMEM; }
    if (reinterpret_cast<uintptr_t>(dev_buf) % kAlign) { set_error("mesh device buffer must be 256-byte aligned"); return SSE_EINVAL; }
    HostMeshTables t;
    if (canonical) t.chain.swap(chain);
    build_tables(d, t);
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *base = static_cast<char *>(dev_buf);
    const void *src[] = {t.cell_edges.data(), t.cell_nbrs.data(), t.cell_nedges.data(), t.cell_div.data(),
                         t.cell_ke.data(), t.cell_edges_t.data(), t.cell_nbrs_t.data(), t.cell_div_t.data(),
                         t.H.data(), t.cmask.data(), t.edge_cells.data(), t.edge_verts.data(), t.eoe.data(),
                         t.neoe.data(), t.w.data(), t.wf.data(), t.dc.data(), t.dv.data(), t.emask.data(),
                         t.vert_edges.data(), t.vert_curl.data(), t.erec.data(), t.inv_dc.data(),
                         t.inv_dv.data(), t.wpair.data(), t.wf_f.data(), t.inv_dc_f.data(),
                         t.cell_div_t_f.data(), t.H_f.data(), t.eoe16.data(), t.ecells16.data(),
                         t.cedges16.data(), t.cnbrs16.data(), ord.cell_old.data(), ord.edge_old.data()};
    static_assert(sizeof(src) / sizeof(src[0]) == kMeshTables, "one source per mesh table");
    size_t nb[kMeshTables];
    mesh_table_sizes(d->n_cells, d->n_edges, d->n_vertices, nb);
    for (int i = 0; i < kMeshTables; ++i)
        SSE_HIP(hipMemcpyAsync(base + lay.off[i], src[i], nb[i], hipMemcpyHostToDevice, s));
    SSE_HIP(hipStreamSynchronize(s));
    sse_mesh *m = new sse_mesh();
    m->C = d->n_cells;
    m->E = d->n_edges;
    m->V = d->n_vertices;
    m->n_ocean_cells = t.n_ocean_cells;
    m->dev_buf = dev_buf;
    m->dev_bytes = bytes;
    DevMesh &dm = m->d;
    dm.C = m->C;
    dm.E = m->E;
    dm.V = m->V;
    auto P = [&](int i) { return static_cast<void *>(base + lay.off[i]); };
    dm.cell_edges = (const int32_t *)P(0);
    dm.cell_nbrs = (const int32_t *)P(1);
    dm.cell_nedges = (const int32_t *)P(2);
    dm.cell_div = (const double *)P(3);
    dm.cell_ke = (const double *)P(4);
    dm.cell_edges_t = (const int32_t *)P(5);
    dm.cell_nbrs_t = (const int32_t *)P(6);
    dm.cell_div_t = (const double *)P(7);
    dm.H = (const double *)P(8);
    dm.cmask = (const uint8_t *)P(9);
    dm.edge_cells = (const int32_t *)P(10);
    dm.edge_verts = (const int32_t *)P(11);
    dm.eoe = (const int32_t *)P(12);
    dm.neoe = (const int32_t *)P(13);
    dm.w = (const double *)P(14);
    dm.wf = (const double *)P(15);
    dm.dc = (const double *)P(16);
    dm.dv = (const double *)P(17);
    dm.emask = (const uint8_t *)P(18);
    dm.vert_edges = (const int32_t *)P(19);
    dm.vert_curl = (const double *)P(20);
    dm.erec = (const int32_t *)P(21);
    dm.inv_dc = (const double *)P(22);
    dm.inv_dv = (const double *)P(23);
    dm.wpair = (const double *)P(24);
    dm.chain = t.chain.empty() ? 0 : 1;
    dm.wf_f = (const float *)P(25);
    dm.inv_dc_f = (const float *)P(26);
    dm.cell_div_t_f = (const float *)P(27);
    dm.H_f = (const float *)P(28);
    dm.eoe16 = (const int16_t *)P(29);
    dm.ecells16 = (const int32_t *)P(30);
    dm.cedges16 = (const int16_t *)P(31);
    dm.cnbrs16 = (const int16_t *)P(32);
    dm.cell_old = (const int32_t *)P(33);
    dm.edge_old = (const int32_t *)P(34);
    dm.delta16 = t.delta16;
    dm.ratio_ce = t.ratio_ce;
    dm.ratio_ec = t.ratio_ec;
    m->cells_on_edge = t.edge_cells;
    m->cell_old = ord.cell_old;
    m->edge_old = ord.edge_old;
    // Gather lists of the LDS-staged edge pass for tiles of 8, 16 and 32
    // edges: space is reserved here, the lists are built when a state first
    // selects the variant (most runs never do).
    size_t cursor = lay.total;
    for (int q = 0; q < kTileVariants; ++q) {
        m->tile_off[q] = cursor;
        m->tile_state[q] = 0;
        m->tiles[q].T = 0;
        cursor += tiles_bytes(d, kTileSizes[q]);
    }
    // Patches of the tiled barotropic substeps (partitioned in the caller's
    // numbering, the same partition the device-bytes query sizes).
    {
        std::vector<int32_t> pid0, pid;
        int nP = 0;
        HostBtTiles hb;
        if (bt_cached_partition(d0, pid0, nP)) {
            pid.resize(d->n_cells);
            for (int i = 0; i < d->n_cells; ++i) pid[i] = pid0[ord.cell_old[i]];
            if (build_bt_tiles(d, pid, nP, &t, hb)) {
                hipError_t put_err = hipSuccess;
                auto put = [&](const void *src, size_t n) -> const void * {
                    char *dst = base + cursor;
                    if (n && put_err == hipSuccess) put_err = hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, s);
                    cursor += (n + kAlign - 1) / kAlign * kAlign;
                    return dst;
                };
                DevBtTiles &b = m->bt;
                b.patch = (const int32_t *)put(hb.patch.data(), hb.patch.size() * 4);
                b.eid = (const int32_t *)put(hb.eid.data(), hb.eid.size() * 4);
                b.cid = (const int32_t *)put(hb.cid.data(), hb.cid.size() * 4);
                b.cH = (const double *)put(hb.cH.data(), hb.cH.size() * 8);
                b.cH_f = (const float *)put(hb.cH_f.data(), hb.cH_f.size() * 4);
                b.ec = (const uint32_t *)put(hb.ec.data(), hb.ec.size() * 4);
                b.enb = (const uint32_t *)put(hb.enb.data(), hb.enb.size() * 4);
                b.ew = (const double *)put(hb.ew.data(), hb.ew.size() * 8);
                b.ew_f = (const float *)put(hb.ew_f.data(), hb.ew_f.size() * 4);
                b.eidc = (const double *)put(hb.eidc.data(), hb.eidc.size() * 8);
                b.eidc_f = (const float *)put(hb.eidc_f.data(), hb.eidc_f.size() * 4);
                b.cen = (const uint32_t *)put(hb.cen.data(), hb.cen.size() * 4);
                b.ccd = (const double *)put(hb.ccd.data(), hb.ccd.size() * 8);
                b.ccd_f = (const float *)put(hb.ccd_f.data(), hb.ccd_f.size() * 4);
                b.cwet = (const uint8_t *)put(hb.cwet.data(), hb.cwet.size());
                SSE_HIP(put_err);
                SSE_HIP(hipStreamSynchronize(s));
                b.nP = hb.nP;
                b.dry = std::any_of(t.emask.begin(), t.emask.end(), [](uint8_t x) { return x == 0; }) ? 1 : 0;
                b.ks = hb.ks;
                b.lds_d = hb.lds_d;
                b.lds_f = hb.lds_f;
            }
        }
    }
    // FP32 weight pairs of the edge pass in mixed precision, last in the image
    if (cursor + wpair_f_bytes(d) > need) {
        delete m;
        set_error("internal: tile tables overflow the mesh buffer");
        return SSE_EINVAL;
    }
    SSE_HIP(hipMemcpyAsync(base + cursor, t.wpair_f.data(), t.wpair_f.size() * 4, hipMemcpyHostToDevice, s));
    SSE_HIP(hipStreamSynchronize(s));
    dm.wpair_f = reinterpret_cast<const float *>(base + cursor);
    cursor += wpair_f_bytes(d);
    m->host_desc.reset(new PermutedDesc(std::move(pd)));
    *out = m;
    return SSE_OK;
}

namespace {

// Builds and uploads the gather lists of edge-pass variant q on first use.
int ensure_tiles(const sse_mesh *cm, int q, hipStream_t s) {
    sse_mesh *m = const_cast<sse_mesh *>(cm);
    std::lock_guard<std::mutex> g(m->tile_mu);
    if (m->tile_state[q] != 0) return SSE_OK;
    HostTiles ht;
    const sse_mesh_desc *d = &m->host_desc->d;
    if (!build_tiles(d, kTileSizes[q], ht)) {
        m->tile_state[q] = -1;
        return SSE_OK;
    }
    char *base = static_cast<char *>(m->dev_buf);
    size_t cursor = m->tile_off[q];
    auto put = [&](const void *src, size_t n) -> const void * {
        char *dst = base + cursor;
        if (n) (void)hipMemcpyAsync(dst, src, n, hipMemcpyHostToDevice, s);
        cursor += (n + kAlign - 1) / kAlign * kAlign;
        return dst;
    };
    DevTiles &dt = m->tiles[q];
    dt.nT = ht.nT;
    dt.max_ue = ht.max_ue;
    dt.max_uv = ht.max_uv;
    dt.max_uc = ht.max_uc;
    dt.ue_off = (const int32_t *)put(ht.ue_off.data(), ht.ue_off.size() * 4);
    dt.uv_off = (const int32_t *)put(ht.uv_off.data(), ht.uv_off.size() * 4);
    dt.uc_off = (const int32_t *)put(ht.uc_off.data(), ht.uc_off.size() * 4);
    dt.ue = (const int32_t *)put(ht.ue.data(), ht.ue.size() * 4);
    dt.uv = (const int32_t *)put(ht.uv.data(), ht.uv.size() * 4);
    dt.uc = (const int32_t *)put(ht.uc.data(), ht.uc.size() * 4);
    dt.loc = (const uint8_t *)put(ht.loc.data(), ht.loc.size());
    SSE_HIP(hipStreamSynchronize(s));
    if (cursor > m->tile_off[q] + tiles_bytes(d, kTileSizes[q])) {
        set_error("internal: tile lists overflow their reserved space");
        m->tile_state[q] = -1;
        return SSE_EINVAL;
    }
    dt.T = ht.T;
    m->tile_state[q] = 1;
    return SSE_OK;
}

}  // namespace

extern "C" int sse_mesh_destroy(sse_mesh *m) {
    delete m;
    return SSE_OK;
}

// ===========================================================================
// State
// ===========================================================================
extern "C" int sse_state_workspace_bytes(const sse_mesh *m, const sse_params *p, size_t *bytes) {
    if (!m || !bytes) { set_error("NULL argument"); return SSE_EINVAL; }
    int rc = check_params(p);
    if (rc) return rc;
    *bytes = workspace_bytes(m->C, m->E, m->V, p->n_layers, real_size(p->precision), bt_size(p->precision), p->hdiff,
                             p->tracer);
    return SSE_OK;
}

extern "C" int sse_footprint_bytes(const sse_mesh_desc *d, const sse_params *p, size_t *bytes) {
    if (!d || !bytes) { set_error("NULL argument"); return SSE_EINVAL; }
    int rc = check_params(p);
    if (rc) return rc;
    std::string err;
    rc = check_topology(d, err);
    if (rc != SSE_OK) { set_error(err); return rc; }
    size_t mb = mesh_layout(d->n_cells, d->n_edges, d->n_vertices).total;
    for (int q = 0; q < kTileVariants; ++q) mb += tiles_bytes(d, kTileSizes[q]);
    mb += bt_tiles_bytes(d);
    mb += wpair_f_bytes(d);
    *bytes = mb + workspace_bytes(d->n_cells, d->n_edges, d->n_vertices, p->n_layers, real_size(p->precision),
                                  bt_size(p->precision), p->hdiff, p->tracer);
    return SSE_OK;
}

extern "C" int sse_state_create(const sse_mesh *m, const sse_params *p, void *dev_workspace, size_t bytes,
                                void *stream, sse_state **out) {
    if (!m || !out) { set_error("NULL argument"); return SSE_EINVAL; }
    *out = nullptr;
    int rc = check_params(p);
    if (rc) return rc;
    const size_t rs = real_size(p->precision), bs = bt_size(p->precision);
    size_t need = workspace_bytes(m->C, m->E, m->V, p->n_layers, rs, bs, p->hdiff, p->tracer);
    if (!dev_workspace || bytes < need) { set_error("state workspace too small"); return SSE_ENOMEM; }
    if (reinterpret_cast<uintptr_t>(dev_workspace) % kAlign) { set_error("state workspace must be 256-byte aligned"); return SSE_EINVAL; }
    sse_state *s = new sse_state();
    s->mesh = m;
    s->p = *p;
    s->stream = static_cast<hipStream_t>(stream);
    s->rs = rs;
    s->bt64 = bs == sizeof(double);
    s->w = carve(dev_workspace, m->C, m->E, m->V, p->n_layers, rs, bs, p->hdiff, p->tracer);
    s->bytes = bytes;
    int dev = 0, lds_max = 0;
    (void)hipGetDevice(&dev);
    s->device = dev;
    (void)scratch_address(dev);  // set-up of the allocation-free entry point on this device
    if (hipDeviceGetAttribute(&lds_max, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess) lds_max = 65536;
    set_tiled_lds_limit((size_t)lds_max);
    s->lds_max = (size_t)lds_max;
    s->edge_variant = -1;
    s->bt_variant = bt_tiles_fit(s) ? 1 : 0;
    for (int q = 0; q < 2; ++q)
        s->bt_capacity[q] = !bt_tiles_fit(s) ? 0
                            : s->bt64 ? bt_loop_capacity<double>(s->mesh->bt, 2 + q)
                                      : bt_loop_capacity<float>(s->mesh->bt, 2 + q);
    *out = s;
    return SSE_OK;
}

extern "C" int sse_state_set_bt_variant(sse_state *s, int variant) {
    if (!s) { set_error("NULL state"); return SSE_EINVAL; }
    if (variant < 0 || variant > 2) { set_error("barotropic variant must be 0, 1 or 2"); return SSE_EINVAL; }
    if (variant >= 1 && !bt_tiles_fit(s)) {
        set_error("barotropic variants 1 and 2: the mesh has no patches that fit a workgroup");
        return SSE_EINVAL;
    }
    if (variant == 2 && !bt_loop_fits(s, s->p.scheme)) {
        set_error("barotropic variant 2: the device cannot hold a workgroup for every patch at once");
        return SSE_EINVAL;
    }
    s->bt_variant = variant;
    if (s->graph_exec) (void)hipGraphExecDestroy(s->graph_exec);
    s->graph_exec = nullptr;
    return SSE_OK;
}

extern "C" int sse_debug_set_barrier_spins(sse_state *s, uint32_t spins) {
    if (!s) { set_error("NULL state"); return SSE_EINVAL; }
    s->barrier_spins = spins ? spins - 1 : kBarrierSpins;  // the kernel gives up once it has slept this often
    return SSE_OK;
}

extern "C" int sse_state_get_bt_variant(const sse_state *s, int *variant) {
    if (!s || !variant) { set_error("NULL argument"); return SSE_EINVAL; }
    *variant = s->bt_variant;
    return SSE_OK;
}

extern "C" int sse_state_set_edge_variant(sse_state *s, int variant) {
    if (!s) { set_error("NULL state"); return SSE_EINVAL; }
    if (variant == -1 || variant == -2) {
        s->edge_variant = variant;
        if (s->graph_exec) (void)hipGraphExecDestroy(s->graph_exec);
        s->graph_exec = nullptr;
        return SSE_OK;
    }
    if (variant < 0 || variant >= kTileVariants) { set_error("edge variant must be -2, -1, 0, 1 or 2"); return SSE_EINVAL; }
    if (s->p.hdiff == SSE_HDIFF_DEL4) {
        set_error("edge variants 0, 1, 2 do not carry the biharmonic viscosity; use -1");
        return SSE_EINVAL;
    }
    const int rc = ensure_tiles(s->mesh, variant, s->stream);
    if (rc) return rc;
    const DevTiles &t = s->mesh->tiles[variant];
    if (!t.T) { set_error("edge variant: a tile of this mesh lists more than 255 columns"); return SSE_EINVAL; }
    const size_t lds = s->rs == 4 ? fe_edge_tiled_lds<float>(t, s->p.n_layers) : fe_edge_tiled_lds<double>(t, s->p.n_layers);
    if (lds > s->lds_max) { set_error("edge variant: the tile does not fit the device's LDS"); return SSE_EINVAL; }
    s->edge_variant = variant;
    if (s->graph_exec) (void)hipGraphExecDestroy(s->graph_exec);
    s->graph_exec = nullptr;
    return SSE_OK;
}

extern "C" int sse_state_get_edge_variant(const sse_state *s, int *variant) {
    if (!s || !variant) { set_error("NULL argument"); return SSE_EINVAL; }
    *variant = s->edge_variant;
    return SSE_OK;
}

extern "C" int sse_state_destroy(sse_state *s) {
    if (!s) return SSE_OK;
    if (s->batch) (void)sse_batch_remove(s->batch, s);
    if (s->graph_exec) (void)hipGraphExecDestroy(s->graph_exec);
    for (auto e : s->events) (void)hipEventDestroy(e);
    delete s;
    return SSE_OK;
}

extern "C" int sse_state_init(sse_state *s, const double *h, const double *u, const double *rho, const double *h_ref) {
    if (!s || !h || !u || !rho) { set_error("NULL argument"); return SSE_EINVAL; }
    const sse_mesh *m = s->mesh;
    const int L = s->p.n_layers;
    const size_t CL = (size_t)m->C * L, EL = (size_t)m->E * L;
    if (s->p.vcoord == SSE_ZSTAR && !h_ref) { set_error("z-star needs h_ref"); return SSE_EINVAL; }
    if (!all_finite(h, CL) || !all_finite(u, EL) || !all_finite(rho, CL) || (h_ref && !all_finite(h_ref, CL))) {
        set_error("non-finite value in the initial state");
        return SSE_ENONFINITE;
    }
    // caller numbering -> internal numbering
    std::vector<double> hi(CL), ri(CL), hri, um(EL), frac(CL, 0.0);
    rows_to_internal(h, hi.data(), m->cell_old, L);
    rows_to_internal(rho, ri.data(), m->cell_old, L);
    rows_to_internal(u, um.data(), m->edge_old, L);
    if (h_ref) {
        hri.resize(CL);
        rows_to_internal(h_ref, hri.data(), m->cell_old, L);
    }
    std::vector<uint8_t> cmask(m->C);
    SSE_HIP(hipMemcpy(cmask.data(), m->d.cmask, m->C, hipMemcpyDeviceToHost));
    for (int e = 0; e < m->E; ++e) {
        const bool wet = cmask[m->cells_on_edge[2 * e]] && cmask[m->cells_on_edge[2 * e + 1]];
        if (!wet) std::fill(um.begin() + (size_t)e * L, um.begin() + (size_t)(e + 1) * L, 0.0);
    }
    if (h_ref) {
        for (int i = 0; i < m->C; ++i) {
            if (!cmask[i]) continue;
            double tot = 0.0;
            for (int k = 0; k < L; ++k) tot += hri[(size_t)i * L + k];
            if (!(tot > 0)) { set_error("h_ref must have a positive column sum on ocean cells"); return SSE_EINVAL; }
            for (int k = 0; k < L; ++k) frac[(size_t)i * L + k] = hri[(size_t)i * L + k] / tot;
        }
    }
    Work &w = s->w;
    SSE_HIP(hipMemcpyAsync(w.Hs, hi.data(), CL * 8, hipMemcpyHostToDevice, s->stream));
    SSE_TRY(upload_real(s, w.U, um.data(), EL));
    SSE_HIP(hipMemcpyAsync(w.rho, ri.data(), CL * 8, hipMemcpyHostToDevice, s->stream));
    SSE_HIP(hipMemcpyAsync(w.frac, frac.data(), CL * 8, hipMemcpyHostToDevice, s->stream));
    SSE_HIP(hipMemsetAsync(w.flag, 0, kAlign, s->stream));
    launch_zeta_from_h(m->d, L, w.Hs, w.zeta_n, s->stream);
    if (s->rs == 4) {
        AssembleArgs<float> a{m->d, L, rp<float>(w.U), nullptr, w.Hs, rp<float>(w.U), w.ubar_n, w.flag};
        launch_assemble<float>(a, s->geom, s->stream);
    } else {
        AssembleArgs<double> a{m->d, L, rp<double>(w.U), nullptr, w.Hs, rp<double>(w.U), w.ubar_n, w.flag};
        launch_assemble<double>(a, s->geom, s->stream);
    }
    SSE_HIP(hipGetLastError());
    SSE_HIP(hipStreamSynchronize(s->stream));
    s->initialized = true;
    return SSE_OK;
}

namespace {

void drop_graph(sse_state *s) {
    if (s->graph_exec) (void)hipGraphExecDestroy(s->graph_exec);
    s->graph_exec = nullptr;
}

void enqueue_step(sse_state *s) {
    if (s->rs == 4)
        step_one<float>(s);
    else
        step_one<double>(s);
}

// Capture one step of launches on `stream` into an executable graph.
template <typename F>
int capture(hipStream_t stream, F &&enqueue, hipGraphExec_t *out) {
    if (!stream) { set_error("HIP graphs need a non-default stream"); return SSE_EINVAL; }
    SSE_HIP(hipStreamBeginCapture(stream, hipStreamCaptureModeThreadLocal));
    enqueue();
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(stream, &graph);
    if (e != hipSuccess) return hip_fail(e, "hipStreamEndCapture");
    const hipError_t e2 = hipGraphInstantiate(out, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e2 != hipSuccess) return hip_fail(e2, "hipGraphInstantiate");
    return SSE_OK;
}

void batch_invalidate(sse_batch *b);

}  // namespace

extern "C" int sse_state_set_tracer(sse_state *s, const double *T) {
    if (!s || !T) { set_error("NULL argument"); return SSE_EINVAL; }
    if (!s->p.tracer) { set_error("the state's parameters carry no tracer"); return SSE_EINVAL; }
    if (!s->initialized) { set_error("state not initialised"); return SSE_ESTATE; }
    const sse_mesh *m = s->mesh;
    const int L = s->p.n_layers;
    const size_t CL = (size_t)m->C * L;
    if (!all_finite(T, CL)) { set_error("non-finite temperature"); return SSE_ENONFINITE; }
    std::vector<double> ti(CL), ri(CL);
    rows_to_internal(T, ti.data(), m->cell_old, L);
    std::vector<uint8_t> cmask(m->C);
    SSE_HIP(hipMemcpy(cmask.data(), m->d.cmask, m->C, hipMemcpyDeviceToHost));
    for (int i = 0; i < m->C; ++i)
        for (int k = 0; k < L; ++k) {
            double &t = ti[(size_t)i * L + k];
            if (!cmask[i]) t = 0.0;
            ri[(size_t)i * L + k] = s->p.rho0 * (1.0 - s->p.eos_alpha * (t - s->p.eos_tref));
        }
    SSE_HIP(hipMemcpyAsync(s->w.Tn, ti.data(), CL * 8, hipMemcpyHostToDevice, s->stream));
    SSE_HIP(hipMemcpyAsync(s->w.rho, ri.data(), CL * 8, hipMemcpyHostToDevice, s->stream));
    SSE_HIP(hipStreamSynchronize(s->stream));
    s->tracer_set = true;
    if (s->batch) batch_invalidate(s->batch);
    return SSE_OK;
}

extern "C" int sse_read_tracer(const sse_state *s, double *T) {
    if (!s || !T) { set_error("NULL argument"); return SSE_EINVAL; }
    if (!s->p.tracer || !s->tracer_set) { set_error("the state carries no temperature"); return SSE_ESTATE; }
    const sse_mesh *m = s->mesh;
    const size_t L = s->p.n_layers;
    std::vector<double> ti((size_t)m->C * L);
    SSE_HIP(hipMemcpyAsync(ti.data(), s->w.Tn, ti.size() * 8, hipMemcpyDeviceToHost, s->stream));
    SSE_HIP(hipStreamSynchronize(s->stream));
    rows_to_user(ti.data(), T, m->cell_old, L);
    return SSE_OK;
}

extern "C" int sse_step_async(sse_state *s, int32_t n) {
    if (!s) { set_error("NULL state"); return SSE_EINVAL; }
    if (!s->initialized) { set_error("state not initialised"); return SSE_ESTATE; }
    if (s->p.tracer && !s->tracer_set) { set_error("tracer runs need sse_state_set_tracer before stepping"); return SSE_ESTATE; }
    if (n < 0) { set_error("n must be >= 0"); return SSE_EINVAL; }
    if (s->use_graph) {
        if (!s->graph_exec) {
            // the captured step uses the per-substep barotropic kernel: the
            // persistent one is a cooperative launch
            s->capturing = true;
            int rc = capture(s->stream, [&] { enqueue_step(s); }, &s->graph_exec);
            s->capturing = false;
            if (rc) return rc;
        }
        for (int i = 0; i < n; ++i) SSE_HIP(hipGraphLaunch(s->graph_exec, s->stream));
        return SSE_OK;
    }
    if (s->prof && s->events.empty()) {
        s->events.resize(8192);
        for (auto &e : s->events) SSE_HIP(hipEventCreate(&e));
    }
    for (int i = 0; i < n; ++i) enqueue_step(s);
    if (int rc = take_launch_error(s)) return rc;
    SSE_HIP(hipGetLastError());
    return SSE_OK;
}

extern "C" int sse_state_set_geometry(sse_state *s, int cols_per_block, int block_2d) {
    if (!s) { set_error("NULL state"); return SSE_EINVAL; }
    Geom g{cols_per_block, block_2d};
    if (!geom_valid(g)) { set_error("geometry: cols_per_block in {1,2,4,8,16}, block_2d a multiple of 64 in [64, 1024]"); return SSE_EINVAL; }
    s->geom = g;
    drop_graph(s);
    return SSE_OK;
}

extern "C" int sse_state_use_graph(sse_state *s, int enable) {
    if (!s) { set_error("NULL state"); return SSE_EINVAL; }
    if (enable && !s->stream) { set_error("HIP graphs need a non-default stream"); return SSE_EINVAL; }
    s->use_graph = enable != 0;
    drop_graph(s);
    return SSE_OK;
}

extern "C" int sse_sync(sse_state *s) {
    if (!s) { set_error("NULL state"); return SSE_EINVAL; }
    return read_flag(s);
}

extern "C" int sse_step(sse_state *s, int32_t n) {
    int rc = sse_step_async(s, n);
    if (rc) return rc;
    return sse_sync(s);
}

extern "C" int sse_read_state(const sse_state *cs, double *h, double *u, double *zeta, double *ubar) {
    if (!cs) { set_error("NULL state"); return SSE_EINVAL; }
    if (!cs->initialized) { set_error("state not initialised"); return SSE_ESTATE; }
    const sse_mesh *m = cs->mesh;
    const size_t L = cs->p.n_layers;
    const Work &w = cs->w;
    hipStream_t st = cs->stream;
    std::vector<double> hi(h ? m->C * L : 0), ui(u ? m->E * L : 0), zi(zeta ? m->C : 0), bi(ubar ? m->E : 0);
    if (h) SSE_HIP(hipMemcpyAsync(hi.data(), w.Hs, hi.size() * 8, hipMemcpyDeviceToHost, st));
    if (u) SSE_TRY(download_real(cs, ui.data(), w.U, ui.size()));
    if (zeta) SSE_HIP(hipMemcpyAsync(zi.data(), w.zeta_n, zi.size() * 8, hipMemcpyDeviceToHost, st));
    if (ubar) SSE_HIP(hipMemcpyAsync(bi.data(), w.ubar_n, bi.size() * 8, hipMemcpyDeviceToHost, st));
    SSE_HIP(hipStreamSynchronize(st));
    if (h) rows_to_user(hi.data(), h, m->cell_old, L);
    if (u) rows_to_user(ui.data(), u, m->edge_old, L);
    if (zeta) rows_to_user(zi.data(), zeta, m->cell_old, 1);
    if (ubar) rows_to_user(bi.data(), ubar, m->edge_old, 1);
    return SSE_OK;
}

extern "C" int sse_profile_enable(sse_state *s, int class_mask) {
    if (!s) { set_error("NULL state"); return SSE_EINVAL; }
    prof_flush(s);
    s->prof_mask = class_mask & ((1 << SSE_PROF_NCLASS) - 1);
    s->prof = s->prof_mask != 0;
    return SSE_OK;
}

extern "C" int sse_profile_read(sse_state *s, int32_t *launches, double *milliseconds) {
    if (!s) { set_error("NULL state"); return SSE_EINVAL; }
    prof_flush(s);
    for (int c = 0; c < SSE_PROF_NCLASS; ++c) {
        if (launches) launches[c] = (int32_t)s->nlaunch[c];
        if (milliseconds) milliseconds[c] = s->ms[c];
        s->nlaunch[c] = 0;
        s->ms[c] = 0.0;
    }
    return SSE_OK;
}

// ===========================================================================
// Debug entry points
// ===========================================================================
extern "C" int sse_debug_baroclinic_feuler(sse_state *s, const double *u, const double *ubar, const double *zeta,
                                           const double *h, double dt, double *ut1, double *G) {
    if (!s || !u || !ubar || !zeta || !h || !ut1 || !G) { set_error("NULL argument"); return SSE_EINVAL; }
    if (!s->initialized) { set_error("state not initialised (rho and h_ref are needed)"); return SSE_ESTATE; }
    const sse_mesh *m = s->mesh;
    const size_t L = s->p.n_layers, C = m->C, E = m->E;
    Work &w = s->w;
    hipStream_t st = s->stream;
    std::vector<double> ui(E * L), bi(E), zi(C), hi(C * L), oi(E * L), gi(E);
    rows_to_internal(u, ui.data(), m->edge_old, L);
    rows_to_internal(ubar, bi.data(), m->edge_old, 1);
    rows_to_internal(zeta, zi.data(), m->cell_old, 1);
    rows_to_internal(h, hi.data(), m->cell_old, L);
    SSE_TRY(upload_real(s, w.T2, ui.data(), E * L));
    SSE_HIP(hipMemcpyAsync(w.ub2, bi.data(), E * 8, hipMemcpyHostToDevice, st));
    SSE_HIP(hipMemcpyAsync(w.z1, zi.data(), C * 8, hipMemcpyHostToDevice, st));
    SSE_HIP(hipMemcpyAsync(w.H1, hi.data(), C * L * 8, hipMemcpyHostToDevice, st));
    const double saved = s->p.dt;
    s->p.dt = dt;
    if (s->rs == 4)
        fe_pass<float>(s, rp<float>(w.T2), nullptr, w.ub2, w.H1, w.z1, COMB_NONE, rp<float>(w.T1), w.G0, w.Sh1,
                       nullptr, nullptr, 0, 0, nullptr, nullptr, nullptr, 0);
    else
        fe_pass<double>(s, rp<double>(w.T2), nullptr, w.ub2, w.H1, w.z1, COMB_NONE, rp<double>(w.T1), w.G0,
                        w.Sh1, nullptr, nullptr, 0, 0, nullptr, nullptr, nullptr, 0);
    s->p.dt = saved;
    SSE_HIP(hipGetLastError());
    SSE_TRY(download_real(s, oi.data(), w.T1, E * L));
    SSE_HIP(hipMemcpyAsync(gi.data(), w.G0, E * 8, hipMemcpyDeviceToHost, st));
    SSE_HIP(hipStreamSynchronize(st));
    rows_to_user(oi.data(), ut1, m->edge_old, L);
    rows_to_user(gi.data(), G, m->edge_old, 1);
    return SSE_OK;
}

extern "C" int sse_debug_edge_gathers(sse_state *s) {
    if (!s) { set_error("NULL state"); return SSE_EINVAL; }
    if (s->rec) { set_error("state is being recorded into a batch"); return SSE_ESTATE; }
    if (!s->initialized) { set_error("state not initialised"); return SSE_ESTATE; }
    const DevMesh &m = s->mesh->d;
    const int L = s->p.n_layers;
    if (!m.chain || L > kWave || (fe_edge_variant(m, L, 0, false) & 8)) {
        set_error("the gather-only edge pass needs canonical stencils, at most 64 layers and arrays below 4 GiB");
        return SSE_EINVAL;
    }
    Work &w = s->w;
    auto go = [&](auto zero) {
        using R = decltype(zero);
        FEEdgeArgs<R> a{};
        a.m = m;
        a.L = L;
        a.X = rp<R>(w.U);
        a.Un = rp<R>(w.U);
        a.h = w.Hs;
        a.rho = w.rho;
        a.B = rp<R>(w.B);
        a.Wtop = rp<R>(w.Wt);
        a.Z = rp<R>(w.Z);
        a.out = rp<R>(w.T2);
        launch_edge_gathers<R>(a, s->geom, s->stream);
    };
    if (s->rs == 4) go(0.0f);
    else go(0.0);
    SSE_HIP(hipGetLastError());
    return SSE_OK;
}

extern "C" int sse_debug_barotropic_substep(sse_state *s, int32_t scheme, int32_t M, double dt, const double *ubar,
                                            const double *zeta, const double *G, double *ubar1, double *zeta1,
                                            double *Fzeta) {
    if (!s || !ubar || !zeta || !G || !ubar1 || !zeta1 || !Fzeta) { set_error("NULL argument"); return SSE_EINVAL; }
    if (scheme != 2 && scheme != 3) { set_error("scheme must be 2 or 3"); return SSE_EINVAL; }
    if (M < 1 || !(dt > 0)) { set_error("M must be >= 1 and dt > 0"); return SSE_EINVAL; }
    const sse_mesh *m = s->mesh;
    const size_t C = m->C, E = m->E;
    Work &w = s->w;
    hipStream_t st = s->stream;
    std::vector<double> bi(E), zi(C), gi(E), bo(E), zo(C), fo(E);
    rows_to_internal(ubar, bi.data(), m->edge_old, 1);
    rows_to_internal(zeta, zi.data(), m->cell_old, 1);
    rows_to_internal(G, gi.data(), m->edge_old, 1);
    SSE_HIP(hipMemcpyAsync(w.ub1, bi.data(), E * 8, hipMemcpyHostToDevice, st));
    SSE_HIP(hipMemcpyAsync(w.z1, zi.data(), C * 8, hipMemcpyHostToDevice, st));
    SSE_HIP(hipMemcpyAsync(w.G0, gi.data(), E * 8, hipMemcpyHostToDevice, st));
    if (s->bt64)
        bt_loop<double>(s, scheme, M, dt, w.ub1, w.z1, w.G0, w.ub2, w.bt_zout, w.Fz1, bt_bufs(w));
    else
        bt_loop<float>(s, scheme, M, dt, w.ub1, w.z1, w.G0, w.ub2, w.bt_zout, w.Fz1, bt_bufs(w));
    if (int rc = take_launch_error(s)) return rc;
    SSE_HIP(hipGetLastError());
    int barrier_err = 0;
    SSE_HIP(hipMemcpyAsync(bo.data(), w.ub2, E * 8, hipMemcpyDeviceToHost, st));
    SSE_HIP(hipMemcpyAsync(zo.data(), w.bt_zout, C * 8, hipMemcpyDeviceToHost, st));
    SSE_HIP(hipMemcpyAsync(fo.data(), w.Fz1, E * 8, hipMemcpyDeviceToHost, st));
    SSE_HIP(hipMemcpyAsync(&barrier_err, w.flag + 32, sizeof(int), hipMemcpyDeviceToHost, st));
    SSE_HIP(hipStreamSynchronize(st));
    if (barrier_err) {
        set_error("a grid barrier of the persistent barotropic loop timed out");
        return SSE_EDEVICE;
    }
    rows_to_user(bo.data(), ubar1, m->edge_old, 1);
    rows_to_user(zo.data(), zeta1, m->cell_old, 1);
    rows_to_user(fo.data(), Fzeta, m->edge_old, 1);
    return SSE_OK;
}

extern "C" int sse_barotropic_substep_noalloc(sse_state *s, int32_t scheme, int32_t M, double dt, const double *ubar,
                                              const double *zeta, const double *G, double *ubar1, double *zeta1,
                                              double *Fzeta) {
    if (!s || !ubar || !zeta || !G || !ubar1 || !zeta1 || !Fzeta) { set_error("NULL argument"); return SSE_EINVAL; }
    if (scheme != 2 && scheme != 3) { set_error("scheme must be 2 or 3"); return SSE_EINVAL; }
    if (M < 1 || !(dt > 0) || !std::isfinite(dt)) { set_error("M must be >= 1 and dt > 0"); return SSE_EINVAL; }
    if (s->rec) { set_error("state is being recorded into a batch"); return SSE_ESTATE; }
    const DevMesh &dm = s->mesh->d;
    const size_t E = dm.E, C = dm.C;
    // 6 edge and 4 cell arrays of doubles (input, forcing, output and flux
    // permuted to the internal numbering, and the stages), each 256-byte aligned
    const size_t need = (6 * E + 4 * C) * sizeof(double) + 16 * kAlign;
    if (need > kStaticScratchBytes) {
        set_error("mesh too large for the allocation-free barotropic entry point (needs (6 E + 4 C) x 8 bytes of "
                  "its 64 MiB scratch)");
        return SSE_ENOMEM;
    }
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev != s->device) {
        set_error("the state's device must be current");
        return SSE_EINVAL;
    }
    void *base = scratch_address(dev);
    if (!base) { set_error("no device address for the static scratch array"); return SSE_EDEVICE; }
    char *p = static_cast<char *>(base);
    auto take = [&](size_t n) {
        void *r = p;
        p += align_up(n);
        return r;
    };
    const size_t bs = s->bt64 ? sizeof(double) : sizeof(float);
    double *iu = static_cast<double *>(take(E * 8)), *iz = static_cast<double *>(take(C * 8));
    double *iG = static_cast<double *>(take(E * 8)), *ou = static_cast<double *>(take(E * 8));
    double *oz = static_cast<double *>(take(C * 8)), *oF = static_cast<double *>(take(E * 8));
    BtBufs b{};
    b.u1 = take(E * bs);
    b.uh = take(E * bs);
    b.z1 = take(C * bs);
    b.zh = take(C * bs);
    if (!s->bt64) {
        b.ua = take(E * bs);
        b.za = take(C * bs);
        b.uo = take(E * bs);
        b.zo = take(C * bs);
    }
    hipStream_t st = s->stream;
    // caller numbering -> internal; every input is read before any output is written
    launch_permute(ubar, dm.edge_old, iu, (int)E, false, s->geom, st);
    launch_permute(zeta, dm.cell_old, iz, (int)C, false, s->geom, st);
    launch_permute(G, dm.edge_old, iG, (int)E, false, s->geom, st);
    const bool prof = s->prof, capturing = s->capturing;
    s->prof = false;  // no per-class events: their bookkeeping would grow host vectors
    // callers may capture this call in a graph, and it must leave the state's
    // workspace alone: never the persistent (cooperative) loop kernel, whose
    // barrier words live in the workspace
    s->capturing = true;
    if (s->bt64)
        bt_loop<double>(s, scheme, M, dt, iu, iz, iG, ou, oz, oF, b);
    else
        bt_loop<float>(s, scheme, M, dt, iu, iz, iG, ou, oz, oF, b);
    s->prof = prof;
    s->capturing = capturing;
    if (int rc = take_launch_error(s)) return rc;
    launch_permute(ou, dm.edge_old, ubar1, (int)E, true, s->geom, st);
    launch_permute(oz, dm.cell_old, zeta1, (int)C, true, s->geom, st);
    launch_permute(oF, dm.edge_old, Fzeta, (int)E, true, s->geom, st);
    SSE_HIP(hipGetLastError());
    return SSE_OK;
}

extern "C" int sse_debug_thickness_stage(sse_state *s, const double *h_in, const double *u, const double *uA,
                                         double dt, double *h_out, double *zeta_out) {
    if (!s || !h_in || !u || !uA || !h_out || !zeta_out) { set_error("NULL argument"); return SSE_EINVAL; }
    if (!s->initialized) { set_error("state not initialised (h_ref is needed)"); return SSE_ESTATE; }
    if (s->p.tracer) {
        set_error("the thickness-stage debug entry needs a state without tracer (tracer stages update the density)");
        return SSE_EINVAL;
    }
    const sse_mesh *m = s->mesh;
    const size_t L = s->p.n_layers, C = m->C, E = m->E;
    Work &w = s->w;
    hipStream_t st = s->stream;
    std::vector<double> hi(C * L), ui(E * L), ai(E), ho(C * L), zo(C);
    rows_to_internal(h_in, hi.data(), m->cell_old, L);
    rows_to_internal(u, ui.data(), m->edge_old, L);
    rows_to_internal(uA, ai.data(), m->edge_old, 1);
    SSE_HIP(hipMemcpyAsync(w.H1, hi.data(), C * L * 8, hipMemcpyHostToDevice, st));
    SSE_TRY(upload_real(s, w.T2, ui.data(), E * L));
    SSE_HIP(hipMemcpyAsync(w.uA, ai.data(), E * 8, hipMemcpyHostToDevice, st));
    const int Li = (int)L;
    if (s->rs == 4) {
        if (s->p.vcoord == SSE_ZSTAR) launch_edge_flux_sum<float>(m->d, Li, w.H1, rp<float>(w.T2), w.uA, w.Ftot, st);
        thickness<float>(s, w.H1, nullptr, COMB_NONE, w.H2, w.z_half, rp<float>(w.T2), 1.0, nullptr, 0.0, nullptr,
                         0.0, dt);
    } else {
        if (s->p.vcoord == SSE_ZSTAR) launch_edge_flux_sum<double>(m->d, Li, w.H1, rp<double>(w.T2), w.uA, w.Ftot, st);
        thickness<double>(s, w.H1, nullptr, COMB_NONE, w.H2, w.z_half, rp<double>(w.T2), 1.0, nullptr, 0.0,
                          nullptr, 0.0, dt);
    }
    SSE_HIP(hipGetLastError());
    SSE_HIP(hipMemcpyAsync(ho.data(), w.H2, C * L * 8, hipMemcpyDeviceToHost, st));
    SSE_HIP(hipMemcpyAsync(zo.data(), w.z_half, C * 8, hipMemcpyDeviceToHost, st));
    SSE_HIP(hipStreamSynchronize(st));
    rows_to_user(ho.data(), h_out, m->cell_old, L);
    rows_to_user(zo.data(), zeta_out, m->cell_old, 1);
    return SSE_OK;
}

// ===========================================================================
// Batched ensembles
// ===========================================================================
namespace {

struct BatchOp {
    Kind kind;
    int nk;
    int var;
    bool add;
    int blocks;
    size_t args_off, table_off;
    size_t lds;
};

}  // namespace

struct sse_batch {
    hipStream_t stream = nullptr;
    std::vector<sse_state *> members;
    Geom geom{};
    bool recorded = false;
    std::vector<BatchOp> prog;
    std::vector<uint8_t> image;   // argument blocks and block tables, device layout
    void *dev = nullptr;
    bool compiled = false;
    bool use_graph = false;
    hipGraphExec_t graph_exec = nullptr;
    size_t launches_per_step = 0;
};

namespace {

void batch_invalidate(sse_batch *b) {
    if (!b) return;
    if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
    b->graph_exec = nullptr;
    b->recorded = b->compiled = false;
    b->prog.clear();
    b->image.clear();
    b->dev = nullptr;
}

// Record one step of every member and merge equal launches into batched ones.
int batch_record(sse_batch *b) {
    if (b->recorded) return SSE_OK;
    if (b->members.empty()) { set_error("batch has no members"); return SSE_ESTATE; }
    const sse_state *s0 = b->members[0];
    struct Key {
        int seq, j, kind, nk, var, add;
        bool operator<(const Key &o) const {
            if (seq != o.seq) return seq < o.seq;
            if (j != o.j) return j < o.j;
            if (kind != o.kind) return kind < o.kind;
            if (nk != o.nk) return nk < o.nk;
            if (var != o.var) return var < o.var;
            return add < o.add;
        }
    };
    std::map<Key, std::vector<std::pair<int, RecEntry>>> groups;
    for (size_t mi = 0; mi < b->members.size(); ++mi) {
        sse_state *s = b->members[mi];
        if (s->p.precision != s0->p.precision || s->p.scheme != s0->p.scheme || s->p.vcoord != s0->p.vcoord) {
            set_error("batch members must share precision, scheme and vertical coordinate");
            return SSE_EINVAL;
        }
        Recorder r;
        const Geom saved = s->geom;
        s->geom = b->geom;
        s->rec = &r;
        enqueue_step(s);
        s->rec = nullptr;
        s->geom = saved;
        for (auto &e : r.entries) groups[Key{e.seq, e.j, (int)e.kind, e.nk, e.var, e.add ? 1 : 0}].emplace_back((int)mi, std::move(e));
    }
    auto align = [](size_t x) { return (x + kAlign - 1) / kAlign * kAlign; };
    b->prog.clear();
    b->image.clear();
    size_t off = 0;
    for (auto &kv : groups) {
        auto &v = kv.second;
        BatchOp op{v[0].second.kind, v[0].second.nk, v[0].second.var, v[0].second.add, 0, 0, 0, 0};
        const size_t asz = v[0].second.args.size();
        std::vector<int2> table;
        for (size_t q = 0; q < v.size(); ++q) {
            if (v[q].second.kind != op.kind || v[q].second.add != op.add || v[q].second.args.size() != asz) {
                set_error("internal: batch members recorded different step structures");
                return SSE_EINVAL;
            }
            for (int blk = 0; blk < v[q].second.blocks; ++blk) table.push_back(int2{(int)q, blk});
            op.lds = std::max(op.lds, v[q].second.lds);
        }
        op.blocks = (int)table.size();
        op.args_off = off;
        off = align(off + asz * v.size());
        op.table_off = off;
        off = align(off + table.size() * sizeof(int2));
        b->image.resize(off, 0);
        for (size_t q = 0; q < v.size(); ++q)
            std::memcpy(b->image.data() + op.args_off + q * asz, v[q].second.args.data(), asz);
        std::memcpy(b->image.data() + op.table_off, table.data(), table.size() * sizeof(int2));
        b->prog.push_back(op);
    }
    b->launches_per_step = b->prog.size();
    b->recorded = true;
    return SSE_OK;
}

template <typename A>
BatchLaunch<A> bl(const sse_batch *b, const BatchOp &op) {
    const char *base = static_cast<const char *>(b->dev);
    return BatchLaunch<A>{reinterpret_cast<const A *>(base + op.args_off),
                          reinterpret_cast<const int2 *>(base + op.table_off), op.blocks};
}

template <typename R>
void batch_enqueue(const sse_batch *b) {
    const Geom &g = b->geom;
    hipStream_t st = b->stream;
    const bool bt64 = b->members[0]->bt64;  // members share their precision mode
    for (const BatchOp &op : b->prog) {
        switch (op.kind) {
            case Kind::FE_CELL: launch_fe_cell_batch<R>(bl<FECellArgs<R>>(b, op), op.nk, op.add, g, st); break;
            case Kind::FE_VERTEX: launch_fe_vertex_batch<R>(bl<FEVertexArgs<R>>(b, op), op.nk, op.add, g, st); break;
            case Kind::FE_EDGE: launch_fe_edge_batch<R>(bl<FEEdgeArgs<R>>(b, op), op.nk, op.add, op.var, g, st); break;
            case Kind::BT_EVAL:
                if (bt64) launch_bt_eval_batch<double>(bl<BTEvalArgs<double>>(b, op), op.var != 0, g, st);
                else launch_bt_eval_batch<float>(bl<BTEvalArgs<float>>(b, op), op.var != 0, g, st);
                break;
            case Kind::BT_TILE:
                if (bt64)
                    launch_bt_substep_batch<double>(bl<BTTileArgs<double>>(b, op), b->members[0]->p.scheme, op.var,
                                                    op.lds, st);
                else
                    launch_bt_substep_batch<float>(bl<BTTileArgs<float>>(b, op), b->members[0]->p.scheme, op.var,
                                                   op.lds, st);
                break;
            case Kind::THICK: launch_thickness_batch(bl<THArgs>(b, op), op.nk, g, st); break;
            case Kind::THICK_ISO: launch_thickness_iso_batch<R>(bl<THIsoArgs<R>>(b, op), op.nk, g, st); break;
            case Kind::RECON: launch_recon_batch(bl<ReconArgs>(b, op), g, st); break;
            case Kind::ASSEMBLE: launch_assemble_batch<R>(bl<AssembleArgs<R>>(b, op), op.nk, g, st); break;
            case Kind::CONV_DF: launch_convert_batch<double, float>(bl<ConvArgs<double, float>>(b, op), g, st); break;
            case Kind::CONV_FD: launch_convert_batch<float, double>(bl<ConvArgs<float, double>>(b, op), g, st); break;
            case Kind::LAP: launch_lap_batch<R>(bl<LapArgs<R>>(b, op), op.nk, g, st); break;
            case Kind::DIV: launch_div_batch<R>(bl<DivArgs<R>>(b, op), op.nk, g, st); break;
            case Kind::TRACER: launch_tracer_batch<R>(bl<TracerArgs<R>>(b, op), op.nk, g, st); break;
        }
    }
}

void batch_enqueue_any(const sse_batch *b) {
    if (b->members[0]->rs == 4)
        batch_enqueue<float>(b);
    else
        batch_enqueue<double>(b);
}

}  // namespace

extern "C" int sse_batch_create(void *stream, sse_batch **out) {
    if (!out) { set_error("out is NULL"); return SSE_EINVAL; }
    sse_batch *b = new sse_batch();
    b->stream = static_cast<hipStream_t>(stream);
    *out = b;
    return SSE_OK;
}

extern "C" int sse_batch_destroy(sse_batch *b) {
    if (!b) return SSE_OK;
    for (sse_state *s : b->members) s->batch = nullptr;
    batch_invalidate(b);
    delete b;
    return SSE_OK;
}

extern "C" int sse_batch_add(sse_batch *b, sse_state *s) {
    if (!b || !s) { set_error("NULL argument"); return SSE_EINVAL; }
    if (!s->initialized) { set_error("batch members must be initialised"); return SSE_ESTATE; }
    if (s->p.tracer && !s->tracer_set) { set_error("tracer members need their temperature first"); return SSE_ESTATE; }
    if (s->batch) { set_error("state already belongs to a batch"); return SSE_ESTATE; }
    if (s->stream != b->stream) { set_error("batch members must use the batch's stream"); return SSE_EINVAL; }
    if (!b->members.empty()) {
        const sse_state *s0 = b->members[0];
        if (s->p.precision != s0->p.precision || s->p.scheme != s0->p.scheme || s->p.vcoord != s0->p.vcoord) {
            set_error("batch members must share precision, scheme and vertical coordinate");
            return SSE_EINVAL;
        }
    }
    b->members.push_back(s);
    s->batch = b;
    batch_invalidate(b);
    return SSE_OK;
}

extern "C" int sse_batch_remove(sse_batch *b, sse_state *s) {
    if (!b || !s) { set_error("NULL argument"); return SSE_EINVAL; }
    auto it = std::find(b->members.begin(), b->members.end(), s);
    if (it == b->members.end()) { set_error("state is not a member of this batch"); return SSE_EINVAL; }
    b->members.erase(it);
    s->batch = nullptr;
    batch_invalidate(b);
    return SSE_OK;
}

extern "C" int sse_batch_size(const sse_batch *b, int32_t *n) {
    if (!b || !n) { set_error("NULL argument"); return SSE_EINVAL; }
    *n = (int32_t)b->members.size();
    return SSE_OK;
}

extern "C" int sse_batch_set_geometry(sse_batch *b, int cols_per_block, int block_2d) {
    if (!b) { set_error("NULL batch"); return SSE_EINVAL; }
    Geom g{cols_per_block, block_2d};
    if (!geom_valid(g)) { set_error("geometry: cols_per_block in {1,2,4,8,16}, block_2d a multiple of 64 in [64, 1024]"); return SSE_EINVAL; }
    b->geom = g;
    batch_invalidate(b);
    return SSE_OK;
}

extern "C" int sse_batch_program_bytes(sse_batch *b, size_t *bytes) {
    if (!b || !bytes) { set_error("NULL argument"); return SSE_EINVAL; }
    int rc = batch_record(b);
    if (rc) return rc;
    *bytes = b->image.size();
    return SSE_OK;
}

extern "C" int sse_batch_compile(sse_batch *b, void *dev_buf, size_t bytes) {
    if (!b) { set_error("NULL batch"); return SSE_EINVAL; }
    int rc = batch_record(b);
    if (rc) return rc;
    if (!dev_buf || bytes < b->image.size()) { set_error("batch program buffer too small"); return SSE_ENOMEM; }
    if (reinterpret_cast<uintptr_t>(dev_buf) % kAlign) { set_error("batch program buffer must be 256-byte aligned"); return SSE_EINVAL; }
    if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
    b->graph_exec = nullptr;
    SSE_HIP(hipMemcpyAsync(dev_buf, b->image.data(), b->image.size(), hipMemcpyHostToDevice, b->stream));
    SSE_HIP(hipStreamSynchronize(b->stream));
    b->dev = dev_buf;
    b->compiled = true;
    return SSE_OK;
}

extern "C" int sse_batch_use_graph(sse_batch *b, int enable) {
    if (!b) { set_error("NULL batch"); return SSE_EINVAL; }
    if (enable && !b->stream) { set_error("HIP graphs need a non-default stream"); return SSE_EINVAL; }
    b->use_graph = enable != 0;
    if (b->graph_exec) (void)hipGraphExecDestroy(b->graph_exec);
    b->graph_exec = nullptr;
    return SSE_OK;
}

extern "C" int sse_batch_launches_per_step(sse_batch *b, int32_t *n) {
    if (!b || !n) { set_error("NULL argument"); return SSE_EINVAL; }
    int rc = batch_record(b);
    if (rc) return rc;
    *n = (int32_t)b->launches_per_step;
    return SSE_OK;
}

extern "C" int sse_batch_step_async(sse_batch *b, int32_t n) {
    if (!b) { set_error("NULL batch"); return SSE_EINVAL; }
    if (n < 0) { set_error("n must be >= 0"); return SSE_EINVAL; }
    if (!b->compiled) { set_error("batch program not compiled (sse_batch_compile)"); return SSE_ESTATE; }
    if (b->use_graph) {
        if (!b->graph_exec) {
            int rc = capture(b->stream, [&] { batch_enqueue_any(b); }, &b->graph_exec);
            if (rc) return rc;
        }
        for (int i = 0; i < n; ++i) SSE_HIP(hipGraphLaunch(b->graph_exec, b->stream));
        return SSE_OK;
    }
    for (int i = 0; i < n; ++i) batch_enqueue_any(b);
    SSE_HIP(hipGetLastError());
    return SSE_OK;
}

extern "C" int sse_batch_sync(sse_batch *b) {
    if (!b) { set_error("NULL batch"); return SSE_EINVAL; }
    SSE_HIP(hipStreamSynchronize(b->stream));
    int worst = SSE_OK;
    for (sse_state *s : b->members) {
        int rc = read_flag(s);
        if (rc && !worst) worst = rc;
    }
    return worst;
}

extern "C" int sse_batch_step(sse_batch *b, int32_t n) {
    int rc = sse_batch_step_async(b, n);
    if (rc) return rc;
    return sse_batch_sync(b);
}
