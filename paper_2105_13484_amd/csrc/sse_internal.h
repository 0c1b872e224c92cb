// Internal declarations shared by the host orchestration and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/ssprkse.h"

namespace sse {

constexpr int kMaxEdges = 6;    // edges per cell (hexagons / pentagons)
constexpr int kMaxEdges2 = 10;  // edges in the tangential-reconstruction stencil
constexpr int kEdgeRec = 32;    // int32 words of one per-edge record (128 bytes)
constexpr int kWave = 64;       // CDNA wavefront
constexpr int kColsPerBlock = 4;
constexpr int kXcd = 8;           // accelerator complex dies of an MI355X
constexpr int kBlock = kWave * kColsPerBlock;
constexpr size_t kAlign = 256;

// Device-resident mesh tables.  Per-entity neighbour lists used by the
// column kernels are stored entity-major ([entity][slot]); the 2D barotropic
// kernels, with one thread per entity, read the slot-major copies
// ([slot][entity]) so that every load instruction is coalesced.
struct DevMesh {
    int C = 0, E = 0, V = 0;
    // cells
    const int32_t *cell_edges = nullptr;    // [C][6], padded with a valid index and zero coefficients
    const int32_t *cell_nbrs = nullptr;     // [C][6]
    const int32_t *cell_nedges = nullptr;   // [C]
    const double *cell_div = nullptr;       // [C][6]  s_{i,e} l_e / A_i
    const double *cell_ke = nullptr;        // [C][6]  l_e d_e / (4 A_i)
    const int32_t *cell_edges_t = nullptr;  // [6][C]
    const int32_t *cell_nbrs_t = nullptr;   // [6][C]
    const double *cell_div_t = nullptr;     // [6][C]
    const double *H = nullptr;              // [C]
    const uint8_t *cmask = nullptr;         // [C]
    // edges
    const int32_t *edge_cells = nullptr;    // [E][2]
    const int32_t *edge_verts = nullptr;    // [E][2]
    const int32_t *eoe = nullptr;           // [10][E]
    const int32_t *neoe = nullptr;          // [E]
    const int32_t *erec = nullptr;          // [E][32] per-edge record for the column kernels:
                                            //   stencil edges [10], cells [2] at 30/31, and either
                                            //   the stencil edges' vertices [10][2] (generic) or the
                                            //   vertex chains of the two cells (chain == 1)
    int chain = 0;                          // 1: stencils in canonical two-cell order (see sse_mesh.cpp)
    const double *w = nullptr;              // [10][E]  W_{e,j}
    const double *wf = nullptr;             // [10][E]  W_{e,j} (f_e + f_j) / 2
    const double *wpair = nullptr;          // [E][10][2] (W_{e,j} / 4, W_{e,j} (f_e + f_j) / 2), entity-major
    const double *dc = nullptr;             // [E]
    const double *dv = nullptr;             // [E]
    const double *inv_dc = nullptr;         // [E] 1 / d_e
    const double *inv_dv = nullptr;         // [E] 1 / l_e
    const uint8_t *emask = nullptr;         // [E]
    // vertices
    const int32_t *vert_edges = nullptr;    // [V][3]
    const double *vert_curl = nullptr;      // [V][3]  r_{v,e} d_e / A_v
    // FP32 copies of the tables the barotropic loop reads in mixed precision
    const float *wf_f = nullptr;            // [10][E]
    const float *inv_dc_f = nullptr;        // [E]
    const float *cell_div_t_f = nullptr;    // [6][C]
    const float *H_f = nullptr;             // [C]
    const float *wpair_f = nullptr;         // [E][10][2] wpair rounded to FP32 (the edge pass in mixed precision)
    // 16-bit index tables of the barotropic evaluation (delta16 == 1 when every
    // offset fits): stencil edges as e + eoe16[j][e]; the cells of edge e as
    // bc(e) + low / high half of ecells16[e]; the edges and neighbours of cell
    // i as be(i) + cedges16[j][i] and i + cnbrs16[j][i], with the fixed-point
    // bases bc(e) = (e ratio_ce) >> 16 and be(i) = (i ratio_ec) >> 16.
    int delta16 = 0;
    uint32_t ratio_ce = 0, ratio_ec = 0;
    const int16_t *eoe16 = nullptr;         // [10][E]
    const int32_t *ecells16 = nullptr;      // [E]
    const int16_t *cedges16 = nullptr;      // [6][C]
    const int16_t *cnbrs16 = nullptr;       // [6][C]
    // the caller's numbering: internal cell i / edge e is caller cell
    // cell_old[i] / edge edge_old[e]
    const int32_t *cell_old = nullptr;      // [C]
    const int32_t *edge_old = nullptr;      // [E]
};

// Fixed-point base of the 16-bit offsets (see DevMesh).
__host__ __device__ inline int delta_base(int x, uint32_t ratio) {
    return (int)(((unsigned long long)x * ratio) >> 16);
}

// Gather lists of the LDS-staged baroclinic edge pass.  The edges are cut
// into tiles of T consecutive edges; for every tile the unique edge columns
// (the tiles' edges and their reconstruction stencils), vertex columns and
// cell columns it reads are listed once, and every edge stores the 8-bit
// positions of its operands in those lists.
constexpr int kTileVariants = 3;
constexpr int kTileSizes[kTileVariants] = {8, 16, 32};
constexpr int kLocPerEdge = 36;  // self, c1, c2, v1, v2, stencil[10], stencil vertices[10][2], pad
struct DevTiles {
    int T = 0, nT = 0;
    int max_ue = 0, max_uv = 0, max_uc = 0;  // largest list sizes over the tiles
    const int32_t *ue_off = nullptr, *uv_off = nullptr, *uc_off = nullptr;  // [nT + 1]
    const int32_t *ue = nullptr, *uv = nullptr, *uc = nullptr;              // global ids
    const uint8_t *loc = nullptr;                                           // [E][kLocPerEdge]
};

}  // namespace sse

namespace sse {
// Tiled barotropic substeps.  The cells are cut into compact patches; a patch
// with its halo rings is everything one SSPRK3 substep (three evaluations)
// of its own cells and edges reads, so one workgroup advances its patch a
// whole substep with the state in LDS and the stencil tables in registers,
// and the launches per barotropic loop drop from 3M to M.
//
// Region of a patch, by level k = 0..3: cells R_k (R_0 the patch, R_{k+1} =
// R_k and its neighbours) and edges E_k (E_0 the owned edges, those whose
// first cell is in the patch; E_k = all edges of R_k for k >= 1), listed
// level by level, so a level-k set is a prefix of the region lists.  The
// evaluation that produces level k reads level k + 1.
constexpr int kBtThreads = 512;    // threads per workgroup
// Workgroups of a CU at once (4 waves per SIMD, 128 VGPRs): two, so one
// workgroup's table loads overlap the other's evaluations.
constexpr int kBtWavesPerSimd = 4;
// Target cells per patch.  Measured, C1 FP64 / mixed ms/step and C2 FP64 /
// mixed ms/step: 1024 threads and 352 cells (one workgroup per CU, no
// overlap): 7.98 / 6.23, 5.69 / 4.46; 512 threads and 176 cells: 7.85 /
// 6.08, 5.77 / 4.49; 160 cells: 7.87 / 6.12, 5.85 / 4.52.  From 192 cells
// the level-2 edges of many patches exceed 2 x 512, and the split halves
// cost more (8.45 ms C1).  256 threads with 72 or 88 cells (four workgroups
// per CU, a deeper halo per cell): the barotropic class alone takes 4.75 /
// 5.68 ms per C1 step in FP64 against 2.92.
constexpr int kBtPatch = 176;
constexpr int kBtEdgeSlots = 2;    // edges of level 2 per thread (at most)
constexpr int kBtRec = 12;         // ints per patch record
struct DevBtTiles {
    int nP = 0;                    // patches (0: tiling not available)
    int ks = 0;                    // edge slots per thread needed (1 or 2)
    int dry = 0;                   // 1: the mesh has land cells or coast edges
    size_t lds_d = 0, lds_f = 0;   // dynamic LDS bytes for R = double / float
    // per patch: e0, es0, c0, cs0, ne[4], nc[4] (offsets into the region
    // lists / the stencil tables, prefix counts per level)
    const int32_t *patch = nullptr;
    const int32_t *eid = nullptr;     // [sum ne3] global edge of each region edge
    const int32_t *cid = nullptr;     // [sum nc3] global cell of each region cell
    const double *cH = nullptr;       // [sum nc3] H of region cells
    const float *cH_f = nullptr;
    // stencil tables of the edges of levels 0..2 (es0 + le), per patch slot-major
    // with stride ne2: entry (j, le) at es0 * J + j * ne2 + le
    const uint32_t *ec = nullptr;     // [sum ne2] local c1 | c2 << 15 | wet << 30
    const uint32_t *enb = nullptr;    // [5][..] local stencil edges, two 16-bit indices per word
    const double *ew = nullptr;       // [10][..] W (f_e + f_j) / 2
    const float *ew_f = nullptr;
    const double *eidc = nullptr;     // [..] 1 / d_e
    const float *eidc_f = nullptr;
    // cell tables of the cells of levels 0..2 (cs0 + lc), stride nc2
    const uint32_t *cen = nullptr;    // [6][..] local edge | local neighbour << 16
    const double *ccd = nullptr;      // [6][..] s l / A
    const float *ccd_f = nullptr;
    const uint8_t *cwet = nullptr;    // [..]
};
}  // namespace sse

namespace sse {
struct PermutedDesc;
}

struct sse_mesh {
    sse::DevMesh d;
    int C = 0, E = 0, V = 0;
    int n_ocean_cells = 0;
    // Internal (locality) numbering: entity i of the device arrays is entity
    // cell_old[i] / edge_old[i] of the caller's numbering.
    std::vector<int32_t> cell_old, edge_old;
    std::vector<int32_t> cells_on_edge;     // host copy (for debug helpers)
    // Gather lists of the LDS-staged edge pass (T = 8, 16, 32 edges per
    // tile), built and uploaded into their reserved part of the mesh buffer
    // the first time a state selects the variant (ensure_tiles).
    sse::DevTiles tiles[sse::kTileVariants];
    size_t tile_off[sse::kTileVariants] = {};
    int tile_state[sse::kTileVariants] = {};  // 0 not built, 1 built, -1 not possible
    std::mutex tile_mu;
    std::unique_ptr<sse::PermutedDesc> host_desc;  // internal numbering, for building the lists
    sse::DevBtTiles bt;                       // patches of the tiled barotropic substeps
    void *dev_buf = nullptr;
    size_t dev_bytes = 0;
};

namespace sse {

// Sizes of the device mesh image (bytes) and the offsets of its tables, in
// the order in which mesh_create uploads them.
constexpr int kMeshTables = 35;
void mesh_table_sizes(int C, int E, int V, size_t (&sizes)[kMeshTables]);
struct MeshLayout {
    size_t off[kMeshTables] = {};
    size_t total = 0;
};
MeshLayout mesh_layout(int C, int E, int V);

// Host-side table building (sse_mesh.cpp).
int validate_desc(const sse_mesh_desc *d, std::string &err);

struct HostMeshTables {
    std::vector<int32_t> cell_edges, cell_nbrs, cell_nedges, cell_edges_t, cell_nbrs_t;
    std::vector<double> cell_div, cell_ke, cell_div_t, H;
    std::vector<uint8_t> cmask;
    std::vector<int32_t> edge_cells, edge_verts, eoe, neoe, erec;
    std::vector<double> w, wf, dc, dv, inv_dc, inv_dv, wpair;
    std::vector<uint8_t> emask;
    std::vector<int32_t> vert_edges;
    std::vector<double> vert_curl;
    std::vector<float> wf_f, inv_dc_f, cell_div_t_f, H_f, wpair_f;
    std::vector<int16_t> eoe16, cedges16, cnbrs16;
    std::vector<int32_t> ecells16;
    int delta16 = 0;
    uint32_t ratio_ce = 0, ratio_ec = 0;
    int n_ocean_cells = 0;
    // [E][kChainWords] vertex chains of canonical stencils (empty: generic)
    std::vector<int32_t> chain;
};
void build_tables(const sse_mesh_desc *d, HostMeshTables &t);

struct HostTiles {
    int T = 0, nT = 0, max_ue = 0, max_uv = 0, max_uc = 0;
    std::vector<int32_t> ue_off, uv_off, uc_off, ue, uv, uc;
    std::vector<uint8_t> loc;
};
// Returns false if a tile needs more than 255 entries in one list.
bool build_tiles(const sse_mesh_desc *d, int T, HostTiles &t);
size_t tiles_bytes(const sse_mesh_desc *d, int T);
// Bytes of the FP32 weight pairs (DevMesh::wpair_f), placed after the tile
// tables so that the other tables keep their offsets in the mesh image.
size_t wpair_f_bytes(const sse_mesh_desc *d);

// Locality order of a mesh (new -> old and old -> new numbering): cells in
// compact breadth-first patches of `patch` cells, edges following the first
// cell that lists them, vertices following the first edge that lists them.
struct MeshOrder {
    std::vector<int32_t> cell_old, edge_old, vert_old;
    std::vector<int32_t> cell_new, edge_new, vert_new;
};
void locality_order(const sse_mesh_desc *d, int patch, MeshOrder &o);

// A copy of a mesh description renumbered by `o` (same conventions; the
// stencil order inside every row is kept, so results do not change).
struct PermutedDesc {
    sse_mesh_desc d{};
    std::vector<int32_t> coe, eoc, neoc, voe, eov, eoe, neoe;
    std::vector<double> w, dc, dv, f, area, H, tri;
    std::vector<uint8_t> mask;
};
void permute_desc(const sse_mesh_desc *d, const MeshOrder &o, PermutedDesc &p);

// Rewrites every reconstruction stencil of p in the canonical two-cell order
// and returns the vertex chains ([E][kChainWords]), or returns false and
// leaves p unchanged when some stencil is not "the other edges of the two
// cells of e" (then the generic tables are used).
constexpr int kChainWords = 11;  // A0..A5, B0..B3, flag (A0 is vertex 0 of the edge)
bool canonical_stencils(PermutedDesc &p, std::vector<int32_t> &chain);

// Patches of the tiled barotropic substeps, computed in the numbering of d:
// breadth-first patches of about kBtPatch cells, split in two (in their
// breadth-first order) until every patch's level-2 region fits the
// workgroup (kBtEdgeSlots edges and one cell per thread).  pid[c] = patch of
// cell c.  Returns false if no such partition exists.
bool bt_partition(const sse_mesh_desc *d, std::vector<int32_t> &pid, int &nP);

struct HostBtTiles {
    int nP = 0, ks = 0;
    size_t lds_d = 0, lds_f = 0;
    std::vector<int32_t> patch, eid, cid;
    std::vector<double> cH, ew, eidc, ccd;
    std::vector<float> cH_f, ew_f, eidc_f, ccd_f;
    std::vector<uint32_t> ec, enb, cen;
    std::vector<uint8_t> cwet;
};
// Region lists and tables of the partition pid (numbering of d, the same
// numbering as the tables t).  With t == nullptr only the sizes are filled
// (patch records, list lengths), which is what the device-bytes query needs.
bool build_bt_tiles(const sse_mesh_desc *d, const std::vector<int32_t> &pid, int nP, const HostMeshTables *t,
                    HostBtTiles &bt);
// Device bytes of the tiled barotropic tables of d (0 if d cannot be tiled),
// and the partition itself; both come from a cache keyed by the topology.
size_t bt_tiles_bytes(const sse_mesh_desc *d);
bool bt_cached_partition(const sse_mesh_desc *d, std::vector<int32_t> &pid, int &nP);
// Range checks of the topology tables the size queries read.
int check_topology(const sse_mesh_desc *d, std::string &err);

void set_error(const std::string &msg);

}  // namespace sse
