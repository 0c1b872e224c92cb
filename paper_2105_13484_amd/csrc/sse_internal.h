// Internal declarations shared by the host orchestration and the kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/ssprkse.h"

namespace sse {

constexpr int kMaxEdges = 6;    // edges per cell (hexagons / pentagons)
constexpr int kMaxEdges2 = 10;  // edges in the tangential-reconstruction stencil
constexpr int kWave = 64;       // CDNA wavefront
constexpr int kColsPerBlock = 4;
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
    const double *w = nullptr;              // [10][E]  W_{e,j}
    const double *wf = nullptr;             // [10][E]  W_{e,j} (f_e + f_j) / 2
    const double *dc = nullptr;             // [E]
    const double *dv = nullptr;             // [E]
    const uint8_t *emask = nullptr;         // [E]
    // vertices
    const int32_t *vert_edges = nullptr;    // [V][3]
    const double *vert_curl = nullptr;      // [V][3]  r_{v,e} d_e / A_v
};

}  // namespace sse

struct sse_mesh {
    sse::DevMesh d;
    int C = 0, E = 0, V = 0;
    int n_ocean_cells = 0;
    std::vector<int32_t> cells_on_edge;     // host copy (for debug helpers)
    void *dev_buf = nullptr;
    size_t dev_bytes = 0;
};

namespace sse {

// Sizes of the device mesh image (bytes) and the offsets of its tables.
struct MeshLayout {
    size_t off[32] = {};
    size_t total = 0;
};
MeshLayout mesh_layout(int C, int E, int V);

// Host-side table building (sse_mesh.cpp).
int validate_desc(const sse_mesh_desc *d, std::string &err);

struct HostMeshTables {
    std::vector<int32_t> cell_edges, cell_nbrs, cell_nedges, cell_edges_t, cell_nbrs_t;
    std::vector<double> cell_div, cell_ke, cell_div_t, H;
    std::vector<uint8_t> cmask;
    std::vector<int32_t> edge_cells, edge_verts, eoe, neoe;
    std::vector<double> w, wf, dc, dv;
    std::vector<uint8_t> emask;
    std::vector<int32_t> vert_edges;
    std::vector<double> vert_curl;
    int n_ocean_cells = 0;
};
void build_tables(const sse_mesh_desc *d, HostMeshTables &t);

void set_error(const std::string &msg);

}  // namespace sse
