// Host-side mesh validation and construction of the device table images.
//
// The TRiSK operators (Section 5 opening of the paper; Thuburn et al. 2009,
// Ringler et al. 2010) are applied on the GPU through precomputed
// per-entity coefficients:
//   divergence  (div F)_i  = sum_j [s_{i,e_j} l_{e_j} / A_i] F_{e_j}
//   kinetic en. K_i        = sum_j [l_{e_j} d_{e_j} / (4 A_i)] u_{e_j}^2
//   curl        zeta_v     = sum_j [r_{v,e_j} d_{e_j} / A_v] u_{e_j}
//   Coriolis    -f k x u   = sum_j [W_{e,j} (f_e + f_{e_j}) / 2] u_{e_j}
// with s = +1 where the edge normal leaves the cell and r = +1 where the
// vertex is the edge's second vertex.
#include <algorithm>
#include <cmath>
#include <deque>
#include <cstdio>
#include <mutex>
#include <cstring>
#include <string>

#include "sse_internal.h"

namespace sse {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

}  // namespace sse

extern "C" const char *sse_last_error(void) { return sse::g_last_error.c_str(); }

extern "C" const char *sse_version(void) { return "ssprkse 0.1 (gfx950)"; }

namespace sse {

static std::string fmt(const char *f, long a = 0, long b = 0, long c = 0) {
    char buf[256];
    std::snprintf(buf, sizeof buf, f, a, b, c);
    return buf;
}

int validate_desc(const sse_mesh_desc *d, std::string &err) {
    if (!d) { err = "mesh description is NULL"; return SSE_EINVAL; }
    const long C = d->n_cells, E = d->n_edges, V = d->n_vertices;
    if (C <= 0 || E <= 0 || V <= 0) { err = "mesh counts must be positive"; return SSE_EINVAL; }
    if (d->max_edges < 3 || d->max_edges > kMaxEdges) { err = "max_edges must be in [3, 6]"; return SSE_EINVAL; }
    if (d->max_edges2 < 1 || d->max_edges2 > kMaxEdges2) { err = "max_edges2 must be in [1, 10]"; return SSE_EINVAL; }
    const void *req[] = {d->cells_on_edge, d->edges_on_cell, d->n_edges_on_cell, d->vertices_on_edge,
                         d->edges_on_vertex, d->edges_on_edge, d->n_edges_on_edge, d->weights_on_edge,
                         d->dc_edge, d->dv_edge, d->f_edge, d->area_cell, d->bottom_depth,
                         d->area_triangle, d->cell_mask};
    for (const void *p : req)
        if (!p) { err = "a required mesh table is NULL"; return SSE_EINVAL; }
    const int me = d->max_edges, me2 = d->max_edges2;
    for (long e = 0; e < E; ++e) {
        for (int s = 0; s < 2; ++s) {
            long c = d->cells_on_edge[2 * e + s], v = d->vertices_on_edge[2 * e + s];
            if (c < 0 || c >= C) { err = fmt("cells_on_edge[%ld] out of range", e); return SSE_EINVAL; }
            if (v < 0 || v >= V) { err = fmt("vertices_on_edge[%ld] out of range", e); return SSE_EINVAL; }
        }
        if (d->cells_on_edge[2 * e] == d->cells_on_edge[2 * e + 1]) { err = fmt("edge %ld joins a cell to itself", e); return SSE_EINVAL; }
        if (!(d->dc_edge[e] > 0) || !(d->dv_edge[e] > 0) || !std::isfinite(d->dc_edge[e]) || !std::isfinite(d->dv_edge[e])) {
            err = fmt("edge %ld has a non-positive length", e); return SSE_EINVAL;
        }
        if (!std::isfinite(d->f_edge[e])) { err = fmt("f_edge[%ld] is not finite", e); return SSE_EINVAL; }
        int n = d->n_edges_on_edge[e];
        if (n < 0 || n > me2) { err = fmt("n_edges_on_edge[%ld] = %ld out of range", e, n); return SSE_EINVAL; }
        for (int j = 0; j < n; ++j) {
            long ep = d->edges_on_edge[e * me2 + j];
            if (ep < 0 || ep >= E) { err = fmt("edges_on_edge[%ld][%ld] out of range", e, j); return SSE_EINVAL; }
            if (!std::isfinite(d->weights_on_edge[e * me2 + j])) { err = fmt("weights_on_edge[%ld][%ld] not finite", e, j); return SSE_EINVAL; }
        }
    }
    for (long i = 0; i < C; ++i) {
        int n = d->n_edges_on_cell[i];
        if (n < 3 || n > me) { err = fmt("n_edges_on_cell[%ld] = %ld out of range", i, n); return SSE_EINVAL; }
        if (!(d->area_cell[i] > 0) || !std::isfinite(d->area_cell[i])) { err = fmt("area_cell[%ld] not positive", i); return SSE_EINVAL; }
        if (!(d->bottom_depth[i] >= 0) || !std::isfinite(d->bottom_depth[i])) { err = fmt("bottom_depth[%ld] invalid", i); return SSE_EINVAL; }
        if (d->cell_mask[i] && !(d->bottom_depth[i] > 0)) { err = fmt("ocean cell %ld has zero depth", i); return SSE_EINVAL; }
        for (int j = 0; j < n; ++j) {
            long e = d->edges_on_cell[i * me + j];
            if (e < 0 || e >= E) { err = fmt("edges_on_cell[%ld][%ld] out of range", i, j); return SSE_EINVAL; }
            if (d->cells_on_edge[2 * e] != i && d->cells_on_edge[2 * e + 1] != i) {
                err = fmt("edge %ld listed on cell %ld does not touch it", e, i); return SSE_EINVAL;
            }
        }
    }
    for (long v = 0; v < V; ++v) {
        if (!(d->area_triangle[v] > 0) || !std::isfinite(d->area_triangle[v])) { err = fmt("area_triangle[%ld] not positive", v); return SSE_EINVAL; }
        for (int j = 0; j < 3; ++j) {
            long e = d->edges_on_vertex[3 * v + j];
            if (e < 0 || e >= E) { err = fmt("edges_on_vertex[%ld][%ld] out of range", v, j); return SSE_EINVAL; }
            if (d->vertices_on_edge[2 * e] != v && d->vertices_on_edge[2 * e + 1] != v) {
                err = fmt("edge %ld listed on vertex %ld does not touch it", e, v); return SSE_EINVAL;
            }
        }
    }
    // Energy neutrality of the Coriolis weights: l_e d_e W_ee' = -l_e' d_e' W_e'e.
    for (long e = 0; e < E; ++e) {
        int n = d->n_edges_on_edge[e];
        double scale = 0;
        for (int j = 0; j < n; ++j)
            scale = std::fmax(scale, std::fabs(d->dv_edge[e] * d->dc_edge[e] * d->weights_on_edge[e * me2 + j]));
        for (int j = 0; j < n; ++j) {
            long ep = d->edges_on_edge[e * me2 + j];
            int np = d->n_edges_on_edge[ep], found = -1;
            for (int q = 0; q < np; ++q)
                if (d->edges_on_edge[ep * me2 + q] == e) { found = q; break; }
            if (found < 0) { err = fmt("edges_on_edge is not symmetric at edges %ld/%ld", e, ep); return SSE_EINVAL; }
            double a = d->dv_edge[e] * d->dc_edge[e] * d->weights_on_edge[e * me2 + j];
            double b = d->dv_edge[ep] * d->dc_edge[ep] * d->weights_on_edge[ep * me2 + found];
            if (std::fabs(a + b) > 1e-10 * (scale + 1e-300)) {
                err = fmt("weights_on_edge are not antisymmetric at edges %ld/%ld", e, ep); return SSE_EINVAL;
            }
        }
    }
    return SSE_OK;
}

void mesh_table_sizes(int C_, int E_, int V_, size_t (&sizes)[kMeshTables]) {
    const size_t C = C_, E = E_, V = V_;
    const size_t tab[kMeshTables] = {
        C * 6 * 4, C * 6 * 4, C * 4, C * 6 * 8, C * 6 * 8,      // cell_edges, cell_nbrs, cell_nedges, cell_div, cell_ke
        C * 6 * 4, C * 6 * 4, C * 6 * 8, C * 8, C,              // cell_edges_t, cell_nbrs_t, cell_div_t, H, cmask
        E * 2 * 4, E * 2 * 4, E * 10 * 4, E * 4, E * 10 * 8,    // edge_cells, edge_verts, eoe, neoe, w
        E * 10 * 8, E * 8, E * 8, E,                            // wf, dc, dv, emask
        V * 3 * 4, V * 3 * 8,                                   // vert_edges, vert_curl
        E * 32 * 4, E * 8, E * 8, E * 20 * 8,                   // erec, inv_dc, inv_dv, wpair
        E * 10 * 4, E * 4, C * 6 * 4, C * 4,                    // wf_f, inv_dc_f, cell_div_t_f, H_f
        E * 10 * 2, E * 4, C * 6 * 2, C * 6 * 2,                // eoe16, ecells16, cedges16, cnbrs16
        C * 4, E * 4};                                          // cell_old, edge_old
    for (int i = 0; i < kMeshTables; ++i) sizes[i] = tab[i];
}

MeshLayout mesh_layout(int C, int E, int V) {
    MeshLayout L;
    size_t sizes[kMeshTables];
    mesh_table_sizes(C, E, V, sizes);
    size_t off = 0;
    for (int i = 0; i < kMeshTables; ++i) {
        L.off[i] = off;
        off += (sizes[i] + kAlign - 1) / kAlign * kAlign;
    }
    L.total = off;
    return L;
}

void build_tables(const sse_mesh_desc *d, HostMeshTables &t) {
    const int C = d->n_cells, E = d->n_edges, V = d->n_vertices;
    const int me = d->max_edges, me2 = d->max_edges2;
    t.cell_edges.assign((size_t)C * 6, 0);
    t.cell_nbrs.assign((size_t)C * 6, 0);
    t.cell_nedges.assign(C, 0);
    t.cell_div.assign((size_t)C * 6, 0.0);
    t.cell_ke.assign((size_t)C * 6, 0.0);
    t.H.assign(C, 0.0);
    t.cmask.assign(C, 0);
    t.n_ocean_cells = 0;
    for (int i = 0; i < C; ++i) {
        int n = d->n_edges_on_cell[i];
        t.cell_nedges[i] = n;
        t.H[i] = d->bottom_depth[i];
        t.cmask[i] = d->cell_mask[i] ? 1 : 0;
        t.n_ocean_cells += t.cmask[i];
        for (int j = 0; j < 6; ++j) {
            if (j < n) {
                int e = d->edges_on_cell[i * me + j];
                int c1 = d->cells_on_edge[2 * e], c2 = d->cells_on_edge[2 * e + 1];
                double s = (c1 == i) ? 1.0 : -1.0;
                t.cell_edges[i * 6 + j] = e;
                t.cell_nbrs[i * 6 + j] = (c1 == i) ? c2 : c1;
                t.cell_div[i * 6 + j] = s * d->dv_edge[e] / d->area_cell[i];
                t.cell_ke[i * 6 + j] = 0.25 * d->dv_edge[e] * d->dc_edge[e] / d->area_cell[i];
            } else {  // padding: a valid index with zero coefficients
                t.cell_edges[i * 6 + j] = t.cell_edges[i * 6];
                t.cell_nbrs[i * 6 + j] = t.cell_nbrs[i * 6];
            }
        }
    }
    t.cell_edges_t.assign((size_t)C * 6, 0);
    t.cell_nbrs_t.assign((size_t)C * 6, 0);
    t.cell_div_t.assign((size_t)C * 6, 0.0);
    for (int i = 0; i < C; ++i)
        for (int j = 0; j < 6; ++j) {
            t.cell_edges_t[(size_t)j * C + i] = t.cell_edges[i * 6 + j];
            t.cell_nbrs_t[(size_t)j * C + i] = t.cell_nbrs[i * 6 + j];
            t.cell_div_t[(size_t)j * C + i] = t.cell_div[i * 6 + j];
        }
    t.edge_cells.assign(d->cells_on_edge, d->cells_on_edge + 2 * (size_t)E);
    t.edge_verts.assign(d->vertices_on_edge, d->vertices_on_edge + 2 * (size_t)E);
    t.eoe.assign((size_t)E * 10, 0);
    t.neoe.assign(E, 0);
    t.w.assign((size_t)E * 10, 0.0);
    t.wf.assign((size_t)E * 10, 0.0);
    t.dc.assign(d->dc_edge, d->dc_edge + E);
    t.dv.assign(d->dv_edge, d->dv_edge + E);
    t.emask.assign(E, 0);
    for (int e = 0; e < E; ++e) {
        int c1 = d->cells_on_edge[2 * e], c2 = d->cells_on_edge[2 * e + 1];
        t.emask[e] = (d->cell_mask[c1] && d->cell_mask[c2]) ? 1 : 0;
        int n = d->n_edges_on_edge[e];
        t.neoe[e] = n;
        for (int j = 0; j < 10; ++j) {
            const int ep = j < n ? d->edges_on_edge[e * me2 + j] : -1;
            if (ep >= 0) {
                double wj = d->weights_on_edge[e * me2 + j];
                t.eoe[(size_t)j * E + e] = ep;
                t.w[(size_t)j * E + e] = wj;
                t.wf[(size_t)j * E + e] = wj * (0.5 * (d->f_edge[e] + d->f_edge[ep]));
            } else {
                t.eoe[(size_t)j * E + e] = e;
            }
        }
    }
    t.wpair.assign((size_t)E * 20, 0.0);
    for (int e = 0; e < E; ++e)
        for (int j = 0; j < 10; ++j) {
            t.wpair[(size_t)e * 20 + 2 * j] = 0.25 * t.w[(size_t)j * E + e];
            t.wpair[(size_t)e * 20 + 2 * j + 1] = t.wf[(size_t)j * E + e];
        }
    t.erec.assign((size_t)E * kEdgeRec, 0);
    t.inv_dc.assign(E, 0.0);
    t.inv_dv.assign(E, 0.0);
    for (int e = 0; e < E; ++e) {
        t.inv_dc[e] = 1.0 / d->dc_edge[e];
        t.inv_dv[e] = 1.0 / d->dv_edge[e];
        int32_t *r = &t.erec[(size_t)e * kEdgeRec];
        for (int j = 0; j < 10; ++j) {
            const int ep = t.eoe[(size_t)j * E + e];
            r[j] = ep;
            if (t.chain.empty()) {
                r[10 + 2 * j] = d->vertices_on_edge[2 * ep];
                r[11 + 2 * j] = d->vertices_on_edge[2 * ep + 1];
            }
        }
        if (!t.chain.empty())
            for (int q = 0; q < kChainWords; ++q) r[10 + q] = t.chain[(size_t)e * kChainWords + q];
        r[30] = d->cells_on_edge[2 * e];
        r[31] = d->cells_on_edge[2 * e + 1];
    }
    t.vert_edges.assign(d->edges_on_vertex, d->edges_on_vertex + 3 * (size_t)V);
    t.vert_curl.assign((size_t)V * 3, 0.0);
    for (int v = 0; v < V; ++v)
        for (int j = 0; j < 3; ++j) {
            int e = d->edges_on_vertex[3 * v + j];
            double r = (d->vertices_on_edge[2 * e + 1] == v) ? 1.0 : -1.0;
            t.vert_curl[v * 3 + j] = r * d->dc_edge[e] / d->area_triangle[v];
        }
    // 16-bit offsets of the barotropic index tables, if every one fits
    t.ratio_ce = (uint32_t)std::lround(65536.0 * C / E);
    t.ratio_ec = (uint32_t)std::lround(65536.0 * E / C);
    t.eoe16.assign((size_t)E * 10, 0);
    t.ecells16.assign(E, 0);
    t.cedges16.assign((size_t)C * 6, 0);
    t.cnbrs16.assign((size_t)C * 6, 0);
    bool fits = true;
    auto put16 = [&](long v) -> int16_t {
        if (v < -32767 || v > 32767) fits = false;
        return (int16_t)(fits ? v : 0);
    };
    for (int e = 0; e < E && fits; ++e) {
        for (int j = 0; j < 10; ++j) t.eoe16[(size_t)j * E + e] = put16((long)t.eoe[(size_t)j * E + e] - e);
        const int bc = delta_base(e, t.ratio_ce);
        const int16_t a = put16((long)t.edge_cells[2 * (size_t)e] - bc);
        const int16_t b = put16((long)t.edge_cells[2 * (size_t)e + 1] - bc);
        t.ecells16[e] = (int32_t)(((uint32_t)(uint16_t)b << 16) | (uint16_t)a);
    }
    for (int i = 0; i < C && fits; ++i) {
        const int be = delta_base(i, t.ratio_ec);
        for (int j = 0; j < 6; ++j) {
            t.cedges16[(size_t)j * C + i] = put16((long)t.cell_edges_t[(size_t)j * C + i] - be);
            t.cnbrs16[(size_t)j * C + i] = put16((long)t.cell_nbrs_t[(size_t)j * C + i] - i);
        }
    }
    t.delta16 = fits ? 1 : 0;
    auto to_f32 = [](const std::vector<double> &src, std::vector<float> &dst) {
        dst.resize(src.size());
        for (size_t i = 0; i < src.size(); ++i) dst[i] = (float)src[i];
    };
    to_f32(t.wf, t.wf_f);
    to_f32(t.inv_dc, t.inv_dc_f);
    to_f32(t.cell_div_t, t.cell_div_t_f);
    to_f32(t.H, t.H_f);
    to_f32(t.wpair, t.wpair_f);
}

bool build_tiles(const sse_mesh_desc *d, int T, HostTiles &t) {
    const int E = d->n_edges, me2 = d->max_edges2;
    t.T = T;
    t.nT = (E + T - 1) / T;
    t.ue_off.assign(t.nT + 1, 0);
    t.uv_off.assign(t.nT + 1, 0);
    t.uc_off.assign(t.nT + 1, 0);
    t.ue.clear();
    t.uv.clear();
    t.uc.clear();
    t.loc.assign((size_t)E * kLocPerEdge, 0);
    t.max_ue = t.max_uv = t.max_uc = 0;
    std::vector<int> ue, uv, uc;
    auto slot = [](std::vector<int> &list, int id) -> int {
        for (size_t i = 0; i < list.size(); ++i)
            if (list[i] == id) return (int)i;
        list.push_back(id);
        return (int)list.size() - 1;
    };
    for (int tile = 0; tile < t.nT; ++tile) {
        ue.clear();
        uv.clear();
        uc.clear();
        const int e0 = tile * T, e1 = std::min(E, e0 + T);
        for (int e = e0; e < e1; ++e) {
            uint8_t *L = &t.loc[(size_t)e * kLocPerEdge];
            int ids[5] = {slot(ue, e), slot(uc, d->cells_on_edge[2 * e]), slot(uc, d->cells_on_edge[2 * e + 1]),
                          slot(uv, d->vertices_on_edge[2 * e]), slot(uv, d->vertices_on_edge[2 * e + 1])};
            for (int q = 0; q < 5; ++q) L[q] = (uint8_t)ids[q];
            const int n = d->n_edges_on_edge[e];
            for (int j = 0; j < kMaxEdges2; ++j) {
                // padded stencil slots point at the edge itself (zero weight)
                const int ep = j < n ? d->edges_on_edge[e * me2 + j] : e;
                L[5 + j] = (uint8_t)slot(ue, ep);
                L[15 + 2 * j] = (uint8_t)slot(uv, d->vertices_on_edge[2 * ep]);
                L[16 + 2 * j] = (uint8_t)slot(uv, d->vertices_on_edge[2 * ep + 1]);
            }
        }
        if (ue.size() > 255 || uv.size() > 255 || uc.size() > 255) return false;
        t.max_ue = std::max(t.max_ue, (int)ue.size());
        t.max_uv = std::max(t.max_uv, (int)uv.size());
        t.max_uc = std::max(t.max_uc, (int)uc.size());
        t.ue.insert(t.ue.end(), ue.begin(), ue.end());
        t.uv.insert(t.uv.end(), uv.begin(), uv.end());
        t.uc.insert(t.uc.end(), uc.begin(), uc.end());
        t.ue_off[tile + 1] = (int32_t)t.ue.size();
        t.uv_off[tile + 1] = (int32_t)t.uv.size();
        t.uc_off[tile + 1] = (int32_t)t.uc.size();
    }
    return true;
}

// Upper bound of the device bytes of one tile table set (lists at their
// worst-case length T * 11, 2T * 11 and 2T per tile).
size_t wpair_f_bytes(const sse_mesh_desc *d) {
    return ((size_t)d->n_edges * 20 * 4 + kAlign - 1) / kAlign * kAlign;
}

size_t tiles_bytes(const sse_mesh_desc *d, int T) {
    const size_t E = d->n_edges, nT = (E + T - 1) / T;
    auto al = [](size_t x) { return (x + kAlign - 1) / kAlign * kAlign; };
    return 3 * al((nT + 1) * 4) + al(nT * T * 11 * 4) + al(nT * T * 22 * 4) + al(nT * T * 2 * 4) +
           al(E * kLocPerEdge);
}


// ---------------------------------------------------------------------------
// Locality ordering
// ---------------------------------------------------------------------------
void locality_order(const sse_mesh_desc *d, int patch, MeshOrder &o) {
    const int C = d->n_cells, E = d->n_edges, V = d->n_vertices, me = d->max_edges;
    o.cell_old.clear();
    o.cell_old.reserve(C);
    std::vector<char> taken(C, 0);
    std::deque<int> front, q;
    int scan = 0;
    auto neighbours = [&](int c, auto &&f) {
        for (int j = 0; j < d->n_edges_on_cell[c]; ++j) {
            const int e = d->edges_on_cell[(size_t)c * me + j];
            if (e < 0) continue;
            const int a = d->cells_on_edge[2 * (size_t)e], b = d->cells_on_edge[2 * (size_t)e + 1];
            const int nb = a == c ? b : a;
            if (nb >= 0 && nb != c) f(nb);
        }
    };
    while ((int)o.cell_old.size() < C) {
        int seed = -1;
        while (!front.empty()) {
            const int c = front.front();
            front.pop_front();
            if (!taken[c]) { seed = c; break; }
        }
        if (seed < 0) {
            while (taken[scan]) ++scan;
            seed = scan;
        }
        // grow one patch breadth-first from the seed
        int count = 0;
        q.clear();
        q.push_back(seed);
        taken[seed] = 1;
        while (!q.empty()) {
            const int c = q.front();
            q.pop_front();
            o.cell_old.push_back(c);
            ++count;
            neighbours(c, [&](int nb) {
                if (taken[nb]) return;
                if (count + (int)q.size() < patch) {
                    taken[nb] = 1;
                    q.push_back(nb);
                } else {
                    front.push_back(nb);
                }
            });
        }
    }
    o.cell_new.assign(C, -1);
    for (int i = 0; i < C; ++i) o.cell_new[o.cell_old[i]] = i;
    o.edge_new.assign(E, -1);
    o.edge_old.clear();
    o.edge_old.reserve(E);
    for (int i = 0; i < C; ++i) {
        const int c = o.cell_old[i];
        for (int j = 0; j < d->n_edges_on_cell[c]; ++j) {
            const int e = d->edges_on_cell[(size_t)c * me + j];
            if (e >= 0 && o.edge_new[e] < 0) {
                o.edge_new[e] = (int)o.edge_old.size();
                o.edge_old.push_back(e);
            }
        }
    }
    for (int e = 0; e < E; ++e)
        if (o.edge_new[e] < 0) {
            o.edge_new[e] = (int)o.edge_old.size();
            o.edge_old.push_back(e);
        }
    o.vert_new.assign(V, -1);
    o.vert_old.clear();
    o.vert_old.reserve(V);
    for (int i = 0; i < E; ++i) {
        const int e = o.edge_old[i];
        for (int k = 0; k < 2; ++k) {
            const int v = d->vertices_on_edge[2 * (size_t)e + k];
            if (v >= 0 && o.vert_new[v] < 0) {
                o.vert_new[v] = (int)o.vert_old.size();
                o.vert_old.push_back(v);
            }
        }
    }
    for (int v = 0; v < V; ++v)
        if (o.vert_new[v] < 0) {
            o.vert_new[v] = (int)o.vert_old.size();
            o.vert_old.push_back(v);
        }
}

void permute_desc(const sse_mesh_desc *d, const MeshOrder &o, PermutedDesc &p) {
    const int C = d->n_cells, E = d->n_edges, V = d->n_vertices, me = d->max_edges, me2 = d->max_edges2;
    auto map = [](const std::vector<int32_t> &nw, int x) { return x < 0 ? x : nw[x]; };
    p.coe.resize((size_t)E * 2);
    p.voe.resize((size_t)E * 2);
    p.eoe.resize((size_t)E * me2);
    p.neoe.resize(E);
    p.w.resize((size_t)E * me2);
    p.dc.resize(E);
    p.dv.resize(E);
    p.f.resize(E);
    for (int i = 0; i < E; ++i) {
        const int e = o.edge_old[i];
        for (int k = 0; k < 2; ++k) {
            p.coe[2 * (size_t)i + k] = map(o.cell_new, d->cells_on_edge[2 * (size_t)e + k]);
            p.voe[2 * (size_t)i + k] = map(o.vert_new, d->vertices_on_edge[2 * (size_t)e + k]);
        }
        for (int j = 0; j < me2; ++j) {
            p.eoe[(size_t)i * me2 + j] = map(o.edge_new, d->edges_on_edge[(size_t)e * me2 + j]);
            p.w[(size_t)i * me2 + j] = d->weights_on_edge[(size_t)e * me2 + j];
        }
        p.neoe[i] = d->n_edges_on_edge[e];
        p.dc[i] = d->dc_edge[e];
        p.dv[i] = d->dv_edge[e];
        p.f[i] = d->f_edge[e];
    }
    p.eoc.resize((size_t)C * me);
    p.neoc.resize(C);
    p.area.resize(C);
    p.H.resize(C);
    p.mask.resize(C);
    for (int i = 0; i < C; ++i) {
        const int c = o.cell_old[i];
        for (int j = 0; j < me; ++j) p.eoc[(size_t)i * me + j] = map(o.edge_new, d->edges_on_cell[(size_t)c * me + j]);
        p.neoc[i] = d->n_edges_on_cell[c];
        p.area[i] = d->area_cell[c];
        p.H[i] = d->bottom_depth[c];
        p.mask[i] = d->cell_mask ? d->cell_mask[c] : 1;
    }
    p.eov.resize((size_t)V * 3);
    p.tri.resize(V);
    for (int i = 0; i < V; ++i) {
        const int v = o.vert_old[i];
        for (int k = 0; k < 3; ++k) p.eov[(size_t)i * 3 + k] = map(o.edge_new, d->edges_on_vertex[(size_t)v * 3 + k]);
        p.tri[i] = d->area_triangle[v];
    }
    p.d = *d;
    p.d.cells_on_edge = p.coe.data();
    p.d.edges_on_cell = p.eoc.data();
    p.d.n_edges_on_cell = p.neoc.data();
    p.d.vertices_on_edge = p.voe.data();
    p.d.edges_on_vertex = p.eov.data();
    p.d.edges_on_edge = p.eoe.data();
    p.d.n_edges_on_edge = p.neoe.data();
    p.d.weights_on_edge = p.w.data();
    p.d.dc_edge = p.dc.data();
    p.d.dv_edge = p.dv.data();
    p.d.f_edge = p.f.data();
    p.d.area_cell = p.area.data();
    p.d.bottom_depth = p.H.data();
    p.d.area_triangle = p.tri.data();
    p.d.cell_mask = p.mask.data();
}


// ---------------------------------------------------------------------------
// Canonical two-cell stencils
//
// On a TRiSK C-grid the tangential reconstruction at edge e combines the
// other edges of its two cells (Thuburn et al. 2009).  Listed in the order of
// the cells' own counter-clockwise edge lists, starting after e, the stencil
// edges of one cell follow the chain of the cell's vertices: stencil edge k
// of cell c1 joins chain vertices A_k and A_{k+1} (A_0 and A_5 are the end
// points of e; a pentagon repeats A_4), and on c2 the chain runs
// A_5, B_0 .. B_3, A_0 back (a pentagon repeats A_0 as B_3).  The edge pass
// then needs the vorticity of these 10 vertices instead of 2 per stencil
// edge.  Slots: 0-4 the edges of c1, 5-9 those of c2 (unused: -1, weight 0).
// ---------------------------------------------------------------------------
bool canonical_stencils(PermutedDesc &p, std::vector<int32_t> &chain) {
    const sse_mesh_desc &d = p.d;
    const int E = d.n_edges, me = d.max_edges, me2 = d.max_edges2;
    if (me2 != 10 || me > 6) return false;
    auto common_vertex = [&](int ea, int eb) -> int {
        const int a0 = d.vertices_on_edge[2 * (size_t)ea], a1 = d.vertices_on_edge[2 * (size_t)ea + 1];
        const int b0 = d.vertices_on_edge[2 * (size_t)eb], b1 = d.vertices_on_edge[2 * (size_t)eb + 1];
        if (a0 >= 0 && (a0 == b0 || a0 == b1)) return a0;
        if (a1 >= 0 && (a1 == b0 || a1 == b1)) return a1;
        return -1;
    };
    std::vector<int32_t> eoe((size_t)E * 10, -1), ch((size_t)E * kChainWords, 0);
    std::vector<double> w((size_t)E * 10, 0.0);
    for (int e = 0; e < E; ++e) {
        int cv[2][6], slot[2][5], n[2];
        for (int s = 0; s < 2; ++s) {
            const int c = d.cells_on_edge[2 * (size_t)e + s];
            if (c < 0) return false;
            n[s] = d.n_edges_on_cell[c];
            if (n[s] < 5 || n[s] > 6) return false;
            const int32_t *ec = d.edges_on_cell + (size_t)c * me;
            int m = -1;
            for (int j = 0; j < n[s]; ++j)
                if (ec[j] == e) m = j;
            if (m < 0) return false;
            for (int k = 0; k < n[s]; ++k) {
                cv[s][k] = common_vertex(ec[(m + k) % n[s]], ec[(m + k + 1) % n[s]]);
                if (cv[s][k] < 0) return false;
            }
            if (n[s] == 5) cv[s][5] = cv[s][4];
            for (int k = 0; k < 5; ++k) slot[s][k] = k < n[s] - 1 ? ec[(m + 1 + k) % n[s]] : -1;
        }
        const int first = cv[0][0], last = cv[0][n[0] - 1];
        if (cv[1][0] != last || cv[1][n[1] - 1] != first) return false;
        const int v1 = d.vertices_on_edge[2 * (size_t)e], v2 = d.vertices_on_edge[2 * (size_t)e + 1];
        if (!((first == v1 && last == v2) || (first == v2 && last == v1))) return false;
        // weights of the canonical slots from the caller's row; every entry of
        // the caller's row with a nonzero weight must be one of them
        const int nr = d.n_edges_on_edge[e];
        const int32_t *ue = d.edges_on_edge + (size_t)e * me2;
        const double *uw = d.weights_on_edge + (size_t)e * me2;
        int used = 0;
        for (int s = 0; s < 2; ++s)
            for (int k = 0; k < 5; ++k) {
                const int ep = slot[s][k];
                const size_t o = (size_t)e * 10 + s * 5 + k;
                if (ep < 0) continue;
                int jj = -1;
                for (int j = 0; j < nr; ++j)
                    if (ue[j] == ep) jj = j;
                if (jj < 0) return false;
                eoe[o] = ep;
                w[o] = uw[jj];
                ++used;
            }
        for (int j = 0; j < nr; ++j) {
            if (ue[j] < 0 || uw[j] == 0.0) continue;
            bool found = false;
            for (int q = 0; q < 10; ++q) found |= eoe[(size_t)e * 10 + q] == ue[j];
            if (!found) return false;
        }
        (void)used;
        int32_t *r = &ch[(size_t)e * kChainWords];
        for (int k = 0; k < 5; ++k) r[k] = cv[0][k];
        r[5] = last;
        for (int k = 0; k < 4; ++k) r[6 + k] = k + 1 < n[1] - 1 ? cv[1][k + 1] : first;
        r[10] = first == v1 ? 1 : 0;
    }
    p.eoe.swap(eoe);
    p.w.swap(w);
    for (int e = 0; e < E; ++e) p.neoe[e] = 10;
    p.d.edges_on_edge = p.eoe.data();
    p.d.weights_on_edge = p.w.data();
    p.d.n_edges_on_edge = p.neoe.data();
    chain.swap(ch);
    return true;
}

// ---------------------------------------------------------------------------
// Patches of the tiled barotropic substeps
// ---------------------------------------------------------------------------
namespace {

// Cells adjacent to c across its edges.
template <typename F>
void for_each_neighbour(const sse_mesh_desc *d, int c, F &&f) {
    const int me = d->max_edges;
    for (int j = 0; j < d->n_edges_on_cell[c]; ++j) {
        const int e = d->edges_on_cell[(size_t)c * me + j];
        if (e < 0) continue;
        const int a = d->cells_on_edge[2 * (size_t)e], b = d->cells_on_edge[2 * (size_t)e + 1];
        const int nb = a == c ? b : a;
        if (nb >= 0 && nb != c) f(nb);
    }
}

// Region of one patch: cells and edges by level (see DevBtTiles).  Stamps
// mark membership without clearing between patches; loc holds the local
// index of every member.
struct RegionBuilder {
    const sse_mesh_desc *d;
    std::vector<int32_t> cst, est, cloc, eloc;
    int stamp = 0;
    std::vector<int32_t> cells, edges;
    int nc[4] = {}, ne[4] = {};

    explicit RegionBuilder(const sse_mesh_desc *d_)
        : d(d_), cst(d_->n_cells, 0), est(d_->n_edges, 0), cloc(d_->n_cells, -1), eloc(d_->n_edges, -1) {}

    void add_cell(int c) { cst[c] = stamp; cloc[c] = (int)cells.size(); cells.push_back(c); }
    void add_edge(int e) { est[e] = stamp; eloc[e] = (int)edges.size(); edges.push_back(e); }

    // own: the patch's cells; pid/p decide edge ownership (first cell).
    void build(const std::vector<int32_t> &own, const std::vector<int32_t> &pid, int p) {
        ++stamp;
        cells.clear();
        edges.clear();
        std::vector<int32_t> lvl(own);
        std::sort(lvl.begin(), lvl.end());
        for (int c : lvl) add_cell(c);
        nc[0] = (int)cells.size();
        const int me = d->max_edges;
        // level-0 edges: owned (first cell in the patch)
        std::vector<int32_t> tmp;
        for (int c : own)
            for (int j = 0; j < d->n_edges_on_cell[c]; ++j) {
                const int e = d->edges_on_cell[(size_t)c * me + j];
                if (e >= 0 && pid[d->cells_on_edge[2 * (size_t)e]] == p) tmp.push_back(e);
            }
        std::sort(tmp.begin(), tmp.end());
        tmp.erase(std::unique(tmp.begin(), tmp.end()), tmp.end());
        for (int e : tmp) add_edge(e);
        ne[0] = (int)edges.size();
        for (int k = 1; k <= 3; ++k) {
            tmp.clear();
            for (int i = 0; i < nc[k - 1]; ++i)
                for_each_neighbour(d, cells[i], [&](int nb) {
                    if (cst[nb] != stamp) { cst[nb] = stamp; tmp.push_back(nb); }
                });
            std::sort(tmp.begin(), tmp.end());
            for (int c : tmp) { cst[c] = 0; add_cell(c); }
            nc[k] = (int)cells.size();
            // edges of level k: every edge of R_k not listed yet
            tmp.clear();
            for (int i = 0; i < nc[k]; ++i) {
                const int c = cells[i];
                for (int j = 0; j < d->n_edges_on_cell[c]; ++j) {
                    const int e = d->edges_on_cell[(size_t)c * me + j];
                    if (e >= 0 && est[e] != stamp) { est[e] = stamp; tmp.push_back(e); }
                }
            }
            std::sort(tmp.begin(), tmp.end());
            for (int e : tmp) { est[e] = 0; add_edge(e); }
            ne[k] = (int)edges.size();
        }
    }
    bool fits() const {
        return ne[2] <= kBtEdgeSlots * kBtThreads && nc[2] <= kBtThreads && nc[3] < (1 << 15) && ne[3] < (1 << 16);
    }
};

template <typename R>
size_t bt_lds_bytes(const int (&ne)[4], const int (&nc)[4]) {
    // U0, U1, U2, Z0, Z1, Z2 (R), H (double), and H in R for FP32 state
    size_t b = sizeof(R) * ((size_t)ne[3] + ne[2] + ne[1] + nc[3] + nc[2] + nc[1]) + 8 * (size_t)nc[3];
    if (sizeof(R) != 8) b += sizeof(R) * (size_t)nc[3];
    return b;
}

constexpr size_t kBtLdsMax = 160 * 1024;

}  // namespace

bool bt_partition(const sse_mesh_desc *d, std::vector<int32_t> &pid, int &nP) {
    const int C = d->n_cells;
    pid.assign(C, -1);
    std::vector<std::vector<int32_t>> patches;
    // breadth-first patches, seeded from the previous patches' frontier
    std::vector<char> taken(C, 0);
    std::deque<int> front, q;
    int scan = 0, done = 0;
    while (done < C) {
        int seed = -1;
        while (!front.empty()) {
            const int c = front.front();
            front.pop_front();
            if (!taken[c]) { seed = c; break; }
        }
        if (seed < 0) {
            while (taken[scan]) ++scan;
            seed = scan;
        }
        std::vector<int32_t> cells;
        q.clear();
        q.push_back(seed);
        taken[seed] = 1;
        while (!q.empty()) {
            const int c = q.front();
            q.pop_front();
            cells.push_back(c);
            for_each_neighbour(d, c, [&](int nb) {
                if (taken[nb]) return;
                if ((int)(cells.size() + q.size()) < kBtPatch) {
                    taken[nb] = 1;
                    q.push_back(nb);
                } else {
                    front.push_back(nb);
                }
            });
        }
        done += (int)cells.size();
        for (int c : cells) pid[c] = (int)patches.size();
        patches.push_back(std::move(cells));
    }
    // split patches whose region does not fit, in their breadth-first order
    RegionBuilder rb(d);
    for (size_t p = 0; p < patches.size(); ++p) {
        for (;;) {
            rb.build(patches[p], pid, (int)p);
            if (rb.fits() && bt_lds_bytes<double>(rb.ne, rb.nc) <= kBtLdsMax) break;
            if (patches[p].size() < 2) return false;
            const size_t half = patches[p].size() / 2;
            std::vector<int32_t> tail(patches[p].begin() + half, patches[p].end());
            patches[p].resize(half);
            for (int c : tail) pid[c] = (int)patches.size();
            patches.push_back(std::move(tail));
        }
    }
    nP = (int)patches.size();
    return true;
}

bool build_bt_tiles(const sse_mesh_desc *d, const std::vector<int32_t> &pid, int nP, const HostMeshTables *t,
                    HostBtTiles &bt) {
    const int C = d->n_cells, E = d->n_edges;
    std::vector<std::vector<int32_t>> own(nP);
    for (int c = 0; c < C; ++c) own[pid[c]].push_back(c);
    RegionBuilder rb(d);
    bt = HostBtTiles();
    bt.nP = nP;
    bt.patch.assign((size_t)nP * kBtRec, 0);
    int e0 = 0, es0 = 0, c0 = 0, cs0 = 0, max_ne2 = 0;
    for (int p = 0; p < nP; ++p) {
        rb.build(own[p], pid, p);
        if (!rb.fits()) return false;
        int32_t *r = &bt.patch[(size_t)p * kBtRec];
        r[0] = e0; r[1] = es0; r[2] = c0; r[3] = cs0;
        for (int k = 0; k < 4; ++k) { r[4 + k] = rb.ne[k]; r[8 + k] = rb.nc[k]; }
        max_ne2 = std::max(max_ne2, rb.ne[2]);
        bt.lds_d = std::max(bt.lds_d, bt_lds_bytes<double>(rb.ne, rb.nc));
        bt.lds_f = std::max(bt.lds_f, bt_lds_bytes<float>(rb.ne, rb.nc));
        if (t) {
            const int ne2 = rb.ne[2], nc2 = rb.nc[2];
            bt.eid.insert(bt.eid.end(), rb.edges.begin(), rb.edges.end());
            bt.cid.insert(bt.cid.end(), rb.cells.begin(), rb.cells.end());
            for (int c : rb.cells) { bt.cH.push_back(t->H[c]); bt.cH_f.push_back(t->H_f[c]); }
            const size_t b = bt.ec.size();
            bt.ec.resize(b + ne2);
            bt.eidc.resize(b + ne2);
            bt.eidc_f.resize(b + ne2);
            bt.enb.resize(5 * (b + ne2));
            bt.ew.resize(10 * (b + ne2));
            bt.ew_f.resize(10 * (b + ne2));
            auto in_c = [&](int c) { return c >= 0 && rb.cst[c] == rb.stamp; };
            auto in_e = [&](int e) { return e >= 0 && rb.est[e] == rb.stamp; };
            for (int le = 0; le < ne2; ++le) {
                const int e = rb.edges[le];
                const int g1 = t->edge_cells[2 * (size_t)e], g2 = t->edge_cells[2 * (size_t)e + 1];
                if (!in_c(g1) || !in_c(g2)) return false;
                const int c1 = rb.cloc[g1], c2 = rb.cloc[g2];
                bt.ec[b + le] = (uint32_t)c1 | ((uint32_t)c2 << 15) | ((uint32_t)(t->emask[e] ? 1 : 0) << 30);
                bt.eidc[b + le] = t->inv_dc[e];
                bt.eidc_f[b + le] = t->inv_dc_f[e];
                uint32_t lj[10];
                for (int j = 0; j < 10; ++j) {
                    const int ep = t->eoe[(size_t)j * E + e];
                    if (!in_e(ep)) return false;  // a stencil reaching past the two cells
                    lj[j] = (uint32_t)rb.eloc[ep];
                    bt.ew[10 * b + (size_t)j * ne2 + le] = t->wf[(size_t)j * E + e];
                    bt.ew_f[10 * b + (size_t)j * ne2 + le] = t->wf_f[(size_t)j * E + e];
                }
                for (int i = 0; i < 5; ++i) bt.enb[5 * b + (size_t)i * ne2 + le] = lj[2 * i] | (lj[2 * i + 1] << 16);
            }
            const size_t cb = bt.cwet.size();
            bt.cwet.resize(cb + nc2);
            bt.cen.resize(6 * (cb + nc2));
            bt.ccd.resize(6 * (cb + nc2));
            bt.ccd_f.resize(6 * (cb + nc2));
            for (int lc = 0; lc < nc2; ++lc) {
                const int i = rb.cells[lc];
                bt.cwet[cb + lc] = t->cmask[i] ? 1 : 0;
                for (int j = 0; j < 6; ++j) {
                    const int e = t->cell_edges_t[(size_t)j * C + i], nb = t->cell_nbrs_t[(size_t)j * C + i];
                    if (!in_e(e) || !in_c(nb)) return false;
                    bt.cen[6 * cb + (size_t)j * nc2 + lc] = (uint32_t)rb.eloc[e] | ((uint32_t)rb.cloc[nb] << 16);
                    bt.ccd[6 * cb + (size_t)j * nc2 + lc] = t->cell_div_t[(size_t)j * C + i];
                    bt.ccd_f[6 * cb + (size_t)j * nc2 + lc] = t->cell_div_t_f[(size_t)j * C + i];
                }
            }
        }
        e0 += rb.ne[3];
        es0 += rb.ne[2];
        c0 += rb.nc[3];
        cs0 += rb.nc[2];
    }
    bt.ks = (max_ne2 + kBtThreads - 1) / kBtThreads;
    if (!t) {
        // sizes only
        bt.eid.resize(e0);
        bt.cid.resize(c0);
        bt.ec.resize(es0);
        bt.cwet.resize(cs0);
    }
    return bt.ks >= 1 && bt.ks <= kBtEdgeSlots;
}

namespace {

// The partition depends on the cell-edge topology only; meshes that share it
// (every request on the same icosahedral level, the size query before the
// creation of a mesh) reuse it from a small cache keyed by a hash of the
// topology tables.
uint64_t topology_hash(const sse_mesh_desc *d) {
    uint64_t h = 1469598103934665603ull;
    auto mix = [&](const void *p, size_t n) {
        const unsigned char *b = static_cast<const unsigned char *>(p);
        for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
    };
    const int32_t cnt[5] = {d->n_cells, d->n_edges, d->n_vertices, d->max_edges, d->max_edges2};
    mix(cnt, sizeof(cnt));
    mix(d->cells_on_edge, 2 * (size_t)d->n_edges * 4);
    mix(d->edges_on_cell, (size_t)d->n_cells * d->max_edges * 4);
    mix(d->n_edges_on_cell, (size_t)d->n_cells * 4);
    return h;
}

struct PartitionEntry {
    uint64_t key;
    bool ok;
    int nP;
    std::vector<int32_t> pid;
    size_t bytes;
};
std::mutex g_part_mu;
std::deque<PartitionEntry> g_part_cache;  // most recent first
constexpr size_t kPartCache = 8;

size_t bt_bytes_of(const HostBtTiles &bt) {
    auto al = [](size_t x) { return (x + kAlign - 1) / kAlign * kAlign; };
    const size_t TE = bt.eid.size(), TC = bt.cid.size(), SE = bt.ec.size(), SC = bt.cwet.size();
    return al(bt.patch.size() * 4) + al(TE * 4) + al(TC * 4) + al(TC * 8) + al(TC * 4) + al(SE * 4) +
           al(SE * 5 * 4) + al(SE * 10 * 8) + al(SE * 10 * 4) + al(SE * 8) + al(SE * 4) + al(SC * 6 * 4) +
           al(SC * 6 * 8) + al(SC * 6 * 4) + al(SC);
}

// Partition of d with its table bytes (0 if d cannot be tiled), cached.
PartitionEntry cached_partition(const sse_mesh_desc *d) {
    const uint64_t key = topology_hash(d);
    {
        std::lock_guard<std::mutex> g(g_part_mu);
        for (auto it = g_part_cache.begin(); it != g_part_cache.end(); ++it)
            if (it->key == key) {
                PartitionEntry e = *it;
                g_part_cache.erase(it);
                g_part_cache.push_front(e);
                return e;
            }
    }
    PartitionEntry e{key, false, 0, {}, 0};
    if (bt_partition(d, e.pid, e.nP)) {
        HostBtTiles bt;
        if (build_bt_tiles(d, e.pid, e.nP, nullptr, bt)) {
            e.ok = true;
            e.bytes = bt_bytes_of(bt);
        }
    }
    std::lock_guard<std::mutex> g(g_part_mu);
    g_part_cache.push_front(e);
    if (g_part_cache.size() > kPartCache) g_part_cache.pop_back();
    return e;
}

}  // namespace

size_t bt_tiles_bytes(const sse_mesh_desc *d) { return cached_partition(d).bytes; }

bool bt_cached_partition(const sse_mesh_desc *d, std::vector<int32_t> &pid, int &nP) {
    PartitionEntry e = cached_partition(d);
    if (!e.ok) return false;
    pid.swap(e.pid);
    nP = e.nP;
    return true;
}

int check_topology(const sse_mesh_desc *d, std::string &err) {
    if (!d) { err = "mesh description is NULL"; return SSE_EINVAL; }
    const int C = d->n_cells, E = d->n_edges;
    if (C <= 0 || E <= 0 || d->n_vertices <= 0) { err = "mesh counts must be positive"; return SSE_EINVAL; }
    if (d->max_edges < 1 || d->max_edges > 6 || d->max_edges2 < 1 || d->max_edges2 > 10) {
        err = "max_edges must be in [1, 6] and max_edges2 in [1, 10]";
        return SSE_EINVAL;
    }
    if (!d->cells_on_edge || !d->edges_on_cell || !d->n_edges_on_cell) { err = "topology tables are NULL"; return SSE_EINVAL; }
    for (size_t i = 0; i < 2 * (size_t)E; ++i)
        if (d->cells_on_edge[i] < 0 || d->cells_on_edge[i] >= C) { err = "cells_on_edge out of range"; return SSE_EINVAL; }
    for (int c = 0; c < C; ++c) {
        const int n = d->n_edges_on_cell[c];
        if (n < 1 || n > d->max_edges) { err = "n_edges_on_cell out of range"; return SSE_EINVAL; }
        for (int j = 0; j < n; ++j) {
            const int e = d->edges_on_cell[(size_t)c * d->max_edges + j];
            if (e < -1 || e >= E) { err = "edges_on_cell out of range"; return SSE_EINVAL; }
        }
    }
    return SSE_OK;
}

}  // namespace sse

extern "C" int sse_mesh_validate(const sse_mesh_desc *d) {
    std::string err;
    int rc = sse::validate_desc(d, err);
    if (rc != SSE_OK) sse::set_error(err);
    return rc;
}

extern "C" int sse_mesh_device_bytes(const sse_mesh_desc *d, size_t *bytes) {
    if (!d || !bytes) { sse::set_error("NULL argument"); return SSE_EINVAL; }
    std::string err;
    const int rc = sse::check_topology(d, err);
    if (rc != SSE_OK) { sse::set_error(err); return rc; }
    *bytes = sse::mesh_layout(d->n_cells, d->n_edges, d->n_vertices).total;
    for (int q = 0; q < sse::kTileVariants; ++q) *bytes += sse::tiles_bytes(d, sse::kTileSizes[q]);
    *bytes += sse::bt_tiles_bytes(d);
    *bytes += sse::wpair_f_bytes(d);
    return SSE_OK;
}
