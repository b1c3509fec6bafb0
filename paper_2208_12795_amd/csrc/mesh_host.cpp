// Host-side canonicalisation of a tet mesh for the etpic library: the sets of
// edges and faces with their global numbering, the tet -> edge / face /
// neighbour incidences, the barycentric gradients of every tet, and the
// vertex -> edge incidence used by the continuity residual.
#include <climits>
#include "mesh_host.hpp"

#include <algorithm>
#include <cmath>
#include <cstdio>

namespace etpic {

namespace {

inline int64_t edge_key(int64_t nv, int64_t a, int64_t b) { return a * nv + b; }
inline int64_t face_key(int64_t nv, int64_t a, int64_t b, int64_t c) { return (a * nv + b) * nv + c; }

int64_t index_of(const std::vector<int64_t> &sorted, int64_t key) {
    auto it = std::lower_bound(sorted.begin(), sorted.end(), key);
    if (it == sorted.end() || *it != key) return -1;
    return it - sorted.begin();
}

}  // namespace

int build_host_mesh(int64_t nv, const double *xyz, int64_t nt, const int32_t *tv, HostMesh &M, std::string &err) {
    if (nv <= 0 || nt <= 0 || !xyz || !tv) { err = "empty mesh or null pointer"; return -1; }
    if (nv > (int64_t)2000000 || nt > (int64_t)INT32_MAX / 8) { err = "mesh too large for 32-bit tables"; return -1; }
    M = HostMesh();
    M.nv = nv;
    M.nt = nt;
    M.grad.resize((size_t)nt * 12);
    M.vol.resize((size_t)nt);
    // validation + barycentric gradients: with columns c_k = r_k - r_0 (k = 1..3)
    // and J = [c1 c2 c3], (lam1, lam2, lam3) = J^{-1} (x - r0), so the gradients
    // are the rows of J^{-1} = [c2 x c3; c3 x c1; c1 x c2] / det J.
    for (int64_t t = 0; t < nt; ++t) {
        const int32_t *v = tv + 4 * t;
        for (int k = 0; k < 4; ++k) {
            if (v[k] < 0 || v[k] >= nv) { err = "tet " + std::to_string(t) + ": vertex id out of range"; return -1; }
            if (k > 0 && v[k] <= v[k - 1]) { err = "tet " + std::to_string(t) + ": vertex ids not ascending"; return -4; }
        }
        double c[3][3];
        for (int k = 0; k < 3; ++k)
            for (int d = 0; d < 3; ++d) c[k][d] = xyz[3 * v[k + 1] + d] - xyz[3 * v[0] + d];
        auto cross = [](const double *a, const double *b, double *o) {
            o[0] = a[1] * b[2] - a[2] * b[1];
            o[1] = a[2] * b[0] - a[0] * b[2];
            o[2] = a[0] * b[1] - a[1] * b[0];
        };
        double r1[3], r2[3], r3[3];
        cross(c[1], c[2], r1);
        cross(c[2], c[0], r2);
        cross(c[0], c[1], r3);
        double det = c[0][0] * r1[0] + c[0][1] * r1[1] + c[0][2] * r1[2];
        double l0 = std::sqrt(c[0][0] * c[0][0] + c[0][1] * c[0][1] + c[0][2] * c[0][2]);
        double l1 = std::sqrt(c[1][0] * c[1][0] + c[1][1] * c[1][1] + c[1][2] * c[1][2]);
        double l2 = std::sqrt(c[2][0] * c[2][0] + c[2][1] * c[2][1] + c[2][2] * c[2][2]);
        if (!(std::fabs(det) > 1e-12 * l0 * l1 * l2)) { err = "tet " + std::to_string(t) + ": degenerate"; return -4; }
        M.vol[t] = std::fabs(det) / 6.0;
        double *g = &M.grad[(size_t)t * 12];
        for (int d = 0; d < 3; ++d) {
            g[3 + d] = r1[d] / det;
            g[6 + d] = r2[d] / det;
            g[9 + d] = r3[d] / det;
            g[d] = -(g[3 + d] + g[6 + d] + g[9 + d]);
        }
    }
    // edges
    std::vector<int64_t> ek((size_t)nt * 6);
    for (int64_t t = 0; t < nt; ++t)
        for (int e = 0; e < 6; ++e) ek[6 * t + e] = edge_key(nv, tv[4 * t + kLocalEdge[e][0]], tv[4 * t + kLocalEdge[e][1]]);
    std::sort(ek.begin(), ek.end());
    ek.erase(std::unique(ek.begin(), ek.end()), ek.end());
    M.ne = (int64_t)ek.size();
    M.edges.resize((size_t)M.ne * 2);
    for (int64_t i = 0; i < M.ne; ++i) {
        M.edges[2 * i] = (int32_t)(ek[i] / nv);
        M.edges[2 * i + 1] = (int32_t)(ek[i] % nv);
    }
    // faces
    std::vector<int64_t> fk((size_t)nt * 4);
    for (int64_t t = 0; t < nt; ++t)
        for (int f = 0; f < 4; ++f)
            fk[4 * t + f] = face_key(nv, tv[4 * t + kLocalFace[f][0]], tv[4 * t + kLocalFace[f][1]], tv[4 * t + kLocalFace[f][2]]);
    std::vector<int64_t> fs(fk);
    std::sort(fs.begin(), fs.end());
    fs.erase(std::unique(fs.begin(), fs.end()), fs.end());
    M.nf = (int64_t)fs.size();
    M.faces.resize((size_t)M.nf * 3);
    for (int64_t i = 0; i < M.nf; ++i) {
        int64_t k = fs[i];
        M.faces[3 * i + 2] = (int32_t)(k % nv);
        k /= nv;
        M.faces[3 * i + 1] = (int32_t)(k % nv);
        M.faces[3 * i] = (int32_t)(k / nv);
    }
    // tet records and neighbours (each face has one or two owning tets)
    M.topo.assign((size_t)nt, TetTopo{});
    std::vector<int64_t> own0((size_t)M.nf, -1), own1((size_t)M.nf, -1);
    for (int64_t t = 0; t < nt; ++t) {
        TetTopo &r = M.topo[t];
        for (int k = 0; k < 4; ++k) r.v[k] = tv[4 * t + k];
        for (int e = 0; e < 6; ++e)
            r.e[e] = (int32_t)index_of(ek, edge_key(nv, tv[4 * t + kLocalEdge[e][0]], tv[4 * t + kLocalEdge[e][1]]));
        for (int f = 0; f < 4; ++f) {
            int64_t id = index_of(fs, fk[4 * t + f]);
            r.f[f] = (int32_t)id;
            if (own0[id] < 0) own0[id] = t;
            else if (own1[id] < 0) own1[id] = t;
            else { err = "face shared by more than two tets (tet " + std::to_string(t) + ")"; return -4; }
        }
        r.pad[0] = r.pad[1] = 0;
    }
    for (int64_t t = 0; t < nt; ++t) {
        TetTopo &r = M.topo[t];
        for (int f = 0; f < 4; ++f) {
            int64_t id = r.f[f];
            r.n[f] = (int32_t)(own0[id] == t ? own1[id] : own0[id]);
        }
    }
    // vertex -> incident edges (CSR), sign carried in the low bit (1 = head)
    M.v2e_ptr.assign((size_t)nv + 1, 0);
    for (int64_t e = 0; e < M.ne; ++e) {
        M.v2e_ptr[M.edges[2 * e] + 1]++;
        M.v2e_ptr[M.edges[2 * e + 1] + 1]++;
    }
    for (int64_t k = 0; k < nv; ++k) M.v2e_ptr[k + 1] += M.v2e_ptr[k];
    M.v2e_code.resize((size_t)M.ne * 2);
    std::vector<int32_t> fill(M.v2e_ptr.begin(), M.v2e_ptr.end() - 1);
    for (int64_t e = 0; e < M.ne; ++e) {
        M.v2e_code[fill[M.edges[2 * e]]++] = (int32_t)(e << 1);
        M.v2e_code[fill[M.edges[2 * e + 1]]++] = (int32_t)((e << 1) | 1);
    }
    // edge -> the (tet, local edge) slots that name it, slot = 8 * tet + local
    // edge, in increasing tet order
    if (nt > (int64_t)(INT32_MAX / 8)) {
        err = "more than 2^28 tets";
        return -1;
    }
    M.e2s_ptr.assign((size_t)M.ne + 1, 0);
    for (int64_t t = 0; t < nt; ++t)
        for (int k = 0; k < 6; ++k) M.e2s_ptr[M.topo[t].e[k] + 1]++;
    for (int64_t e = 0; e < M.ne; ++e) M.e2s_ptr[e + 1] += M.e2s_ptr[e];
    M.e2s_slot.resize((size_t)nt * 6);
    std::vector<int32_t> efill(M.e2s_ptr.begin(), M.e2s_ptr.end() - 1);
    for (int64_t t = 0; t < nt; ++t)
        for (int k = 0; k < 6; ++k) M.e2s_slot[efill[M.topo[t].e[k]]++] = (int32_t)(8 * t + k);
    return 0;
}

void build_start_grid(const HostMesh &m, const double *xyz, double tets_per_cell, StartGrid &g) {
    double lo[3] = {xyz[0], xyz[1], xyz[2]}, hi[3] = {xyz[0], xyz[1], xyz[2]};
    for (int64_t i = 1; i < m.nv; ++i)
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::min(lo[d], xyz[3 * i + d]);
            hi[d] = std::max(hi[d], xyz[3 * i + d]);
        }
    double ext[3], vol = 1.0;
    for (int d = 0; d < 3; ++d) {
        ext[d] = std::max(hi[d] - lo[d], 1e-300);
        vol *= ext[d];
    }
    const double cells = std::max(1.0, std::min((double)m.nt / tets_per_cell, (double)(1 << 24)));
    const double h = std::cbrt(vol / cells);
    int64_t total = 1;
    for (int d = 0; d < 3; ++d) {
        g.dims[d] = (int32_t)std::max(1.0, std::min(std::ceil(ext[d] / h), 4096.0));
        g.lo[d] = lo[d];
        g.inv[d] = g.dims[d] / ext[d];
        total *= g.dims[d];
    }
    g.cell.assign((size_t)total, -1);
    auto cell_of = [&](const double *x) {
        int64_t c[3];
        for (int d = 0; d < 3; ++d)
            c[d] = std::min<int64_t>(g.dims[d] - 1, std::max<int64_t>(0, (int64_t)std::floor((x[d] - g.lo[d]) * g.inv[d])));
        return c[0] + g.dims[0] * (c[1] + (int64_t)g.dims[1] * c[2]);
    };
    for (int64_t t = 0; t < m.nt; ++t) {
        double c[3] = {0, 0, 0};
        for (int k = 0; k < 4; ++k)
            for (int d = 0; d < 3; ++d) c[d] += 0.25 * xyz[3 * m.topo[t].v[k] + d];
        int32_t &slot = g.cell[(size_t)cell_of(c)];
        if (slot < 0) slot = (int32_t)t;
    }
    // cells without a centroid take a face-neighbour cell's tet, in passes
    const int64_t nx = g.dims[0], ny = g.dims[1], nz = g.dims[2];
    for (bool changed = true; changed;) {
        changed = false;
        std::vector<int32_t> prev(g.cell);
        for (int64_t k = 0; k < nz; ++k)
            for (int64_t j = 0; j < ny; ++j)
                for (int64_t i = 0; i < nx; ++i) {
                    const int64_t id = i + nx * (j + ny * k);
                    if (prev[id] >= 0) continue;
                    const int64_t nb[6][3] = {{i - 1, j, k}, {i + 1, j, k}, {i, j - 1, k},
                                              {i, j + 1, k}, {i, j, k - 1}, {i, j, k + 1}};
                    for (const auto &q : nb) {
                        if (q[0] < 0 || q[0] >= nx || q[1] < 0 || q[1] >= ny || q[2] < 0 || q[2] >= nz) continue;
                        const int32_t t = prev[q[0] + nx * (q[1] + ny * q[2])];
                        if (t >= 0) {
                            g.cell[id] = t;
                            changed = true;
                            break;
                        }
                    }
                }
    }
}

// Spanning tree of the vertex graph (breadth first from the lowest vertex of
// each component, incident edges in ascending id) and of the dual graph of
// tets plus one exterior node (every boundary face joins its tet to the
// exterior; tets reached first from the exterior in ascending id, then
// breadth first through interior faces).
void tree_cotree(const etpic::HostMesh &H, uint8_t *edge_tree, uint8_t *face_tree) {
    std::vector<uint8_t> seen((size_t)H.nv, 0);
    std::vector<int32_t> queue;
    queue.reserve((size_t)H.nv);
    std::fill(edge_tree, edge_tree + H.ne, (uint8_t)0);
    for (int32_t root = 0; root < (int32_t)H.nv; ++root) {
        if (seen[root]) continue;
        seen[root] = 1;
        queue.assign(1, root);
        for (size_t h = 0; h < queue.size(); ++h) {
            const int32_t u = queue[h];
            for (int32_t k = H.v2e_ptr[u]; k < H.v2e_ptr[u + 1]; ++k) {
                const int32_t e = H.v2e_code[k] >> 1;
                const int32_t w = (H.v2e_code[k] & 1) ? H.edges[2 * e] : H.edges[2 * e + 1];
                if (seen[w]) continue;
                seen[w] = 1;
                edge_tree[e] = 1;
                queue.push_back(w);
            }
        }
    }
    std::vector<uint8_t> tseen((size_t)H.nt, 0);
    std::fill(face_tree, face_tree + H.nf, (uint8_t)0);
    queue.clear();
    for (int64_t t = 0; t < H.nt; ++t)
        for (int k = 0; k < 4; ++k)
            if (H.topo[t].n[k] < 0) {
                tseen[t] = 1;
                face_tree[H.topo[t].f[k]] = 1;
                queue.push_back((int32_t)t);
                break;
            }
    for (size_t h = 0; h < queue.size(); ++h) {
        const etpic::TetTopo &tp = H.topo[queue[h]];
        for (int k = 0; k < 4; ++k) {
            const int32_t nb = tp.n[k];
            if (nb < 0 || tseen[nb]) continue;
            tseen[nb] = 1;
            face_tree[tp.f[k]] = 1;
            queue.push_back(nb);
        }
    }
}


}  // namespace etpic
