// Assembly of the Whitney edge mass and curl-curl matrices (field update).
//
// With barycentrics l_k (gradients g_k, constant in a tet of volume V):
//   int_T l_p l_r dV = V (1 + [p == r]) / 20,
//   W1_pq = l_p g_q - l_q g_p  =>  int W1_pq . W1_rs = I_pr g_q.g_s - I_ps g_q.g_r - I_qr g_p.g_s + I_qs g_p.g_r,
//   curl W1_pq = 2 g_p x g_q   =>  int curl W1_pq . curl W1_rs = 4 V (g_p x g_q).(g_r x g_s).
// Local edges keep the global orientation (tet vertices are in ascending id).
//
// The nodal operator of the non-solenoidal field is the linear-element
// stiffness: int grad l_p . grad l_r dV = V g_p . g_r.
#include "field_host.hpp"

#include <algorithm>
#include <cmath>

namespace etpic {

namespace {

struct Entry {
    int64_t key;
    double m, k;
};

inline double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
inline void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}

}  // namespace

int build_field_system(const HostMesh &mesh, double eps, double mu, FieldSystem &S, std::string &err,
                       bool dirichlet) {
    if (!(eps > 0.0) || !(mu > 0.0)) {
        err = "eps and mu must be positive";
        return -1;
    }
    const int64_t ne = mesh.ne, nt = mesh.nt, nf = mesh.nf, nv = mesh.nv;
    S = FieldSystem();
    S.ne = ne;
    S.nf = nf;
    // boundary edges: the edges of faces owned by one tet
    S.dirichlet.assign((size_t)ne, 0);
    for (int64_t t = 0; t < nt; ++t) {
        const TetTopo &tp = mesh.topo[t];
        for (int f = 0; f < 4; ++f) {
            if (tp.n[f] >= 0) continue;
            for (int e = 0; e < 6; ++e) {
                const int i = kLocalEdge[e][0], j = kLocalEdge[e][1];
                if (i != f && j != f) S.dirichlet[tp.e[e]] = 1;   // edge on the face opposite vertex f
            }
        }
    }
    std::vector<Entry> ent;
    ent.reserve((size_t)nt * 36 + (size_t)ne);
    for (int64_t t = 0; t < nt; ++t) {
        const TetTopo &tp = mesh.topo[t];
        const double *g = &mesh.grad[(size_t)t * 12];
        const double V = mesh.vol[t];
        double gg[4][4], cr[6][3];
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b) gg[a][b] = dot3(g + 3 * a, g + 3 * b);
        for (int e = 0; e < 6; ++e) cross3(g + 3 * kLocalEdge[e][0], g + 3 * kLocalEdge[e][1], cr[e]);
        auto I = [V](int p, int r) { return V * (p == r ? 2.0 : 1.0) / 20.0; };
        for (int e = 0; e < 6; ++e) {
            const int p = kLocalEdge[e][0], q = kLocalEdge[e][1], ge = tp.e[e];
            if (dirichlet && S.dirichlet[ge]) continue;
            for (int f = 0; f < 6; ++f) {
                const int r = kLocalEdge[f][0], s = kLocalEdge[f][1], gf = tp.e[f];
                if (dirichlet && S.dirichlet[gf]) continue;
                const double m = I(p, r) * gg[q][s] - I(p, s) * gg[q][r] - I(q, r) * gg[p][s] + I(q, s) * gg[p][r];
                const double k = 4.0 * V * dot3(cr[e], cr[f]);
                ent.push_back({(int64_t)ge * ne + gf, eps * m, k / mu});
            }
        }
    }
    if (dirichlet)
        for (int64_t e = 0; e < ne; ++e)
            if (S.dirichlet[e]) ent.push_back({e * ne + e, 1.0, 0.0});
    std::sort(ent.begin(), ent.end(), [](const Entry &x, const Entry &y) { return x.key < y.key; });
    S.rowptr.assign((size_t)ne + 1, 0);
    for (size_t i = 0; i < ent.size();) {
        size_t j = i;
        double m = 0.0, k = 0.0;
        while (j < ent.size() && ent[j].key == ent[i].key) {
            m += ent[j].m;
            k += ent[j].k;
            ++j;
        }
        const int64_t row = ent[i].key / ne, c = ent[i].key % ne;
        S.col.push_back((int32_t)c);
        S.M.push_back(m);
        S.K.push_back(k);
        S.rowptr[row + 1]++;
        i = j;
    }
    for (int64_t r = 0; r < ne; ++r) S.rowptr[r + 1] += S.rowptr[r];
    S.nnz = (int64_t)S.col.size();
    // face -> edges (a,b), (b,c), (a,c)
    std::vector<int64_t> ekeys((size_t)ne);
    for (int64_t e = 0; e < ne; ++e) ekeys[e] = (int64_t)mesh.edges[2 * e] * nv + mesh.edges[2 * e + 1];
    auto find = [&](int64_t a, int64_t b) -> int32_t {
        auto it = std::lower_bound(ekeys.begin(), ekeys.end(), a * nv + b);
        return (int32_t)(it - ekeys.begin());
    };
    S.face_edge.resize((size_t)nf * 3);
    for (int64_t f = 0; f < nf; ++f) {
        const int64_t a = mesh.faces[3 * f], b = mesh.faces[3 * f + 1], c = mesh.faces[3 * f + 2];
        S.face_edge[3 * f] = find(a, b);
        S.face_edge[3 * f + 1] = find(b, c);
        S.face_edge[3 * f + 2] = find(a, c);
    }
    return 0;
}

int build_ns_system(const HostMesh &mesh, double eps, NsSystem &S, std::string &err) {
    if (!(eps > 0.0)) {
        err = "eps must be positive";
        return -1;
    }
    const int64_t nt = mesh.nt, nv = mesh.nv;
    S = NsSystem();
    S.nv = nv;
    S.wall.assign((size_t)nv, 0);
    for (int64_t t = 0; t < nt; ++t) {
        const TetTopo &tp = mesh.topo[t];
        for (int f = 0; f < 4; ++f) {
            if (tp.n[f] >= 0) continue;
            for (int k = 0; k < 4; ++k)
                if (k != f) S.wall[tp.v[k]] = 1;
        }
    }
    struct NEntry {
        int64_t key;
        double s;
    };
    std::vector<NEntry> ent;
    ent.reserve((size_t)nt * 16 + (size_t)nv);
    for (int64_t t = 0; t < nt; ++t) {
        const TetTopo &tp = mesh.topo[t];
        const double *g = &mesh.grad[(size_t)t * 12];
        const double V = mesh.vol[t];
        for (int a = 0; a < 4; ++a) {
            const int32_t i = tp.v[a];
            if (S.wall[i]) continue;
            for (int b = 0; b < 4; ++b) {
                const int32_t j = tp.v[b];
                if (S.wall[j]) continue;
                ent.push_back({(int64_t)i * nv + j, eps * V * dot3(g + 3 * a, g + 3 * b)});
            }
        }
    }
    for (int64_t i = 0; i < nv; ++i)
        if (S.wall[i]) ent.push_back({i * nv + i, 1.0});
    std::sort(ent.begin(), ent.end(), [](const NEntry &x, const NEntry &y) { return x.key < y.key; });
    S.rowptr.assign((size_t)nv + 1, 0);
    for (size_t i = 0; i < ent.size();) {
        size_t j = i;
        double s = 0.0;
        while (j < ent.size() && ent[j].key == ent[i].key) s += ent[j++].s;
        S.col.push_back((int32_t)(ent[i].key % nv));
        S.S.push_back(s);
        S.rowptr[ent[i].key / nv + 1]++;
        i = j;
    }
    for (int64_t r = 0; r < nv; ++r) S.rowptr[r + 1] += S.rowptr[r];
    S.nnz = (int64_t)S.col.size();
    return 0;
}

}  // namespace etpic
