// Host-side tet-mesh tables of the etpic library (internal header).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

namespace etpic {

// Local edge (i<j) and local face (opposite vertex k) tables of a tet whose
// vertices are stored in ascending global id.
constexpr int kLocalEdge[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
constexpr int kLocalFace[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};

// Per-tet integer record as laid out on the device (80 bytes, 16-byte aligned).
struct alignas(16) TetTopo {
    int32_t e[6];   // global edge ids of the local edges
    int32_t f[4];   // global face ids, face k opposite local vertex k
    int32_t v[4];   // global vertex ids (ascending)
    int32_t n[4];   // neighbouring tet across face k, -1 at the domain boundary
    int32_t pad[2];
};
static_assert(sizeof(TetTopo) == 80, "TetTopo layout");

struct HostMesh {
    int64_t nv = 0, ne = 0, nf = 0, nt = 0;
    std::vector<int32_t> edges;     // ne*2, (a<b), lexicographic
    std::vector<int32_t> faces;     // nf*3, (a<b<c), lexicographic
    std::vector<TetTopo> topo;      // nt
    std::vector<double> grad;       // nt*12: grad lambda_0..3 (x,y,z each)
    std::vector<double> vol;        // nt: |volume|
    std::vector<int32_t> v2e_ptr;   // nv+1: CSR of vertex -> incident edges
    std::vector<int32_t> v2e_code;  // 2*ne: (edge << 1) | (vertex is the head)
    std::vector<int32_t> e2s_ptr;   // ne+1: CSR of edge -> the tet-local slots that name it
    std::vector<int32_t> e2s_slot;  // 6*nt: 8 * tet + local edge (0..5)
};

// Uniform grid over the mesh's bounding box that gives every cell one tet to
// start a point-location walk from (a tet whose centroid lies in the cell, or,
// for a cell holding no centroid, one borrowed from a nearby cell).
struct StartGrid {
    double lo[3] = {0, 0, 0};    // box corner
    double inv[3] = {1, 1, 1};   // cells per unit length, per axis
    int32_t dims[3] = {1, 1, 1};
    std::vector<int32_t> cell;    // dims[0]*dims[1]*dims[2], x fastest
};

// About one cell per `tets_per_cell` tets (at least one cell per axis).
void build_start_grid(const HostMesh &m, const double *xyz, double tets_per_cell, StartGrid &g);

// Tree-cotree split: edge_tree[ne] marks the edges of a spanning tree of the
// vertex graph (breadth first from the lowest vertex of each component,
// incident edges in ascending id); face_tree[nf] the faces of a spanning tree
// of the dual graph of tets plus one exterior node (every boundary face joins
// its tet to the exterior; tets reached first from the exterior in ascending
// id, then breadth first through interior faces).
void tree_cotree(const HostMesh &H, uint8_t *edge_tree, uint8_t *face_tree);

// Builds every table from the raw mesh.  Returns 0, -1 (bad input) or -4
// (unsorted row, degenerate tet, non-manifold face); err gets the reason.
int build_host_mesh(int64_t nv, const double *xyz, int64_t nt, const int32_t *tv, HostMesh &out,
                    std::string &err);

}  // namespace etpic
