// Host-side assembly of the edge-element matrices of the field update (internal header).
#pragma once
#include <cstdint>
#include <string>
#include <vector>

#include "mesh_host.hpp"

namespace etpic {

// Galerkin matrices on the Whitney edge space, one CSR pattern (rows sorted):
//   M[i][j] = eps   * int W1_i . W1_j            (edge mass, the [*eps] of Appendix A)
//   K[i][j] = 1/mu  * int curl W1_i . curl W1_j  (curl-curl stiffness)
// Rows and columns of boundary edges (edges of faces with one owning tet) are
// replaced by the identity in M and zero in K (perfect-conductor walls: the
// tangential field on the boundary is zero).
struct FieldSystem {
    int64_t ne = 0, nf = 0, nnz = 0;
    std::vector<int32_t> rowptr;     // ne + 1
    std::vector<int32_t> col;        // nnz
    std::vector<double> M, K;        // nnz each
    std::vector<uint8_t> dirichlet;  // ne
    std::vector<int32_t> face_edge;  // nf*3: edges (a,b), (b,c), (a,c) of face (a<b<c)
};

// dirichlet = false keeps every row and column (the plain Galerkin matrices;
// the mask is still filled).
int build_field_system(const HostMesh &mesh, double eps, double mu, FieldSystem &out, std::string &err,
                       bool dirichlet = true);

// Nodal operator of the non-solenoidal field (eq. ns_equation):
//   S[i][j] = eps int grad W0_i . grad W0_j = (D^T [*eps] D)[i][j],
// D the node-to-edge incidence.  Wall nodes (vertices of faces with one
// owning tet) are grounded: their rows are the identity and their columns
// are dropped from the other rows.  Rows sorted.
struct NsSystem {
    int64_t nv = 0, nnz = 0;
    std::vector<int32_t> rowptr;     // nv + 1
    std::vector<int32_t> col;        // nnz
    std::vector<double> S;           // nnz
    std::vector<uint8_t> wall;       // nv
};

int build_ns_system(const HostMesh &mesh, double eps, NsSystem &out, std::string &err);

}  // namespace etpic
