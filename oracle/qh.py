"""Oracle of the quasi-Helmholtz projectors (float64, numpy / scipy).

TEST INFRASTRUCTURE only.  Shares no code with the HIP library.

Projectors of the Quasi Helmholtz or Coulomb gauge section (eqs. proj_es,
proj_el, bfld_projector) with the App. A operators:

    P^Sigma_e = Sigma (Sigma^T Sigma)^+ Sigma^T,   P^Lambda_e = I - P^Sigma_e,
    P^Lambda_b = I - Sigma_m (Sigma_m^T Sigma_m)^+ Sigma_m^T,

Sigma = eps0 M_g (N_e x N_n) and Sigma_m = [div]^T (N_f x N_t).  With the
Whitney spaces, eps0 M_g = [*eps] D (D the node-to-edge incidence: the
gradient of a hat function is a signed sum of edge functions) and
[div] = [*rho]^-1 M_d is the tet-to-face incidence: +1 where the face's
global normal (right-handed in its ascending vertex order) points out of the
tet, -1 where it points in.  + is the Moore-Penrose pseudoinverse.  The
decomposition of the flux density (eq. efld_projected) is
D = Sigma E_ns + P^Lambda_e D with E_ns = (Sigma^T Sigma)^+ Sigma^T D.

The end of the module builds the Z blocks of the solenoidal system (eq.
sol_disc) densely on small meshes: a study of its spectrum, and the
reference for the library's matrix-free blocks and its step of the system.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import field, gauss


def face_signs(mesh):
    """[N_t, 4] +-1: orientation of the global normal of face k (opposite
    local vertex k) relative to the outward normal of the tet."""
    xyz, tv = mesh.xyz, mesh.tv.astype(np.int64)
    fc = mesh.faces().astype(np.int64)
    tf = mesh.tet_faces().astype(np.int64)
    s = np.empty(tf.shape)
    for k in range(4):
        f = fc[tf[:, k]]
        a, b, c = xyz[f[:, 0]], xyz[f[:, 1]], xyz[f[:, 2]]
        n = np.cross(b - a, c - a)
        out = np.einsum("ij,ij->i", n, a - xyz[tv[:, k]])
        s[:, k] = np.where(out > 0, 1.0, -1.0)
    return s


def div_matrix(mesh):
    """[div] [N_t, N_f]: sum over a tet's faces of the signed face DoFs."""
    tf = mesh.tet_faces().astype(np.int64)
    s = face_signs(mesh)
    rows = np.repeat(np.arange(mesh.nt), 4)
    return sp.csr_matrix((s.ravel(), (rows, tf.ravel())), shape=(mesh.nt, mesh.nf))


def _solve_real(lu, rhs):
    rhs = np.asarray(rhs)
    if np.iscomplexobj(rhs):
        return lu.solve(np.ascontiguousarray(rhs.real)) + 1j * lu.solve(np.ascontiguousarray(rhs.imag))
    return lu.solve(np.ascontiguousarray(rhs, dtype=np.float64))


class QhOracle:
    """The three projectors on one mesh (permittivity eps in [*eps])."""

    def __init__(self, mesh, eps):
        self.mesh = mesh
        self.div = div_matrix(mesh)
        # Sigma_m^T Sigma_m = div div^T: nonsingular once a tet has a boundary face
        self.lu_b = spla.splu((self.div @ self.div.T).tocsc())
        M, _, _ = field.assemble(mesh, eps, 1.0)
        self.M = M
        self.D = gauss.incidence(mesh)
        self.Sigma = (M @ self.D).tocsr()
        SS = (self.Sigma.T @ self.Sigma).tocsr()
        # Sigma^T Sigma has the constants as its null space (mesh connected):
        # ground node 0 for a solution, then remove the mean for the minimum-norm one
        self.lu_e = spla.splu(SS[1:, 1:].tocsc())
        self.SS = SS

    def project_b(self, b):
        """P^Lambda_b b (face DoFs, real or complex)."""
        y = _solve_real(self.lu_b, self.div @ b)
        return b - self.div.T @ y

    def e_ns(self, d):
        """(Sigma^T Sigma)^+ Sigma^T d: the minimum-norm nodal solution."""
        rhs = self.Sigma.T @ d
        y = np.zeros(self.mesh.nv, dtype=np.result_type(rhs, np.float64))
        y[1:] = _solve_real(self.lu_e, rhs[1:])
        return y - y.mean()

    def project_e(self, d):
        """(P^Sigma_e d, P^Lambda_e d, E_ns) for edge DoFs d (real or complex)."""
        y = self.e_ns(d)
        ps = self.Sigma @ y
        return ps, d - ps, y


# ------------------------------------------------- solenoidal system (study)
# eq. sol_disc couples the solenoidal unknowns on the cotree edges and faces
# through the Z blocks of App. A.  The helpers below build them densely for
# small meshes, to study the semi-discrete system's spectrum (E'' = -A E with
# omega = 0, B eliminated): a lossless closed cavity must give real, positive
# eigenvalues, the squares of its resonance frequencies.

LF = [(1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)]


def face_mass(mesh, mu):
    """[*mu^-1]_ij = (1/mu) int W2_i . W2_j with W2_ijk = 2 (l_i g_j x g_k +
    l_j g_k x g_i + l_k g_i x g_j) (flux 1 through its face, oriented like the
    face DoFs), 4-point rule (exact for the quadratic integrand); dense."""
    g, vol = field.tet_gradients(mesh.xyz, mesh.tv)
    tf = mesh.tet_faces()
    Ml = np.zeros((mesh.nt, 4, 4))
    for lam in field.QPTS:
        W = np.stack([2 * (lam[i] * np.cross(g[:, j], g[:, k]) + lam[j] * np.cross(g[:, k], g[:, i])
                           + lam[k] * np.cross(g[:, i], g[:, j])) for i, j, k in LF], axis=1)
        Ml += np.einsum("tka,tla->tkl", W, W) * (vol / 4.0)[:, None, None]
    F = np.zeros((mesh.nf, mesh.nf))
    for a in range(4):
        for b in range(4):
            np.add.at(F, (tf[:, a], tf[:, b]), Ml[:, a, b] / mu)
    return F


def curl_incidence(mesh):
    """C [N_f, N_e]: (C e)_f = e_ab + e_bc - e_ac for the face (a < b < c)."""
    fe = field.face_edges(mesh)
    C = np.zeros((mesh.nf, mesh.ne))
    r = np.arange(mesh.nf)
    C[r, fe[:, 0]] += 1.0
    C[r, fe[:, 1]] += 1.0
    C[r, fe[:, 2]] -= 1.0
    return C


def spanning_trees(mesh):
    """(edge_tree, face_tree) booleans: breadth-first spanning tree of the
    vertex graph from the lowest vertex of each component (incident edges in
    ascending id), and of the dual graph of tets plus the exterior (boundary
    faces first, tets in ascending id, then breadth first)."""
    ed = mesh.edges().astype(np.int64)
    adj = [[] for _ in range(mesh.nv)]
    for e, (a, b) in enumerate(ed):
        adj[a].append((e, b))
        adj[b].append((e, a))
    et = np.zeros(mesh.ne, dtype=bool)
    seen = np.zeros(mesh.nv, dtype=bool)
    for root in range(mesh.nv):
        if seen[root]:
            continue
        seen[root] = True
        queue = [root]
        for u in queue:
            for e, w in sorted(adj[u]):
                if not seen[w]:
                    seen[w] = True
                    et[e] = True
                    queue.append(w)
    nb, tf = mesh.neighbours(), mesh.tet_faces()
    ft = np.zeros(mesh.nf, dtype=bool)
    tseen = np.zeros(mesh.nt, dtype=bool)
    queue = []
    for t in range(mesh.nt):
        for k in range(4):
            if nb[t, k] < 0:
                tseen[t] = True
                ft[tf[t, k]] = True
                queue.append(t)
                break
    for t in queue:
        for k in range(4):
            n = nb[t, k]
            if n >= 0 and not tseen[n]:
                tseen[n] = True
                ft[tf[t, k]] = True
                queue.append(n)
    return et, ft


def solenoidal_blocks(mesh, eps, mu, weighted):
    """Dense (Z11, Z12, Z21, Z22) of eq. sol_disc on the cotree unknowns.
    weighted = False: the blocks as printed in App. A (Euclidean projectors,
    [curl] = C since curl W1 is a signed sum of W2, [*eps]^-1 as a dense
    inverse).  weighted = True: the same structure with the projectors made
    orthogonal in the energy products ([*eps] on edges, [*mu^-1] on faces),
    the fields parameterised as e = P_e C_e E_s, b = P_b C_b B_s and the two
    equations (Faraday, Ampere) tested with those same fields."""
    Q = QhOracle(mesh, eps)
    M = Q.M.toarray()
    D = Q.D.toarray()
    div = Q.div.toarray()
    C = curl_incidence(mesh)
    F = face_mass(mesh, mu)
    et, ft = spanning_trees(mesh)
    Ce = np.eye(mesh.ne)[:, ~et]
    Cb = np.eye(mesh.nf)[:, ~ft]
    if not weighted:
        Sig = M @ D
        Pe = np.eye(mesh.ne) - Sig @ np.linalg.pinv(Sig.T @ Sig) @ Sig.T
        Pb = np.eye(mesh.nf) - div.T @ np.linalg.solve(div @ div.T, div)
        Z11 = Cb.T @ Pb @ Cb
        Z12 = Cb.T @ C @ np.linalg.solve(M, Pe @ M @ Ce)
        Z21 = Ce.T @ Pe @ M @ Ce
        Z22 = Ce.T @ C.T @ F @ Pb @ Cb
        return Z11, Z12, Z21, Z22, (Ce, Cb, C)
    Pe = np.eye(mesh.ne) - D @ np.linalg.pinv(D.T @ M @ D) @ D.T @ M
    Fi = np.linalg.inv(F)
    Pb = np.eye(mesh.nf) - Fi @ div.T @ np.linalg.solve(div @ Fi @ div.T, div)
    Ee, Bb = Pe @ Ce, Pb @ Cb
    return Bb.T @ F @ Bb, Bb.T @ F @ C @ Ee, Ee.T @ M @ Ee, Ee.T @ C.T @ F @ Bb, (Ce, Cb, C)


def solenoidal_spectrum(mesh, eps, mu, weighted):
    """Eigenvalues of A in E'' = -A E (omega = 0, source free), from
    Z11 B' = -Z12 E and Z21 E' = Z22 B."""
    Z11, Z12, Z21, Z22, _ = solenoidal_blocks(mesh, eps, mu, weighted)
    return np.linalg.eigvals(np.linalg.solve(Z21, Z22) @ np.linalg.solve(Z11, Z12))


def inner_nodes(mesh):
    """Indices of the nodes off the conducting wall, ascending ([C^e_z] of
    eq. ns_equation selects them)."""
    return np.flatnonzero(~gauss.wall_nodes(mesh))


def solenoidal_source_blocks(mesh, eps):
    """Dense (Z13, Z23, Cz) of eq. sol_disc as printed in App. A:
    Z13 = C_b^T [curl] [*eps]^-1 Sigma C_z and Z23 = C_e^T Sigma C_z, with
    Sigma = [*eps] D and [*eps]^-1 as a dense inverse."""
    Q = QhOracle(mesh, eps)
    M = Q.M.toarray()
    Sig = M @ Q.D.toarray()
    C = curl_incidence(mesh)
    et, ft = spanning_trees(mesh)
    Ce = np.eye(mesh.ne)[:, ~et]
    Cb = np.eye(mesh.nf)[:, ~ft]
    Cz = np.eye(mesh.nv)[:, inner_nodes(mesh)]
    return Cb.T @ C @ np.linalg.solve(M, Sig @ Cz), Ce.T @ Sig @ Cz, Cz


def solenoidal_step(mesh, eps, mu, dt, omega, Bs, Es, src_b=None, src_e=None):
    """One step of eq. sol_disc as printed (Euclidean projectors), the time
    derivatives by the trapezoidal rule over [t_n, t_n + dt]:
        Z11 (B1 - B0)/dt + j w Z11 (B1 + B0)/2 + Z12 (E1 + E0)/2 = src_b,
        Z21 (E1 - E0)/dt + j w Z21 (E1 + E0)/2 - Z22 (B1 + B0)/2 = src_e,
    solved densely for (B1, E1) on the cotree unknowns; src_b, src_e are the
    right-hand sides at the midpoint (zero if None)."""
    Z11, Z12, Z21, Z22, _ = solenoidal_blocks(mesh, eps, mu, weighted=False)
    nb, ne_ = Z11.shape[0], Z21.shape[0]
    a, ab = 1.0 / dt + 0.5j * omega, 1.0 / dt - 0.5j * omega
    A = np.block([[a * Z11, 0.5 * Z12], [-0.5 * Z22, a * Z21]])
    rb = ab * (Z11 @ Bs) - 0.5 * (Z12 @ Es) + (0 if src_b is None else src_b)
    re = ab * (Z21 @ Es) + 0.5 * (Z22 @ Bs) + (0 if src_e is None else src_e)
    # B and E carry units a factor ~c apart and the rows scale with 1/dt and
    # eps: equilibrate rows and columns (Ruiz) before the dense solve, or its
    # error grows with the raw condition number (~1e15)
    r, c = np.ones(nb + ne_), np.ones(nb + ne_)
    As = A.copy()
    for _ in range(5):
        rr, cc = 1.0 / np.sqrt(np.abs(As).max(axis=1)), 1.0 / np.sqrt(np.abs(As).max(axis=0))
        As = rr[:, None] * As * cc[None, :]
        r, c = r * rr, c * cc
    x = c * np.linalg.solve(As, r * np.concatenate([rb, re]))
    return x[:nb], x[nb:]


def solenoidal_b_field(mesh, eps, Bs):
    """The face field P^Lambda_b C_b B_s of the cotree unknowns B_s (the
    divergence-free magnetic flux the printed blocks act on)."""
    Q = QhOracle(mesh, eps)
    _, ft = spanning_trees(mesh)
    b = np.zeros(mesh.nf, dtype=np.result_type(Bs, np.float64))
    b[~ft] = Bs
    return Q.project_b(b)
