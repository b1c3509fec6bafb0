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
