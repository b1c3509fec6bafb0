"""Oracle of the non-solenoidal field solve of the quasi-Helmholtz split
(float64, numpy / scipy).

TEST INFRASTRUCTURE only.  Shares no code with the HIP library.

Gauss' law is discretised on its own (Quasi Helmholtz or Coulomb gauge,
Discrete System, eq. ns_equation): the non-solenoidal electric field is the
discrete gradient of nodal coefficients x,

    C_z^T [grad]^T [*eps] [grad] C_z x = -C_z^T [grad]^T e^{-j w t} G,
    e_ns = [grad] C_z x,

with (App. A) [*eps]_ij = eps int W1_i . W1_j the Whitney edge mass and
[grad] = eps [*eps]^-1 M_g, M_ij = int W1_i . grad W0_j.  The gradient of a
nodal hat function is spanned by the edge functions (grad W0_j = sum over
the edges e at j of +-W1_e, + where j is the edge's head), so [grad] is the
node-to-edge incidence D (-1 at the tail, +1 at the head of each edge, edges
oriented from the lower to the higher vertex id).  C_z keeps the nodes that
do not lie on the conducting wall (their coefficient is zero).  G is the real
path integral of the deposited current; the charge present when it started
(nodal, rho0) is added to D^T G, since D^T G counts only the change.

Because the operator is real, x = e^{-j w t} y with y real.

`correct` applies the same operator to a given edge field u: it adds the
gradient D y that makes u obey Gauss' law exactly, which leaves its curl
(and so the face field) unchanged.

`solenoidal_part` and `solenoidal_source` are the projector of the split in
the [*eps] inner product (the energy-orthogonal reading of P^Lambda_e and its
transpose): P u = u - D y with D^T [*eps] D y = D^T [*eps] u, and
P^T g = g - [*eps] D y with D^T [*eps] D y = D^T g, both at the inner nodes.
The solenoidal system is the field step with its state in the range of P and
its source replaced by P^T g.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import field


def incidence(mesh):
    """D [N_e, N_n]: -1 at each edge's tail (lower vertex id), +1 at its head."""
    ed = mesh.edges().astype(np.int64)
    ne = ed.shape[0]
    rows = np.repeat(np.arange(ne), 2)
    cols = ed.ravel()
    vals = np.tile([-1.0, 1.0], ne)
    return sp.csr_matrix((vals, (rows, cols)), shape=(ne, mesh.nv))


def wall_nodes(mesh):
    """Boolean [N_n]: vertices of the faces that belong to one tet only."""
    tv = mesh.tv.astype(np.int64)
    nb = mesh.neighbours()
    wall = np.zeros(mesh.nv, dtype=bool)
    for k in range(4):
        on = nb[:, k] < 0
        for j in range(4):
            if j != k:
                wall[tv[on, j]] = True
    return wall


class NsOracle:
    """The operator of eq. ns_equation on one mesh, factorised once."""

    def __init__(self, mesh, eps):
        self.mesh, self.eps = mesh, eps
        M, _, bnd = field.assemble(mesh, eps, 1.0)
        self.M = M
        self.bnd = bnd                                      # edges of boundary faces
        self.D = incidence(mesh)
        self.S = (self.D.T @ M @ self.D).tocsr()           # D^T [*eps] D on every node
        self.wall = wall_nodes(mesh)
        self.inner = np.flatnonzero(~self.wall)
        self.lu = spla.splu(self.S[self.inner][:, self.inner].tocsc())

    def solve_nodal(self, b):
        """Real y with y = 0 on the wall and (D^T [*eps] D y)_i = b_i at the other nodes."""
        y = np.zeros(self.mesh.nv)
        if self.inner.size:
            y[self.inner] = self.lu.solve(np.asarray(b, dtype=np.float64)[self.inner])
        return y

    def rhs(self, G=None, rho0=None):
        """-(D^T G + rho0), the right-hand side before the carrier phase."""
        r = np.zeros(self.mesh.nv)
        if G is not None:
            r -= self.D.T @ np.asarray(G, dtype=np.float64)
        if rho0 is not None:
            r -= rho0
        return r

    def solve(self, G=None, rho0=None, t=0.0, omega=0.0):
        """(x [N_n] complex, e_ns [N_e] complex) of eq. ns_equation."""
        y = self.solve_nodal(self.rhs(G, rho0))
        ph = np.exp(-1j * omega * t)
        return y * ph, (self.D @ y) * ph

    def correct(self, u, G=None, rho0=None, t=0.0, omega=0.0):
        """e = u + D y, y zero on the wall, with D^T [*eps] e = -e^{-j w t}(D^T G + rho0)
        at the other nodes (u complex on the edges)."""
        rhs = self.rhs(G, rho0) * np.exp(-1j * omega * t) - self.D.T @ (self.M @ u)
        y = self.solve_nodal(rhs.real) + 1j * self.solve_nodal(rhs.imag)
        return u + self.D @ y

    def gauss_residual(self, e_ns, G=None, rho0=None, t=0.0, omega=0.0):
        """max over the inner nodes of |D^T [*eps] e_ns - e^{-j w t} rhs| and max |rhs|."""
        r = self.rhs(G, rho0) * np.exp(-1j * omega * t)
        lhs = self.D.T @ (self.M @ e_ns)
        I = self.inner
        return np.abs(lhs[I] - r[I]).max(initial=0.0), np.abs(r[I]).max(initial=0.0)

    def solenoidal_part(self, u):
        """P u = u - D y, y zero on the wall, D^T [*eps] D y = D^T [*eps] u at the
        other nodes: D^T [*eps] P u = 0 there and the curl is that of u."""
        rhs = self.D.T @ (self.M @ u)
        if np.iscomplexobj(rhs):
            y = self.solve_nodal(rhs.real) + 1j * self.solve_nodal(rhs.imag)
        else:
            y = self.solve_nodal(rhs)
        return u - self.D @ y

    def solenoidal_source(self, g):
        """P^T g = g - [*eps] D y, y zero on the wall, D^T [*eps] D y = D^T g at
        the other nodes (g real, on the edges): D^T P^T g = 0 there.  On the
        edges of boundary faces, where the field step takes no source, g is
        kept."""
        g = np.asarray(g, dtype=np.float64)
        gs = g - self.M @ (self.D @ self.solve_nodal(self.D.T @ g))
        gs[self.bnd] = g[self.bnd]
        return gs
