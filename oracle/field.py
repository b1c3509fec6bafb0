"""Oracle of the implicit envelope field step (float64, numpy / scipy).

TEST INFRASTRUCTURE only.  Shares no code with the HIP library.

The envelope curl equations (Formulation) with the face envelope eliminated,
tested with the Whitney edge functions (Formulation; Appendix A: the Galerkin
mass [*eps] and the curl operators), give for the complex edge envelope e

    M e'' + 2 j w M e' + (K - w^2 M) e = f,    f = -e^{-j w t} g'',
    M_ij = eps int W1_i . W1_j,    K_ij = (1/mu) int curl W1_i . curl W1_j,

stepped with Newmark-beta, gamma = 1/2, beta = 1/4 (Formulation).  The face
envelope obeys (j w + d/dt) b = -C e, integrated with the trapezoidal rule.
Boundary (perfect-conductor) edges carry zero tangential field: the oracle
solves on the interior edges only.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

LE = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
LF = [(1, 2, 3), (0, 2, 3), (0, 1, 3), (0, 1, 2)]
# 4-point rule on the tetrahedron, exact for quadratics (barycentric points, weight V/4)
QA, QB = 0.5854101966249685, 0.1381966011250105
QPTS = np.array([[QA, QB, QB, QB], [QB, QA, QB, QB], [QB, QB, QA, QB], [QB, QB, QB, QA]])


def tet_gradients(xyz, tv):
    """grad lambda_k for every tet [N_t, 4, 3] and |volume| [N_t]: lambda_k vanishes on
    the face opposite k, so its gradient is that face's normal n over n.(r_k - r_a)."""
    r = xyz[tv]                                    # [N_t, 4, 3]
    g = np.empty((tv.shape[0], 4, 3))
    for k, (a, b, c) in enumerate(LF):
        n = np.cross(r[:, b] - r[:, a], r[:, c] - r[:, a])
        g[:, k] = n / np.einsum("ij,ij->i", n, r[:, k] - r[:, a])[:, None]
    vol = np.abs(np.einsum("ij,ij->i", r[:, 1] - r[:, 0], np.cross(r[:, 2] - r[:, 0], r[:, 3] - r[:, 0]))) / 6.0
    return g, vol


def assemble(mesh, eps, mu):
    """(M, K) as scipy CSR [N_e, N_e] on all edges, and the boolean boundary-edge mask."""
    xyz, tv = mesh.xyz, mesh.tv
    te = mesh.tet_edges()
    g, vol = tet_gradients(xyz, tv)
    nt = tv.shape[0]
    # Whitney edge functions at the quadrature points: W[q][t, e, :]
    Ml = np.zeros((nt, 6, 6))
    for lam in QPTS:
        W = np.stack([lam[i] * g[:, j] - lam[j] * g[:, i] for i, j in LE], axis=1)   # [N_t, 6, 3]
        Ml += np.einsum("tea,tfa->tef", W, W) * (vol / 4.0)[:, None, None]
    curl = np.stack([2.0 * np.cross(g[:, i], g[:, j]) for i, j in LE], axis=1)         # [N_t, 6, 3]
    Kl = np.einsum("tea,tfa->tef", curl, curl) * vol[:, None, None]
    rows = np.repeat(te, 6, axis=1).ravel()
    cols = np.tile(te, (1, 6)).ravel()
    M = sp.csr_matrix((eps * Ml.ravel(), (rows, cols)), shape=(mesh.ne, mesh.ne))
    K = sp.csr_matrix((Kl.ravel() / mu, (rows, cols)), shape=(mesh.ne, mesh.ne))
    nb = mesh.neighbours()
    bnd = np.zeros(mesh.ne, dtype=bool)
    for k in range(4):
        on = nb[:, k] < 0
        for e, (i, j) in enumerate(LE):
            if i != k and j != k:
                bnd[te[on, e]] = True
    return M, K, bnd


def face_edges(mesh):
    """[N_f, 3] edge ids of (a,b), (b,c), (a,c) for each face (a<b<c)."""
    ed = mesh.edges().astype(np.int64)
    fc = mesh.faces().astype(np.int64)
    key = ed[:, 0] * mesh.nv + ed[:, 1]

    def idx(a, b):
        return np.searchsorted(key, a * mesh.nv + b)
    return np.stack([idx(fc[:, 0], fc[:, 1]), idx(fc[:, 1], fc[:, 2]), idx(fc[:, 0], fc[:, 2])], axis=1)


class FieldOracle:
    """solver: "lu" (sparse direct, scipy's splu) or "gmres" (scipy's restarted
    GMRES, unpreconditioned, to a relative residual of 1e-15: the step's system
    is dominated by the mass term, so it converges in ~50 iterations, where a
    direct factorisation of a 10^5-unknown 3-D system takes minutes).  The
    default takes the direct solve up to 40,000 interior edges."""

    def __init__(self, mesh, dt, omega, eps, mu, solver=None):
        self.mesh, self.dt, self.w = mesh, dt, omega
        self.M, self.K, self.bnd = assemble(mesh, eps, mu)
        self.inner = np.flatnonzero(~self.bnd)
        self.fe = face_edges(mesh)
        Mi = self.M[self.inner][:, self.inner]
        Ki = self.K[self.inner][:, self.inner]
        self.Mi, self.Ki = Mi.tocsc(), Ki.tocsc()
        alpha = 1.0 + 1j * omega * dt - 0.25 * omega ** 2 * dt ** 2
        self.A = (alpha * Mi + (0.25 * dt ** 2) * Ki).tocsc()
        self.solver = solver or ("lu" if self.inner.size <= 40_000 else "gmres")
        if self.solver == "lu":
            self.lu = spla.splu(self.A)
        elif self.solver == "gmres":
            self.Ar = self.A.tocsr()
        else:
            raise ValueError(f"unknown solver {solver!r}")

    def solve(self, rhs):
        """x with A x = rhs on the interior edges."""
        if self.solver == "lu":
            return self.lu.solve(rhs)
        x, info = spla.gmres(self.Ar, rhs, rtol=1e-15, atol=0.0, restart=300, maxiter=20)
        if info != 0 or np.linalg.norm(self.Ar @ x - rhs) > 1e-13 * np.linalg.norm(rhs):
            raise RuntimeError(f"oracle GMRES did not converge (info {info})")
        return x

    def step(self, t_next, u, v, a, b, gdd=None):
        """Newmark-beta (1/2, 1/4) step in acceleration form; returns (u, v, a, b)."""
        dt, w, I = self.dt, self.w, self.inner
        us = u + dt * v + 0.25 * dt * dt * a
        vs = v + 0.5 * dt * a
        f = np.zeros(u.shape, complex) if gdd is None else -np.exp(-1j * w * t_next) * gdd
        rhs = f[I] - self.Mi @ (2j * w * vs[I] - w * w * us[I]) - self.Ki @ us[I]
        an = np.zeros_like(u)
        an[I] = self.solve(rhs)
        un = us + 0.25 * dt * dt * an
        vn = vs + 0.5 * dt * an
        ce = lambda e: e[self.fe[:, 0]] + e[self.fe[:, 1]] - e[self.fe[:, 2]]
        bn = ((1 - 0.5j * w * dt) * b - 0.5 * dt * ce(u + un)) / (1 + 0.5j * w * dt)
        return un, vn, an, bn

    def energy(self, u, v):
        """0.5 v^H M v + 0.5 u^H (K - w^2 M) u, conserved by the source-free step."""
        I = self.inner
        return 0.5 * np.vdot(v[I], self.Mi @ v[I]).real + 0.5 * np.vdot(u[I], (self.Ki @ u[I] - self.w ** 2 * (self.Mi @ u[I]))).real
