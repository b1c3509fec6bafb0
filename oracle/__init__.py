"""ctypes front-end of the FP64 C oracle (oracle.c).

TEST INFRASTRUCTURE: imported only by tests/, the smoke check and the
benchmark's CPU-baseline leg.  Nothing in the product package imports it."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None

_dp = C.POINTER(C.c_double)
_ip = C.POINTER(C.c_int32)
_lp = C.POINTER(C.c_int64)


def _load():
    global _LIB
    if _LIB is not None:
        return _LIB
    path = os.path.join(HERE, "liboracle.so")
    if not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(os.path.join(HERE, "oracle.c")):
        from . import build as _b
        _b.build()
    lib = C.CDLL(path)
    vp = C.c_void_p
    lib.ora_mesh_build.argtypes = [C.c_int64, _dp, C.c_int64, _ip, C.POINTER(vp)]
    lib.ora_mesh_build.restype = C.c_int
    lib.ora_mesh_free.argtypes = [vp]
    for name in ("ora_mesh_edges", "ora_mesh_faces", "ora_mesh_tet_edges", "ora_mesh_tet_faces", "ora_mesh_neighbours"):
        getattr(lib, name).argtypes = [vp, _ip]
    lib.ora_mesh_counts.argtypes = [vp, _lp]
    lib.ora_grad.argtypes = [vp, C.c_int64, _dp]
    lib.ora_bary.argtypes = [vp, C.c_int64, _dp, _dp]
    lib.ora_point.argtypes = [vp, C.c_int64, _dp, _dp]
    lib.ora_whitney1.argtypes = [vp, C.c_int64, _dp, _dp]
    lib.ora_whitney2.argtypes = [vp, C.c_int64, _dp, _dp]
    lib.ora_fields.argtypes = [vp, C.c_int64, _dp, C.c_double, C.c_double, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.ora_boris.argtypes = [_dp, _dp, _dp, C.c_double, C.c_double]
    lib.ora_step.argtypes = [vp, C.c_int64, _ip, _dp, _dp, C.c_double, C.c_double, C.c_double, C.c_int64,
                             C.c_double, C.c_double, _dp, _dp, _dp, _dp, _dp, _dp, _ip, C.c_int]
    lib.ora_step.restype = C.c_int
    lib.ora_step_t.argtypes = [vp, C.c_int64, _ip, _dp, _dp, C.c_double, C.c_double, C.c_double, C.c_double,
                               C.c_double, C.c_double, _dp, _dp, _dp, _dp, _dp, _dp, _ip, C.c_int]
    lib.ora_step_t.restype = C.c_int
    lib.ora_step_one.argtypes = [vp, _ip, _dp, _dp, C.c_double, C.c_double, C.c_double, C.c_int64, C.c_double,
                                 C.c_double, _dp, _dp, _dp, _dp, _dp, _lp, _ip]
    lib.ora_step_one.restype = C.c_int
    lib.ora_charge.argtypes = [vp, C.c_int64, _ip, _dp, C.c_double, C.c_double, _dp]
    lib.ora_gauss.argtypes = [vp, _dp, _dp, _dp, _dp]
    lib.ora_vjp.argtypes = [vp, C.c_int64, _ip, _dp, _dp, C.c_double, C.c_double, C.c_double, C.c_int64, C.c_int,
                            C.c_double, C.c_double, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp, C.c_int]
    lib.ora_vjp.restype = C.c_int
    lib.ora_jvp.argtypes = [vp, C.c_int64, _ip, _dp, _dp, C.c_double, C.c_double, C.c_int64, C.c_int, C.c_double,
                            C.c_double, _dp, _dp, _dp, _dp, _dp, _dp, _dp, C.c_int]
    lib.ora_jvp.restype = C.c_int
    lib.ora_locate.argtypes = [vp, _dp, _dp]
    lib.ora_locate.restype = C.c_int64
    lib.ora_ds_weights.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, _dp, _dp, _dp, _dp, _dp, _dp]
    lib.ora_ds_step.argtypes = [vp, C.c_int64, _ip, _dp, _dp, _dp, _dp, _dp, C.c_int, C.c_double, C.c_double,
                                C.c_double, C.c_double, C.c_double, C.c_double, _dp, _dp, _dp, _dp, _dp, _dp, C.c_int]
    lib.ora_ds_step.restype = C.c_int
    _LIB = lib
    return lib


def _p(a, ty=_dp):
    return None if a is None else a.ctypes.data_as(ty)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _cplx(z):
    """complex128[N] -> contiguous float64[N,2]"""
    if z is None:
        return None
    z = np.asarray(z)
    if np.iscomplexobj(z):
        return np.ascontiguousarray(np.stack([z.real, z.imag], axis=1))
    return _f64(z)


class OracleMesh:
    """Own connectivity of a tet mesh (built by the C oracle)."""

    def __init__(self, xyz, tet_vert):
        lib = _load()
        self.xyz = _f64(xyz)
        self.tv = np.ascontiguousarray(tet_vert, dtype=np.int32)
        h = C.c_void_p()
        rc = lib.ora_mesh_build(self.xyz.shape[0], _p(self.xyz), self.tv.shape[0], _p(self.tv, _ip), C.byref(h))
        if rc != 0:
            raise ValueError(f"oracle mesh build failed ({rc})")
        self.h = h
        cnt = np.zeros(4, dtype=np.int64)
        lib.ora_mesh_counts(h, _p(cnt, _lp))
        self.nv, self.ne, self.nf, self.nt = (int(x) for x in cnt)

    def __del__(self):
        if getattr(self, "h", None) and _LIB is not None:
            _LIB.ora_mesh_free(self.h)
            self.h = None

    def _int_table(self, name, cols, rows):
        out = np.zeros((rows, cols), dtype=np.int32)
        getattr(_load(), name)(self.h, _p(out, _ip))
        return out

    def edges(self):
        return self._int_table("ora_mesh_edges", 2, self.ne)

    def faces(self):
        return self._int_table("ora_mesh_faces", 3, self.nf)

    def tet_edges(self):
        return self._int_table("ora_mesh_tet_edges", 6, self.nt)

    def tet_faces(self):
        return self._int_table("ora_mesh_tet_faces", 4, self.nt)

    def neighbours(self):
        return self._int_table("ora_mesh_neighbours", 4, self.nt)

    # -- pointwise geometry / basis -------------------------------------------
    def grad(self, T):
        g = np.zeros((4, 3))
        _load().ora_grad(self.h, int(T), _p(g))
        return g

    def bary(self, T, x):
        lam = np.zeros(4)
        _load().ora_bary(self.h, int(T), _p(_f64(x)), _p(lam))
        return lam

    def point(self, T, lam4):
        x = np.zeros(3)
        _load().ora_point(self.h, int(T), _p(_f64(lam4)), _p(x))
        return x

    def whitney1(self, T, lam4):
        W = np.zeros((6, 3))
        _load().ora_whitney1(self.h, int(T), _p(_f64(lam4)), _p(W))
        return W

    def whitney2(self, T, lam4):
        W = np.zeros((4, 3))
        _load().ora_whitney2(self.h, int(T), _p(_f64(lam4)), _p(W))
        return W

    def fields(self, T, lam4, omega, t, e_env, b_env, e_dc=None, b_dc=None):
        E = np.zeros(3)
        B = np.zeros(3)
        ee, bb = _cplx(e_env), _cplx(b_env)
        ed = None if e_dc is None else _f64(e_dc)
        bd = None if b_dc is None else _f64(b_dc)
        _load().ora_fields(self.h, int(T), _p(_f64(lam4)), float(omega), float(t), _p(ee), _p(ed), _p(bb), _p(bd),
                           _p(E), _p(B))
        return E, B

    def locate(self, x):
        ml = C.c_double()
        t = _load().ora_locate(self.h, _p(_f64(x)), C.byref(ml))
        return int(t), ml.value

    # -- the step ---------------------------------------------------------------
    def step(self, tet, lam, vel, *, q, m, w, step, dt, omega, e_env, b_env, e_dc=None, b_dc=None,
             dG=None, rho=None, want_hops=False, nthreads=1):
        """One step for all particles, in place on (tet, lam, vel).  dG / rho
        accumulate.  Returns (status, hops or None)."""
        assert tet.dtype == np.int32 and tet.flags.c_contiguous
        assert lam.dtype == np.float64 and lam.flags.c_contiguous
        assert vel.dtype == np.float64 and vel.flags.c_contiguous
        n = tet.shape[0]
        ee, bb = _cplx(e_env), _cplx(b_env)
        ed = None if e_dc is None else _f64(e_dc)
        bd = None if b_dc is None else _f64(b_dc)
        hops = np.zeros(n, dtype=np.int32) if want_hops else None
        rc = _load().ora_step(self.h, n, _p(tet, _ip), _p(lam), _p(vel), float(q), float(m), float(w), int(step),
                              float(dt), float(omega), _p(ee), _p(ed), _p(bb), _p(bd), _p(dG), _p(rho),
                              _p(hops, _ip), int(nthreads))
        return rc, hops

    def step_at(self, tet, lam, vel, *, q, m, w, t, dt, omega, e_env, b_env, e_dc=None, b_dc=None, dG=None,
                rho=None, nthreads=1):
        """One step gathering at time t (instead of step*dt), in place."""
        assert tet.dtype == np.int32 and tet.flags.c_contiguous
        assert lam.dtype == np.float64 and lam.flags.c_contiguous
        assert vel.dtype == np.float64 and vel.flags.c_contiguous
        ee, bb = _cplx(e_env), _cplx(b_env)
        ed = None if e_dc is None else _f64(e_dc)
        bd = None if b_dc is None else _f64(b_dc)
        return _load().ora_step_t(self.h, tet.shape[0], _p(tet, _ip), _p(lam), _p(vel), float(q), float(m),
                                  float(w), float(t), float(dt), float(omega), _p(ee), _p(ed), _p(bb), _p(bd),
                                  _p(dG), _p(rho), None, int(nthreads))

    def ds_step(self, tet, lam, vel, hist_state, *, hist, q, m, w, t, dt, omega, e_env, b_env, e_dc=None,
                b_dc=None, dG=None, rho=None, nthreads=1):
        """One downshifted step (velocity by the carrier-exact quadrature of the
        interpolated envelope samples, positions by Adams-Bashforth) at t_n = t,
        in place on (tet, lam, vel) and on hist_state = DsHistory(n).  hist =
        number of downshifted steps before this one.  Returns the status."""
        assert tet.dtype == np.int32 and tet.flags.c_contiguous
        assert lam.dtype == np.float64 and lam.flags.c_contiguous
        assert vel.dtype == np.float64 and vel.flags.c_contiguous
        ee, bb = _cplx(e_env), _cplx(b_env)
        ed = None if e_dc is None else _f64(e_dc)
        bd = None if b_dc is None else _f64(b_dc)
        H = hist_state
        return _load().ora_ds_step(self.h, tet.shape[0], _p(tet, _ip), _p(lam), _p(vel), _p(H.v), _p(H.e), _p(H.b),
                                   int(hist), float(q), float(m), float(w), float(t), float(dt), float(omega),
                                   _p(ee), _p(ed), _p(bb), _p(bd), _p(dG), _p(rho), int(nthreads))

    def coarse_step(self, tet, lam, vel, *, q, m, w, e_snaps, b_snaps, t_coarse, dt_coarse, fine_steps, omega,
                    e_dc=None, b_dc=None, dG=None, rho=None, nthreads=1):
        """One coarse field step at the fine step (Particle Push section): the
        envelope known at t_coarse - dt_coarse, t_coarse, t_coarse + dt_coarse
        (e_snaps, b_snaps: three complex arrays each) is reconstructed at each
        fine time t_j = t_coarse + j dt with the quadratic Lagrange basis
        (eqs. newmark_L / newmark_N), N_k(t) = prod_{i != k} (t - tau_i) /
        (tau_k - tau_i) over the node times tau; the carrier multiplies the
        reconstructed envelope at t_j.  fine_steps Lorentz steps of
        dt = dt_coarse / fine_steps; dG sums the path integrals of all fine steps
        (eq. G_integral); rho gets the charge of the final positions."""
        tau = [t_coarse - dt_coarse, t_coarse, t_coarse + dt_coarse]
        dt = dt_coarse / fine_steps
        for j in range(fine_steps):
            t = t_coarse + j * dt
            N = []
            for k in range(3):
                val = 1.0
                for i in range(3):
                    if i != k:
                        val *= (t - tau[i]) / (tau[k] - tau[i])
                N.append(val)
            e_t = N[0] * np.asarray(e_snaps[0]) + N[1] * np.asarray(e_snaps[1]) + N[2] * np.asarray(e_snaps[2])
            b_t = N[0] * np.asarray(b_snaps[0]) + N[1] * np.asarray(b_snaps[1]) + N[2] * np.asarray(b_snaps[2])
            rc = self.step_at(tet, lam, vel, q=q, m=m, w=w, t=t, dt=dt, omega=omega, e_env=e_t, b_env=b_t,
                              e_dc=e_dc, b_dc=b_dc, dG=dG, rho=rho if j == fine_steps - 1 else None,
                              nthreads=nthreads)
            if rc != 0:
                return rc
        return 0

    def step_one(self, tet, lam3, v, *, q, m, w, step, dt, omega, e_env, b_env, e_dc=None, b_dc=None, dG=None):
        """Single particle; returns (status, tet, lam3, v, piece_tets)."""
        t = np.array([tet], dtype=np.int32)
        l = _f64(lam3).copy()
        vv = _f64(v).copy()
        pt = np.zeros(130, dtype=np.int64)
        npc = np.zeros(1, dtype=np.int32)
        if dG is None:
            dG = np.zeros(self.ne)
        ee, bb = _cplx(e_env), _cplx(b_env)
        ed = None if e_dc is None else _f64(e_dc)
        bd = None if b_dc is None else _f64(b_dc)
        rc = _load().ora_step_one(self.h, _p(t, _ip), _p(l), _p(vv), float(q), float(m), float(w), int(step),
                                  float(dt), float(omega), _p(ee), _p(ed), _p(bb), _p(bd), _p(dG),
                                  _p(pt, _lp), _p(npc, _ip))
        return rc, int(t[0]), l, vv, pt[: int(npc[0])].copy()

    def charge(self, tet, lam, q, w, rho=None):
        if rho is None:
            rho = np.zeros(self.nv)
        _load().ora_charge(self.h, tet.shape[0], _p(np.ascontiguousarray(tet, dtype=np.int32), _ip),
                           _p(_f64(lam)), float(q), float(w), _p(rho))
        return rho

    def gauss(self, dG, rho_new, rho_old):
        out = np.zeros(2)
        _load().ora_gauss(self.h, _p(_f64(dG)), _p(_f64(rho_new)), _p(_f64(rho_old)), _p(out))
        return out[0], out[1]

    def positions(self, tet, lam):
        """Cartesian positions x = sum_k lambda_k r_k (numpy, for comparisons)."""
        l0 = 1.0 - lam.sum(axis=1)
        r = self.xyz[self.tv[tet]]
        return l0[:, None] * r[:, 0] + lam[:, 0:1] * r[:, 1] + lam[:, 1:2] * r[:, 2] + lam[:, 2:3] * r[:, 3]


def _vjp_method(self, tet, lam, vel, *, q, m, w, step0, nsteps, dt, omega, e_env, b_env, vbar, xbar=None,
                e_dc=None, b_dc=None, nthreads=1):
    """Reverse-mode gradient of nsteps steps from (tet, lam, vel): returns
    (status, grad_e complex128[N_e], vbar0[N,3], xbar0[N,3]) for the given
    adjoints vbar (final velocity) and xbar (final position, default 0)."""
    n = tet.shape[0]
    g = np.zeros(2 * self.ne)
    vb0 = np.zeros((n, 3))
    xb0 = np.zeros((n, 3))
    ee, bb = _cplx(e_env), _cplx(b_env)
    ed = None if e_dc is None else _f64(e_dc)
    bd = None if b_dc is None else _f64(b_dc)
    xb = None if xbar is None else _f64(xbar)
    rc = _load().ora_vjp(self.h, n, _p(np.ascontiguousarray(tet, dtype=np.int32), _ip), _p(_f64(lam)),
                         _p(_f64(vel)), float(q), float(m), float(w), int(step0), int(nsteps), float(dt), float(omega),
                         _p(ee), _p(ed), _p(bb), _p(bd), _p(_f64(vbar)), _p(xb), _p(g), _p(vb0), _p(xb0),
                         int(nthreads))
    return rc, g[0::2] + 1j * g[1::2], vb0, xb0


OracleMesh.vjp = _vjp_method


def _jvp_method(self, tet, lam, vel, *, q, m, step0, nsteps, dt, omega, e_env, b_env, de, e_dc=None, b_dc=None,
                nthreads=1):
    """Tangent-linear derivative of nsteps steps from (tet, lam, vel) along the
    complex edge-envelope direction de: returns (status, dv[N,3], dx[N,3]), the
    derivatives of the final velocities and Cartesian positions."""
    n = tet.shape[0]
    dv = np.zeros((n, 3))
    dx = np.zeros((n, 3))
    ee, bb, dd = _cplx(e_env), _cplx(b_env), _cplx(de)
    ed = None if e_dc is None else _f64(e_dc)
    bd = None if b_dc is None else _f64(b_dc)
    rc = _load().ora_jvp(self.h, n, _p(np.ascontiguousarray(tet, dtype=np.int32), _ip), _p(_f64(lam)),
                         _p(_f64(vel)), float(q), float(m), int(step0), int(nsteps), float(dt), float(omega),
                         _p(ee), _p(ed), _p(bb), _p(bd), _p(dd), _p(dv), _p(dx), int(nthreads))
    return rc, dv, dx


OracleMesh.jvp = _jvp_method


class DsHistory:
    """Per-particle history of the downshifted integrator in the oracle's own
    layout: v[n, 3, 3] = v^{n-1}, v^{n-2}, v^{n-3}; e / b [n, 2, 9] = the field
    samples at t_{n-1}, t_{n-2}, each (Re[3], Im[3], dc[3])."""

    def __init__(self, n):
        self.v = np.zeros((n, 3, 3))
        self.e = np.zeros((n, 2, 9))
        self.b = np.zeros((n, 2, 9))

    def take(self, idx):
        h = DsHistory(0)
        h.v, h.e, h.b = (np.ascontiguousarray(a[idx]) for a in (self.v, self.e, self.b))
        return h


def ds_weights(K, t0, h, omega):
    """Weights of one downshifted step [t0, t0 + h] with K Lagrange nodes at
    t0, t0 - h, ...: dict of Mr, Mi, P [K] and Lr, Li, Q [K, K]."""
    out = {k: np.zeros(K) for k in ("Mr", "Mi", "P")}
    out.update({k: np.zeros((K, K)) for k in ("Lr", "Li", "Q")})
    _load().ora_ds_weights(int(K), float(t0), float(h), float(omega), _p(out["Mr"]), _p(out["Mi"]), _p(out["P"]),
                           _p(out["Lr"]), _p(out["Li"]), _p(out["Q"]))
    return out
