"""Pins of the oracle's downshifted integrator (Particle Push section, the
scheme that treats the carrier analytically inside the velocity update, with
fourth-order Adams-Bashforth positions, eq. newtons).

What fixes it independently of its own code: the carrier weights against the
integration-by-parts closed form of int t^p e^{jwt}; their w = 0 limit (the
Adams-Bashforth coefficients); exactness of the velocity update for envelopes
that are polynomials of degree <= 2 in time at any carrier step w h (the point
of the scheme); the cyclotron orbit (matrix exponential) at third order;
constant-acceleration positions (Adams-Bashforth is exact for polynomial
velocities); the specular wall mirroring the whole velocity history; the
discrete continuity law."""
import math

import numpy as np
import pytest
from scipy.linalg import expm

from paper_2208_12795_amd import synth

Q_E = -1.602176634e-19
M_E = 9.1093837015e-31
QM = Q_E / M_E
AB = {1: [1.0], 2: [1.5, -0.5], 3: [23 / 12, -16 / 12, 5 / 12], 4: [55 / 24, -59 / 24, 37 / 24, -9 / 24]}


def exp_moments(pmax, t0, h, omega):
    """int_0^h tau^p e^{jw(t0 + tau)} dtau for p = 0..pmax: by the recurrence
    I_p = [tau^p e^{jw tau}]_0^h / (jw) - p/(jw) I_{p-1} for w h >= 1, by the
    power series sum_m (jw)^m h^{p+m+1} / (m! (p+m+1)) below (the recurrence
    cancels there)."""
    jw = 1j * omega
    out = []
    for p in range(pmax + 1):
        if abs(omega * h) < 1.0:
            ip = sum((jw * h) ** m / math.factorial(m) * h ** (p + 1) / (p + m + 1) for m in range(40))
        elif p == 0:
            ip = (np.exp(jw * h) - 1.0) / jw
        else:
            ip = h ** p * np.exp(jw * h) / jw - p / jw * out[-1]
        out.append(ip)
    return np.exp(jw * t0) * np.array(out)


def lagrange_coeffs(K, h):
    """monomial coefficients (ascending) of the Lagrange basis on tau = 0, -h, -2h..."""
    nodes = -h * np.arange(K)
    V = np.vander(nodes, K, increasing=True)
    return np.linalg.inv(V).T          # row k: coefficients of N_k


@pytest.mark.parametrize("K", [1, 2, 3])
def test_weights_at_zero_frequency_are_adams_bashforth(ora, K):
    h = 1e-11
    w = ora.ds_weights(K, 3e-10, h, 0.0)
    assert np.allclose(w["P"] / h, AB[K], rtol=0, atol=1e-14)
    assert np.allclose(w["Mr"], w["P"], rtol=0, atol=1e-14 * h) and np.abs(w["Mi"]).max() == 0.0
    assert np.allclose(w["Lr"], w["Q"], rtol=0, atol=1e-14 * h) and np.abs(w["Li"]).max() == 0.0
    assert np.allclose(w["Q"], w["Q"].T, rtol=0, atol=1e-15 * h)
    assert np.allclose(w["Q"].sum(axis=1), w["P"], rtol=0, atol=1e-14 * h)   # partition of unity


@pytest.mark.parametrize("K", [2, 3])
@pytest.mark.parametrize("wh", [0.05, 1.0, 3.0])
def test_weights_match_closed_form(ora, K, wh):
    h, t0 = 1e-11, 7.3e-10
    omega = wh / h
    w = ora.ds_weights(K, t0, h, omega)
    C = lagrange_coeffs(K, h)
    mom = exp_moments(2 * K - 2, t0, h, omega)
    for k in range(K):
        ref = np.dot(C[k], mom[:K])                         # int N_k e^{jwt}
        assert abs(complex(w["Mr"][k], -w["Mi"][k]) - ref) <= 1e-12 * h
        for j in range(K):
            prod = np.convolve(C[j], C[k])                  # N_j N_k
            ref2 = np.dot(prod, mom[:len(prod)])
            assert abs(complex(w["Lr"][j, k], -w["Li"][j, k]) - ref2) <= 1e-12 * h


def uniform_edge_dofs(xyz, edges, vec):
    return (xyz[edges[:, 1]] - xyz[edges[:, 0]]) @ np.asarray(vec)


def uniform_face_dofs(xyz, faces, vec):
    a, b, c = xyz[faces[:, 0]], xyz[faces[:, 1]], xyz[faces[:, 2]]
    return 0.5 * np.cross(b - a, c - a) @ np.asarray(vec, dtype=np.float64)


class One:
    """One electron on the small jittered cube, driven through the oracle."""

    def __init__(self, ora, x0, v0):
        w = synth.make_workload(1, n_particles=10)
        self.M = ora.OracleMesh(w.xyz, w.tet_vert)
        self.xyz, self.tv = w.xyz, w.tet_vert
        self.edges, self.faces = self.M.edges(), self.M.faces()
        T, ml = self.M.locate(np.asarray(x0, float))
        assert ml > 0
        l4 = self.M.bary(T, np.asarray(x0, float))
        self.tet = np.array([T], np.int32)
        self.lam = np.ascontiguousarray(l4[1:][None, :])
        self.vel = np.asarray(v0, float)[None, :].copy()
        self.H = ora.DsHistory(1)
        self.dG = np.zeros(self.M.ne)

    def x(self):
        l = self.lam[0]
        return self.M.point(int(self.tet[0]), np.array([1 - l.sum(), *l]))

    def step(self, hist, t, h, omega, e_env, b_env, e_dc=None, b_dc=None):
        rc = self.M.ds_step(self.tet, self.lam, self.vel, self.H, hist=hist, q=Q_E, m=M_E, w=1.0, t=t, dt=h,
                            omega=omega, e_env=e_env, b_env=b_env, e_dc=e_dc, b_dc=b_dc, dG=self.dG)
        assert rc == 0


@pytest.mark.parametrize("degree", [0, 1, 2])
@pytest.mark.parametrize("wh", [0.3, 1.5])
def test_polynomial_envelope_velocity_is_exact_at_coarse_carrier_steps(ora, degree, wh):
    """Uniform field Re{g(t) E0 e^{jwt}} x with g a polynomial of degree <= 2:
    once the interpolation has degree+1 nodes, every velocity increment equals
    q/m int E dt to rounding, even with the carrier sampled only every w h =
    1.5 rad; the fine-step Boris update at the same step is off by O(1)."""
    h = 1e-11
    omega = wh / h
    coef = [1.0 + 0.5j, (0.3 - 0.2j) / (20 * h), (0.1 + 0.05j) / (20 * h) ** 2][: degree + 1]
    E0 = 1e3
    p = One(ora, (0.5, 0.5, 0.5), (1e4, -5e3, 2e3))
    unit = uniform_edge_dofs(p.xyz, p.edges, (1.0, 0.0, 0.0))
    zero_b = np.zeros(p.M.nf, complex)
    for n in range(8):
        t = n * h
        g = sum(c * t ** i for i, c in enumerate(coef))
        v_before = p.vel[0].copy()
        p.step(min(n, 3), t, h, omega, E0 * g * unit, zero_b)
        dv = p.vel[0] - v_before
        mom = exp_moments(len(coef) - 1, t, h, omega)
        exact = QM * E0 * np.real(sum(c * sum(math.comb(i, r) * t ** (i - r) * mom[r] for r in range(i + 1))
                                      for i, c in enumerate(coef)))
        if n >= degree:
            assert abs(dv[0] - exact) <= 1e-11 * abs(QM * E0 * h), (n, dv[0], exact)
            assert abs(dv[1]) + abs(dv[2]) <= 1e-11 * abs(QM * E0 * h)
        if n == degree + 1 and wh > 1.0:
            Eb = E0 * np.real(g * np.exp(1j * omega * t))   # fine-step scheme: field sampled at t_n
            assert abs(QM * Eb * h - exact) > 0.05 * abs(exact)


@pytest.mark.parametrize("wh_cyc", [0.1])
def test_cyclotron_third_order(ora, wh_cyc):
    """Uniform B = B0 z (dc face DoFs), E = 0, exact history from the orbit:
    the velocity error after a fixed time falls as h^3 (ratio ~8 per halving)."""
    B0 = 0.1
    Om = QM * B0
    A = np.array([[0.0, Om, 0.0], [-Om, 0.0, 0.0], [0.0, 0.0, 0.0]])     # dv/dt = (q/m) v x B
    v0 = np.array([1e5, 3e4, 2e4])
    errs = []
    for refine in (1, 2, 4):
        h = wh_cyc / abs(Om) / refine
        p = One(ora, (0.5, 0.5, 0.5), v0)
        bdc = uniform_face_dofs(p.xyz, p.faces, (0.0, 0.0, B0))
        zero_e = np.zeros(p.M.ne, complex)
        zero_b = np.zeros(p.M.nf, complex)
        for j in range(3):
            p.H.v[0, j] = expm(A * (-(j + 1) * h)) @ v0
            p.H.b[0, min(j, 1), 6:9] = (0.0, 0.0, B0)
        nsteps = 20 * refine
        for n in range(nsteps):
            p.step(3, n * h, h, 0.0, zero_e, zero_b, b_dc=bdc)
        errs.append(np.abs(p.vel[0] - expm(A * nsteps * h) @ v0).max() / np.abs(v0).max())
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 6.0 < r1 < 10.5 and 6.0 < r2 < 10.5, errs


def test_constant_acceleration_positions_are_exact(ora):
    """Uniform dc E (ω plays no part), B = 0, exact velocity history: the
    Adams-Bashforth positions reproduce x0 + v0 t + a t^2 / 2."""
    h = 2e-11
    Evec = np.array([300.0, -200.0, 100.0])
    a = QM * Evec
    x0, v0 = np.array([0.45, 0.52, 0.48]), np.array([2e4, 1e4, -3e4])
    p = One(ora, x0, v0)
    edc = uniform_edge_dofs(p.xyz, p.edges, Evec)
    for j in range(3):
        p.H.v[0, j] = v0 - a * (j + 1) * h
        p.H.e[0, min(j, 1), 6:9] = Evec
    zero_e = np.zeros(p.M.ne, complex)
    zero_b = np.zeros(p.M.nf, complex)
    for n in range(12):
        p.step(3, n * h, h, 7e10, zero_e, zero_b, e_dc=edc)
        t = (n + 1) * h
        assert np.abs(p.vel[0] - (v0 + a * t)).max() <= 1e-12 * np.abs(a * t).max()
        disp = v0 * t + 0.5 * a * t * t
        assert np.abs(p.x() - (x0 + disp)).max() <= 1e-9 * np.abs(disp).max() + 1e-15


def test_wall_mirrors_the_velocity_history(ora):
    """No field, constant velocity towards the wall x = 0: after the bounce the
    path is the mirror image of the straight line, which needs the stored
    velocities to be mirrored too (else Adams-Bashforth mixes the two)."""
    h = 1e-9
    v0 = np.array([-2e6, 3e5, 1e5])
    x0 = np.array([0.004, 0.5, 0.5])
    p = One(ora, x0, v0)
    for j in range(3):
        p.H.v[0, j] = v0
    zero_e = np.zeros(p.M.ne, complex)
    zero_b = np.zeros(p.M.nf, complex)
    for n in range(6):
        p.step(3, n * h, h, 0.0, zero_e, zero_b)
        free = x0 + v0 * (n + 1) * h
        mirrored = np.array([abs(free[0]), free[1], free[2]])
        assert np.abs(p.x() - mirrored).max() <= 1e-14
    assert p.vel[0][0] > 0 and np.allclose(p.H.v[0, :, 0], -v0[0])


def test_ramp_up_first_step_is_euler(ora):
    """hist = 0: one node and first-order Adams-Bashforth, i.e.
    v1 = v0 + q/m int Re{E(x0) e^{jwt}} dt over the step, x1 = x0 + h v0."""
    w = synth.make_workload(1, n_particles=50)
    M = ora.OracleMesh(w.xyz, w.tet_vert)
    H = ora.DsHistory(50)
    tet, lam, vel = w.tet.copy(), w.lam.copy(), w.vel.copy()
    x0 = M.positions(tet, lam)
    t, h = 4e-10, w.dt
    dG = np.zeros(M.ne)
    assert M.ds_step(tet, lam, vel, H, hist=0, q=w.q, m=w.m, w=w.w, t=t, dt=h, omega=w.omega, e_env=w.e_env,
                     b_env=w.b_env, b_dc=w.b_dc, dG=dG) == 0
    mom = exp_moments(0, t, h, w.omega)[0]
    ze, zb = np.zeros(M.ne, complex), np.zeros(M.nf, complex)
    for i in range(50):
        l4 = np.array([1 - w.lam[i].sum(), *w.lam[i]])
        # envelope parts at x0 from the physical-field routine at zero phase
        Er = M.fields(w.tet[i], l4, 0.0, 0.0, w.e_env.real + 0j, zb)[0]
        Ei = M.fields(w.tet[i], l4, 0.0, 0.0, w.e_env.imag + 0j, zb)[0]
        Br = M.fields(w.tet[i], l4, 0.0, 0.0, ze, w.b_env.real + 0j)[1]
        Bi = M.fields(w.tet[i], l4, 0.0, 0.0, ze, w.b_env.imag + 0j)[1]
        Bd = M.fields(w.tet[i], l4, 0.0, 0.0, ze, zb, b_dc=w.b_dc)[1]
        Eint = Er * mom.real - Ei * mom.imag
        Bint = Br * mom.real - Bi * mom.imag + Bd * h
        ref = w.vel[i] + w.q / w.m * (Eint + np.cross(w.vel[i], Bint))
        assert np.abs(vel[i] - ref).max() <= 1e-12 * np.abs(ref - w.vel[i]).max()
    x1 = M.positions(tet, lam)
    assert np.abs(x1 - (x0 + h * w.vel)).max() <= 1e-15


def test_continuity_of_downshifted_steps(ora):
    """D^T dG = rho_end - rho_start for each of 6 downshifted steps (ramp
    included) of the small workload."""
    w = synth.make_workload(1)
    M = ora.OracleMesh(w.xyz, w.tet_vert)
    H = ora.DsHistory(w.tet.shape[0])
    tet, lam, vel = w.tet.copy(), w.lam.copy(), w.vel.copy()
    for n in range(6):
        rho0 = M.charge(tet, lam, w.q, w.w)
        dG, rho1 = np.zeros(M.ne), np.zeros(M.nv)
        assert M.ds_step(tet, lam, vel, H, hist=min(n, 3), q=w.q, m=w.m, w=w.w, t=n * w.dt, dt=w.dt,
                         omega=w.omega, e_env=w.e_env, b_env=w.b_env, b_dc=w.b_dc, dG=dG, rho=rho1) == 0
        r, p = M.gauss(dG, rho1, rho0)
        assert r / p < 1e-13


def test_lower_oversampling_than_the_fine_step_scheme(ora):
    """The trend the Particle Push section reports for this scheme: at equal
    accuracy of the path (hence of G), fewer steps per carrier period than the
    fine-step scheme that samples the modulated field.  One electron in the
    uniform field Re{(c0 + c1 t) E0 e^{jwt}} x (10 GHz), B = 0, both schemes
    started on the exact trajectory (leapfrog v^{-1/2}; downshifted history at
    t_{-1..-3}), position error after 10.37 periods against the closed form:
    fourth order for the downshifted scheme, second order for the fine-step
    Boris scheme; the downshifted scheme at 24 steps per period beats the
    fine-step one at 64."""
    f = 10e9
    om, Tper, E0 = 2 * np.pi * f, 1.0 / f, 1e4
    v0, Edir = np.array([1e5, 2e4, -3e4]), np.array([1.0, 0.0, 0.0])
    c0, c1 = 1.0 + 0.3j, (0.4 - 0.2j) / (20 * Tper)
    jw = 1j * om
    acc = QM * E0 * Edir

    def g(t):
        return c0 + c1 * t

    def iv(t):      # int_0^t g(s) e^{jws} ds
        e = np.exp(jw * t)
        return c0 * (e - 1) / jw + c1 * (t * e / jw - (e - 1) / jw ** 2)

    def ix(t):      # int_0^t iv(u) du
        e = np.exp(jw * t)
        ie, iue = (e - 1) / jw, t * e / jw - (e - 1) / jw ** 2
        return c0 * (ie - t) / jw + c1 * (iue / jw - ie / jw ** 2 + t / jw ** 2)

    def vex(t):
        return v0 + acc * np.real(iv(t))

    def xex(t):
        return v0 * t + acc * np.real(ix(t))

    err = {}
    for M in (8, 16, 24, 32, 64):
        h = Tper / M
        n = int(round(10.37 * M))
        for scheme in ("fine", "ds"):
            p = One(ora, (0.5, 0.5, 0.5), v0)
            unit = uniform_edge_dofs(p.xyz, p.edges, Edir)
            zb = np.zeros(p.M.nf, complex)
            x0 = p.x()
            if scheme == "ds":
                for j in range(3):
                    p.H.v[0, j] = vex(-(j + 1) * h)
                for j in range(2):
                    gj = g(-(j + 1) * h) * E0
                    p.H.e[0, j, 0:3] = np.real(gj) * Edir
                    p.H.e[0, j, 3:6] = np.imag(gj) * Edir
                for k in range(n):
                    p.step(3, k * h, h, om, E0 * g(k * h) * unit, zb)
            else:
                p.vel[0] = vex(-h / 2)
                for k in range(n):
                    rc, _ = p.M.step(p.tet, p.lam, p.vel, q=Q_E, m=M_E, w=1.0, step=k, dt=h, omega=om,
                                     e_env=E0 * g(k * h) * unit, b_env=zb, dG=p.dG)
                    assert rc == 0
            ref = xex(n * h)
            err[scheme, M] = np.abs((p.x() - x0) - ref).max() / np.abs(ref).max()
    print("position error vs steps per period:",
          {M: (f"{err['fine', M]:.2e}", f"{err['ds', M]:.2e}") for M in (8, 16, 24, 32, 64)})
    assert err["ds", 32] / err["ds", 64] > 10.0                 # fourth order
    assert err["ds", 64] < err["fine", 64] / 20.0
    assert err["ds", 24] < err["fine", 64]                      # ~2.7x fewer steps for the same accuracy
