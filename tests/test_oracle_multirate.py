"""Pins of the oracle's coarse field step at the fine step: envelope snapshots
at three coarse times reconstructed at each fine time with the quadratic
Lagrange basis (eqs. newmark_L / newmark_N), fine Lorentz steps, path
integrals summed over the fine steps (eq. G_integral)."""
import numpy as np
import pytest

from paper_2208_12795_amd import synth


def run_fine(M, w, tet, lam, vel, times, dt, envs, dG):
    t, l, v = tet.copy(), lam.copy(), vel.copy()
    for ti, (e, b) in zip(times, envs):
        rc = M.step_at(t, l, v, q=w.q, m=w.m, w=w.w, t=ti, dt=dt, omega=w.omega, e_env=e, b_env=b, b_dc=w.b_dc,
                       dG=dG)
        assert rc == 0
    return t, l, v


def coarse(M, w, snaps, t_c, dtc, fine, dG, rho=None):
    t, l, v = w.tet.copy(), w.lam.copy(), w.vel.copy()
    rc = M.coarse_step(t, l, v, q=w.q, m=w.m, w=w.w, e_snaps=[s[0] for s in snaps], b_snaps=[s[1] for s in snaps],
                       t_coarse=t_c, dt_coarse=dtc, fine_steps=fine, omega=w.omega, b_dc=w.b_dc, dG=dG, rho=rho)
    assert rc == 0
    return t, l, v


@pytest.mark.parametrize("degree", [0, 1, 2])
def test_polynomial_envelopes_are_reproduced(ora, degree):
    """Snapshots sampled from an envelope polynomial in time of degree <= 2:
    the reconstruction is exact, so the coarse step equals fine steps with the
    exact envelope at every fine time."""
    w = synth.make_workload(1, n_particles=400)
    M = ora.OracleMesh(w.xyz, w.tet_vert)
    (a_e, a_b), (b_e, b_b), (c_e, c_b) = synth.envelope_snapshots(w, seed=3)
    coeffs = [(a_e, a_b), (b_e - a_e, b_b - a_b), (c_e - a_e, c_b - a_b)][: degree + 1]
    dtc, fine = 8 * w.dt, 8
    t_c = 40 * w.dt

    def env(t):
        x = (t - t_c) / dtc
        return (sum(ce * x ** i for i, (ce, _) in enumerate(coeffs)), sum(cb * x ** i for i, (_, cb) in enumerate(coeffs)))

    snaps = [env(t_c - dtc), env(t_c), env(t_c + dtc)]
    dG1 = np.zeros(M.ne)
    got = coarse(M, w, snaps, t_c, dtc, fine, dG1)
    dt = dtc / fine
    times = [t_c + j * dt for j in range(fine)]
    dG2 = np.zeros(M.ne)
    ref = run_fine(M, w, w.tet, w.lam, w.vel, times, dt, [env(t) for t in times], dG2)
    assert np.array_equal(got[0], ref[0])
    assert np.abs(got[1] - ref[1]).max() < 1e-13
    assert np.abs(got[2] - ref[2]).max() < 1e-13 * np.abs(ref[2]).max()
    assert np.abs(dG1 - dG2).max() < 1e-13 * np.abs(dG2).max()


def test_node_times_pick_the_snapshots(ora):
    """At the node time t_coarse the reconstruction is the middle snapshot: a
    coarse step with one fine step equals one step with snapshot 1."""
    w = synth.make_workload(1, n_particles=300)
    M = ora.OracleMesh(w.xyz, w.tet_vert)
    snaps = synth.envelope_snapshots(w, seed=5)
    t_c, dtc = 13 * w.dt, w.dt
    dG1, dG2 = np.zeros(M.ne), np.zeros(M.ne)
    got = coarse(M, w, snaps, t_c, dtc, 1, dG1)
    ref = run_fine(M, w, w.tet, w.lam, w.vel, [t_c], dtc, [snaps[1]], dG2)
    for a, b in zip(got, ref):
        assert np.array_equal(a, b)
    assert np.array_equal(dG1, dG2)


def test_coarse_step_conserves_charge(ora):
    """The summed path integrals of the fine steps satisfy the discrete
    continuity law over the coarse step: D^T G = rho(end) - rho(start)."""
    w = synth.make_workload(1, n_particles=1000)
    M = ora.OracleMesh(w.xyz, w.tet_vert)
    snaps = synth.envelope_snapshots(w, seed=7)
    rho0 = M.charge(w.tet, w.lam, w.q, w.w)
    dG, rho1 = np.zeros(M.ne), np.zeros(M.nv)
    coarse(M, w, snaps, 20 * w.dt, 10 * w.dt, 10, dG, rho1)
    r, p = M.gauss(dG, rho1, rho0)
    assert r / p < 1e-13
