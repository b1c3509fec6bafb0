"""The cold-plasma loop of the tests (particles in the field of their own
charge, closed through the non-solenoidal solve) run with the oracle, and
the frequency fit of its recorded signal."""
import os

import numpy as np

NTH = max(1, min(16, os.cpu_count() or 1))


def mode_shape(cp, edges):
    """Edge coefficients of -grad psi (psi(tail) - psi(head)): the field of
    the oscillating mode per unit potential amplitude."""
    k = np.pi / cp.extent[0]
    x = cp.xyz
    psi = np.sin(k * x[:, 0]) * np.sin(k * x[:, 1]) * np.sin(k * x[:, 2])
    return psi[edges[:, 0]] - psi[edges[:, 1]]


def mode_amplitude(e_real, shape):
    """Least-squares amplitude of the mode shape in the edge field."""
    return float(e_real @ shape / (shape @ shape))


def oracle_loop(ora, cp, nsteps, dt, shape, omega=0.0, record=None, per=1):
    """nsteps oracle steps of the plasma cp in the field solved from the
    background-neutralised charge every `per` steps (held in between, as real
    unmodulated edge DoFs).  Returns (states, G, signal, rho0): states[j] =
    (tet, lam, vel, G) after step j (for j in record, all if None), signal[j]
    = the mode amplitude of the field used at step j."""
    from oracle import gauss
    m = ora.OracleMesh(cp.xyz, cp.tet_vert)
    ns = gauss.NsOracle(m, 8.8541878128e-12)
    rho0 = m.charge(cp.tet, cp.lam, cp.q, cp.w) - m.charge(cp.tet0, cp.lam0, cp.q, cp.w)
    t, l, v = cp.tet.copy(), cp.lam.copy(), cp.vel.copy()
    G = np.zeros(m.ne)
    ez = np.zeros(m.ne, complex)
    bz = np.zeros(m.nf, complex)
    states, sig = [], []
    for j in range(nsteps):
        if j % per == 0:
            _, e = ns.solve(G=G, rho0=rho0)
            edc = e.real.copy()
        sig.append(mode_amplitude(edc, shape))
        rc, _ = m.step(t, l, v, q=cp.q, m=cp.m, w=cp.w, step=j, dt=dt, omega=omega, e_env=ez, b_env=bz, e_dc=edc,
                       dG=G, nthreads=NTH)
        assert rc == 0
        if record is None or j in record:
            states.append((t.copy(), l.copy(), v.copy(), G.copy()))
    return states, G, np.array(sig), rho0


def fit_frequency(sig, dt, w0, span=0.1, n=4001):
    """omega of the least-squares fit A cos(wt) + B sin(wt) + C, scanned over
    w0 (1 +- span)."""
    t = np.arange(len(sig)) * dt
    best = None
    for om in np.linspace((1 - span) * w0, (1 + span) * w0, n):
        A = np.stack([np.cos(om * t), np.sin(om * t), np.ones_like(t)], axis=1)
        c = np.linalg.lstsq(A, sig, rcond=None)[0]
        r = np.sum((A @ c - sig) ** 2)
        if best is None or r < best[0]:
            best = (r, om, c)
    return best[1], best[2]


def oracle_em_loop(ora, cp, nsteps, dt, shape, correct=True, record=None, split=False):
    """The loop through the implicit field step: each step pushes the
    particles in the current fields (e, b), takes the field step to the next
    time with the source G'' from the second difference of the running path
    integral, and (correct) replaces the new field's gradient part so that
    Gauss' law holds exactly for the deposited charge.  split: the field step
    takes the solenoidal source P^T G'' instead and starts from the
    solenoidal part of the initial field, and e = u + the field of eq.
    ns_equation (the two halves of the split summed).  omega = 0.  Returns
    (states, signal, gauss): states[j] = (tet, lam, vel, G) after step j (for
    j in record, all if None), signal[j] the mode amplitude of e used at step
    j, gauss[j] = max |D^T [*eps] e + (D^T G + rho0)| / max |D^T G + rho0| at
    the inner nodes after the field step j."""
    from oracle import field, gauss
    eps0, mu0 = 8.8541878128e-12, 1.25663706212e-6
    m = ora.OracleMesh(cp.xyz, cp.tet_vert)
    ns = gauss.NsOracle(m, eps0)
    F = field.FieldOracle(m, dt, 0.0, eps0, mu0)
    rho0 = m.charge(cp.tet, cp.lam, cp.q, cp.w) - m.charge(cp.tet0, cp.lam0, cp.q, cp.w)
    t, l, v = cp.tet.copy(), cp.lam.copy(), cp.vel.copy()
    G = np.zeros(m.ne)
    G_prev = np.zeros(m.ne)
    e = ns.correct(np.zeros(m.ne, complex), None, rho0)       # the static start: Gauss for rho0
    u, vv, a = (ns.solenoidal_part(e) if split else e.copy()), np.zeros(m.ne, complex), np.zeros(m.ne, complex)
    b = np.zeros(m.nf, complex)
    states, sig, gres = [], [], []
    for j in range(nsteps):
        sig.append(mode_amplitude(e.real, shape))
        G_old = G.copy()
        rc, _ = m.step(t, l, v, q=cp.q, m=cp.m, w=cp.w, step=j, dt=dt, omega=0.0, e_env=e, b_env=b, dG=G,
                       nthreads=NTH)
        assert rc == 0
        gdd = (G - 2 * G_old + G_prev) / dt ** 2
        G_prev = G_old
        if split:
            u, vv, a, b = F.step((j + 1) * dt, u, vv, a, b, ns.solenoidal_source(gdd))
            e = u + ns.solve(G, rho0)[1]
        else:
            u, vv, a, b = F.step((j + 1) * dt, u, vv, a, b, gdd)
            e = ns.correct(u, G, rho0) if correct else u
        r, scale = ns.gauss_residual(e, G, rho0)
        gres.append(r / scale)
        if record is None or j in record:
            states.append((t.copy(), l.copy(), v.copy(), G.copy()))
    return states, np.array(sig), np.array(gres)
