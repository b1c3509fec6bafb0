"""Pins of the oracle of the non-solenoidal (Gauss-law) field solve: the
operator against the textbook linear-element stiffness, a manufactured Poisson
problem converging at second order, Gauss' theorem on the wall, the discrete
maximum principle, and the field of moved charge equal to the field of the
charge where it ends; and the cold-plasma oscillation of the loop closed
through the solve."""
import os
import sys

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2208_12795_amd import synth

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

EPS0 = 8.8541878128e-12
NTH = max(1, min(16, os.cpu_count() or 1))


def p1_stiffness(xyz, tv, eps):
    """eps int grad l_i . grad l_j from the inverse of each tet's [1 x y z] matrix."""
    nv = xyz.shape[0]
    rows, cols, vals = [], [], []
    for t in range(tv.shape[0]):
        A = np.ones((4, 4))
        A[1:, :] = xyz[tv[t]].T
        inv = np.linalg.inv(A)
        g = inv[:, 1:]                      # row k: grad of the hat function of vertex k
        V = abs(np.linalg.det(A)) / 6.0
        loc = eps * V * g @ g.T
        rows.append(np.repeat(tv[t], 4))
        cols.append(np.tile(tv[t], 4))
        vals.append(loc.ravel())
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(nv, nv))


@pytest.fixture(scope="module")
def jittered(ora):
    xyz, tv = synth.kuhn_mesh((4, 3, 5), (1.0, 0.8, 1.2), 0.15, np.random.default_rng(8))
    return ora.OracleMesh(xyz, tv)


def test_operator_is_linear_element_stiffness(jittered):
    """D^T [*eps] D (edge mass by quadrature, incidence) equals the nodal
    stiffness eps int grad W0_i . grad W0_j, and constants are in its kernel."""
    from oracle import gauss
    ns = gauss.NsOracle(jittered, EPS0)
    ref = p1_stiffness(jittered.xyz, jittered.tv, EPS0)
    assert abs(ns.S - ref).max() <= 1e-12 * abs(ref).max()
    assert np.abs(ns.S @ np.ones(jittered.nv)).max() <= 1e-12 * abs(ref).max()
    # wall nodes of the box are exactly those on its faces
    x = jittered.xyz
    on_box = (np.isclose(x[:, 0], 0) | np.isclose(x[:, 0], 1.0) | np.isclose(x[:, 1], 0) | np.isclose(x[:, 1], 0.8)
              | np.isclose(x[:, 2], 0) | np.isclose(x[:, 2], 1.2))
    assert np.array_equal(ns.wall, on_box)


def test_round_trip_of_a_potential(jittered):
    """G = -[*eps] D y for a potential y that vanishes on the wall makes
    D^T G = -D^T [*eps] D y, so the solve returns y (times the carrier phase)."""
    from oracle import gauss
    ns = gauss.NsOracle(jittered, EPS0)
    rng = np.random.default_rng(4)
    y = rng.standard_normal(jittered.nv) * ~ns.wall
    G = -(ns.M @ (ns.D @ y))
    t, w = 3.1e-10, 2 * np.pi * 1.7e9
    x, e = ns.solve(G, t=t, omega=w)
    ph = np.exp(-1j * w * t)
    assert np.abs(x - y * ph).max() <= 1e-10 * np.abs(y).max()
    assert np.abs(e - (ns.D @ y) * ph).max() <= 1e-10 * np.abs(ns.D @ y).max()
    r, scale = ns.gauss_residual(e, G, t=t, omega=w)
    assert r <= 1e-12 * scale


def load_vector(mesh, f):
    """b_i = int f W0_i with the 4-point rule (exact for quadratics)."""
    from oracle import field
    _, vol = field.tet_gradients(mesh.xyz, mesh.tv)
    b = np.zeros(mesh.nv)
    r = mesh.xyz[mesh.tv]                                  # [N_t, 4, 3]
    for lam in field.QPTS:
        xq = np.einsum("k,tka->ta", lam, r)
        fq = f(xq) * vol / 4.0
        for k in range(4):
            np.add.at(b, mesh.tv[:, k], fq * lam[k])
    return b


def test_manufactured_poisson_second_order(ora):
    """-div(eps grad phi) = rho with phi = sin(pi x) sin(pi y) sin(pi z) on the
    grounded unit cube: E = -grad phi, so the solve of -rho returns -phi at
    the nodes, with an error that falls about 4x per halving of h; the edge
    coefficients approach the line integrals of E."""
    from oracle import gauss
    phi = lambda x: np.sin(np.pi * x[:, 0]) * np.sin(np.pi * x[:, 1]) * np.sin(np.pi * x[:, 2])
    rho = lambda x: 3 * np.pi ** 2 * EPS0 * phi(x)
    errs, eerrs = [], []
    for n in (4, 8, 16):
        xyz, tv = synth.kuhn_mesh((n, n, n), (1.0, 1.0, 1.0), 0.0)
        m = ora.OracleMesh(xyz, tv)
        ns = gauss.NsOracle(m, EPS0)
        x, e = ns.solve(rho0=load_vector(m, rho))
        assert np.abs(x.imag).max() == 0.0
        errs.append(np.abs(x.real + phi(xyz)).max())
        # line integral of E = -grad phi along each edge: phi(tail) - phi(head)
        ed = m.edges()
        exact = phi(xyz[ed[:, 0]]) - phi(xyz[ed[:, 1]])
        eerrs.append(np.abs(e.real - exact).max() / np.abs(exact).max())
    rate = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    erate = np.log2(np.array(eerrs[:-1]) / np.array(eerrs[1:]))
    assert rate.min() > 1.8, (errs, rate)
    assert erate.min() > 1.5, (eerrs, erate)
    assert errs[-1] < 1e-2


def test_point_charge_gauss_theorem_and_maximum_principle(ora):
    """A positive charge inside the grounded box: the potential -x is positive
    at every inner node and largest at a vertex of the charge's tet, and the
    flux leaving through the wall, sum over wall nodes of D^T [*eps] e, is the
    charge."""
    from oracle import gauss
    xyz, tv = synth.kuhn_mesh((6, 5, 7), (1.0, 1.0, 1.0), 0.0)
    m = ora.OracleMesh(xyz, tv)
    ns = gauss.NsOracle(m, EPS0)
    T = int(np.flatnonzero((xyz[tv].mean(axis=1) > 0.4).all(axis=1))[0])
    lam = np.array([[0.2, 0.3, 0.1]])
    q, wgt = 1.602e-19, 1e4
    rho = m.charge(np.array([T], dtype=np.int32), lam, q, wgt)
    x, e = ns.solve(rho0=rho)
    pot = -x.real
    assert pot[ns.inner].min() > 0.0
    assert pot.argmax() in set(tv[T].tolist())
    flux = ns.D.T @ (ns.M @ e.real)
    assert np.isclose(flux[ns.wall].sum(), q * wgt, rtol=1e-10)


def test_moved_charge_field_equals_field_of_charge_at_its_end(ora):
    """Electrons pushed by the oracle's step (no field, fast enough that most
    change tet) deposit G; the solve from the starting charge plus D^T G is
    the solve of the charge where the particles end (exact charge
    conservation of the split, Discrete System)."""
    from oracle import gauss
    w = synth.make_workload(1, n_particles=300)
    m = ora.OracleMesh(w.xyz, w.tet_vert)
    ns = gauss.NsOracle(m, EPS0)
    rho_a = m.charge(w.tet, w.lam, w.q, w.w)
    t, l, v = w.tet.copy(), w.lam.copy(), w.vel * 200.0
    dG = np.zeros(m.ne)
    rc, _ = m.step(t, l, v, q=w.q, m=w.m, w=w.w, step=0, dt=2e-9, omega=w.omega, e_env=np.zeros_like(w.e_env),
                   b_env=np.zeros_like(w.b_env), dG=dG, nthreads=NTH)
    assert rc == 0 and (t != w.tet).mean() > 0.3
    rho_b = m.charge(t, l, w.q, w.w)
    ta, wa = 1.3e-9, w.omega
    x1, e1 = ns.solve(G=dG, rho0=rho_a, t=ta, omega=wa)
    x2, e2 = ns.solve(rho0=rho_b, t=ta, omega=wa)
    assert np.abs(x1 - x2).max() <= 1e-11 * np.abs(x2).max()
    assert np.abs(e1 - e2).max() <= 1e-11 * np.abs(e2).max()


def test_cold_plasma_oscillation(ora):
    """The loop field -> particles -> G -> field closed through the solve:
    electrons displaced by xi = a grad psi (psi = sin sin sin, grounded box)
    over a neutralising background.  In the continuum the potential is
    phi = n q a psi / eps (negative for electrons pushed towards the centre)
    and every electron oscillates at the plasma frequency
    omega_p = sqrt(n q^2 / (eps m)).  The oracle's loop (omega_p dt = 0.1,
    two periods) oscillates at omega_p to 1 %, with a mode amplitude that
    approaches n q a / eps at second order in the cell size."""
    import plasma_util as P
    ratios = {}
    for n in (4, 8):
        cp = synth.cold_plasma(n, 50_000)
        shape = P.mode_shape(cp, synth.mesh_edges(cp.tet_vert, cp.xyz.shape[0]))
        dt = 0.1 / cp.omega_p
        _, _, sig, _ = P.oracle_loop(ora, cp, 126, dt, shape, record=[])
        om, _ = P.fit_frequency(sig, dt, cp.omega_p)
        assert abs(om / cp.omega_p - 1) < 0.01, (n, om / cp.omega_p)
        phi0 = cp.density * cp.q * cp.a / EPS0
        ratios[n] = sig[0] / phi0
    assert 0.85 < ratios[4] < ratios[8] < 1.0, ratios
    assert (1 - ratios[4]) / (1 - ratios[8]) > 3.0, ratios


def test_structured_mesh_gives_the_seven_point_stencil(ora):
    """On the unjittered Kuhn (Freudenthal) grid the linear-element stiffness
    is the 7-point Laplacian: eps h (6 on the diagonal, -1 for the six axis
    neighbours, 0 for the others).  With one inner node (2^3 cells) the solve
    is x = -rho / (6 eps h) in closed form."""
    from oracle import gauss
    n, h = 4, 0.25
    xyz, tv = synth.kuhn_mesh((n, n, n), (1.0, 1.0, 1.0), 0.0)
    m = ora.OracleMesh(xyz, tv)
    S = gauss.NsOracle(m, EPS0).S.toarray() / (EPS0 * h)
    d = xyz[:, None, :] - xyz[None, :, :]
    axis = (np.abs(np.abs(d).sum(axis=2) - h) < 1e-12) & ((np.abs(d) > 1e-12).sum(axis=2) == 1)
    inner = ~gauss.wall_nodes(m)
    for i in np.flatnonzero(inner):
        ref = -axis[i].astype(float)
        ref[i] = 6.0
        assert np.abs(S[i] - ref).max() < 1e-12, i
    xyz, tv = synth.kuhn_mesh((2, 2, 2), (1.0, 1.0, 1.0), 0.0)
    m = ora.OracleMesh(xyz, tv)
    c = int(np.argmin(((xyz - 0.5) ** 2).sum(axis=1)))
    rho = np.zeros(m.nv)
    rho[c] = 1e-12
    x, _ = gauss.NsOracle(m, EPS0).solve(rho0=rho)
    assert np.isclose(x[c].real, -1e-12 / (6 * EPS0 * 0.5), rtol=1e-14)
    assert np.count_nonzero(x) == 1


def test_gauss_correction_of_a_field_step_state(ora, jittered):
    """The correction e = u + D y: Gauss' law exact for e, the curl of e that
    of u, a pure gradient removed, a field that already obeys Gauss left
    alone.  And the motivation (Quasi Helmholtz section): the plain Newmark
    field step carries a gradient part along untouched by the curl-curl
    stiffness, so a gradient in the initial velocity makes D^T [*eps] u grow
    exactly linearly in time (20 source-free steps); the correction removes
    it at every step."""
    from oracle import field, gauss, qh
    ns = gauss.NsOracle(jittered, EPS0)
    rng = np.random.default_rng(21)
    M, K, bnd = field.assemble(jittered, EPS0, 1.25663706212e-6)
    inner_e = ~bnd
    u = (rng.standard_normal(jittered.ne) + 1j * rng.standard_normal(jittered.ne)) * inner_e
    G = rng.standard_normal(jittered.ne) * 1e-15
    rho0 = rng.standard_normal(jittered.nv) * 1e-15
    t, w = 2.1e-10, 2 * np.pi * 1.1e9
    e = ns.correct(u, G, rho0, t, w)
    r, scale = ns.gauss_residual(e, G, rho0, t, w)
    assert r <= 1e-12 * scale
    C = qh.curl_incidence(jittered)
    assert np.abs(C @ (e - u)).max() <= 1e-12 * np.abs(C @ u).max()
    phi = rng.standard_normal(jittered.nv) * ~ns.wall
    assert np.abs(ns.correct(ns.D @ phi)).max() <= 1e-10 * np.abs(ns.D @ phi).max()
    _, e_ns = ns.solve(G, rho0, t, w)
    assert np.abs(ns.correct(e_ns, G, rho0, t, w) - e_ns).max() <= 1e-10 * np.abs(e_ns).max()
    # null-space growth of the plain step, removed by the correction
    F = field.FieldOracle(jittered, 1e-11, 0.0, EPS0, 1.25663706212e-6)
    u0 = np.zeros(jittered.ne, complex)
    v0 = (ns.D @ phi) * 1e9 * inner_e                      # a gradient velocity only
    a0 = np.zeros_like(u0)
    b0 = np.zeros(jittered.nf, complex)
    uu, vv, aa, bb = u0, v0, a0, b0
    I = ns.inner
    g0 = (ns.D.T @ (ns.M @ v0))[I]
    for n in range(1, 21):
        uu, vv, aa, bb = F.step(n * 1e-11, uu, vv, aa, bb)
        div = (ns.D.T @ (ns.M @ uu))[I]
        assert np.abs(div - n * 1e-11 * g0).max() <= 1e-9 * np.abs(n * 1e-11 * g0).max()
        assert np.abs(ns.D.T @ (ns.M @ ns.correct(uu)))[I].max() <= 1e-12 * np.abs(div).max()


def test_em_loop_with_gauss_correction(ora):
    """The loop through the implicit field step (Newmark, source G'' from the
    path integral's second difference, a step behind): corrected every step,
    Gauss' law holds to rounding and the cold plasma oscillates at omega_p to
    1 %; left plain, the lagged source breaks Gauss' law by order one."""
    import plasma_util as P
    cp = synth.cold_plasma(4, 50_000)
    shape = P.mode_shape(cp, synth.mesh_edges(cp.tet_vert, cp.xyz.shape[0]))
    dt = 0.1 / cp.omega_p
    _, sig, gres = P.oracle_em_loop(ora, cp, 126, dt, shape, correct=True, record=[])
    om, _ = P.fit_frequency(sig, dt, cp.omega_p)
    assert abs(om / cp.omega_p - 1) < 0.01, om / cp.omega_p
    assert gres.max() < 1e-12, gres.max()
    _, _, gplain = P.oracle_em_loop(ora, cp, 40, dt, shape, correct=False, record=[])
    assert gplain.max() > 1e-2, gplain.max()


def test_solenoidal_projector_and_source(jittered):
    """The projector of the split in the [*eps] inner product: P^T g has no
    discrete divergence at the inner nodes, what it removes is [*eps] times a
    gradient (the curl of its [*eps]^-1 image vanishes), it is idempotent,
    kills a pure gradient flux, and is the transpose of P u = u - D y on
    fields that vanish on the boundary edges."""
    import scipy.sparse.linalg as spla
    from oracle import gauss, qh
    ns = gauss.NsOracle(jittered, EPS0)
    rng = np.random.default_rng(31)
    I, inn = ns.inner, ~ns.bnd
    C = qh.curl_incidence(jittered)
    g = rng.standard_normal(jittered.ne)
    gs = ns.solenoidal_source(g)
    assert np.abs((ns.D.T @ gs)[I]).max() <= 1e-12 * np.abs((ns.D.T @ g)[I]).max()
    assert np.array_equal(gs[ns.bnd], g[ns.bnd])
    x = np.zeros(jittered.ne)
    x[inn] = spla.spsolve(ns.M[inn][:, inn].tocsc(), (g - gs)[inn])
    assert np.abs(C @ x).max() <= 1e-10 * np.abs(x).max()
    assert np.abs(ns.solenoidal_source(gs) - gs).max() <= 1e-12 * np.abs(gs).max()
    phi = rng.standard_normal(jittered.nv) * ~ns.wall
    f = ns.M @ (ns.D @ phi)
    assert np.abs(ns.solenoidal_source(f)[inn]).max() <= 1e-10 * np.abs(f).max()
    u = (rng.standard_normal(jittered.ne) + 1j * rng.standard_normal(jittered.ne)) * inn
    pu = ns.solenoidal_part(u)
    assert np.abs((ns.D.T @ (ns.M @ pu))[I]).max() <= 1e-12 * np.abs((ns.D.T @ (ns.M @ u))[I]).max()
    assert np.abs(C @ (u - pu)).max() <= 1e-12 * np.abs(u).max()
    assert np.abs(ns.solenoidal_part(pu) - pu).max() <= 1e-12 * np.abs(pu).max()
    assert abs(gs @ u - g @ pu) <= 1e-12 * np.abs(g).sum() * np.abs(u).max()


def test_solenoidal_step_is_the_projected_field_step(jittered):
    """The field step commutes with the split: projecting the state after a
    step equals stepping the projected state with the projected source P^T
    g'' (the curl-curl stiffness annihilates gradients and P is orthogonal in
    [*eps]), and the face field is the same.  So the solenoidal system is the
    field step run on the range of P, driven by P^T g''; any carrier."""
    from oracle import field, gauss
    ns = gauss.NsOracle(jittered, EPS0)
    F = field.FieldOracle(jittered, 1e-11, 2 * np.pi * 1.1e9, EPS0, 1.25663706212e-6)
    rng = np.random.default_rng(33)
    inn = ~ns.bnd
    cplx = lambda n: rng.standard_normal(n) + 1j * rng.standard_normal(n)
    u, v, a = (cplx(jittered.ne) * inn * s for s in (1.0, 1e10, 1e20))
    b = cplx(jittered.nf) * 1e-9
    gdd = rng.standard_normal(jittered.ne) * 1e3
    P = ns.solenoidal_part
    full = F.step(3.3e-10, u, v, a, b, gdd)
    sol = F.step(3.3e-10, P(u), P(v), P(a), b, ns.solenoidal_source(gdd))
    for x, y in zip(full[:3], sol[:3]):
        assert np.abs(P(x) - y).max() <= 1e-10 * np.abs(y).max()
    assert np.abs(full[3] - sol[3]).max() <= 1e-10 * np.abs(sol[3]).max()


def test_split_loop_equals_corrected_loop(ora):
    """The electromagnetic loop in the form of the split (field step on the
    solenoidal part driven by P^T G'', plus the field of eq. ns_equation) and
    the loop corrected every step give the same particles, fields and Gauss'
    law: the same field, reached along the two routes."""
    import plasma_util as P
    cp = synth.cold_plasma(4, 20_000)
    shape = P.mode_shape(cp, synth.mesh_edges(cp.tet_vert, cp.xyz.shape[0]))
    dt = 0.1 / cp.omega_p
    sa, siga, ga = P.oracle_em_loop(ora, cp, 20, dt, shape, correct=True)
    sb, sigb, gb = P.oracle_em_loop(ora, cp, 20, dt, shape, split=True)
    assert gb.max() < 1e-12, gb.max()
    assert np.abs(sigb - siga).max() <= 1e-12 * np.abs(siga).max()
    for (ta, la, va, Ga), (tb, lb, vb, Gb) in zip(sa, sb):
        assert np.array_equal(ta, tb)
        assert np.abs(lb - la).max() < 1e-12
        assert np.abs(vb - va).max() <= 1e-12 * np.abs(va).max()
        assert np.abs(Gb - Ga).max() <= 1e-12 * np.abs(Ga).max()
