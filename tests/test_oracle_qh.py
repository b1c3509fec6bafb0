"""Pins of the quasi-Helmholtz projector oracle: the tet-face divergence
against Gauss' theorem for linear fields and against the curl (div curl = 0),
Sigma = eps0 M_g against a quadrature of W1 . grad W0, and the projector
identities (idempotent, symmetric, the ranges they keep and kill)."""
import numpy as np
import pytest

from paper_2208_12795_amd import synth

EPS0 = 8.8541878128e-12


@pytest.fixture(scope="module")
def mesh(ora):
    xyz, tv = synth.kuhn_mesh((4, 3, 5), (1.0, 0.8, 1.2), 0.15, np.random.default_rng(12))
    return ora.OracleMesh(xyz, tv)


@pytest.fixture(scope="module")
def Q(mesh):
    from oracle import qh
    return qh.QhOracle(mesh, EPS0)


def rel(x, y):
    return np.abs(x - y).max() / np.abs(y).max()


def test_divergence_of_linear_fields(mesh, Q):
    """B(r) = G r + B0: the face DoFs (fluxes, exact by the centroid rule on a
    flat face) summed with the tet's outward signs give tr(G) times the tet
    volume (Gauss' theorem)."""
    from oracle import field
    G = np.array([[1.3, 0.2, -0.7], [0.4, -2.1, 0.3], [0.9, 0.5, 0.35]])
    B0 = np.array([0.2, -1.0, 0.6])
    fc = mesh.faces()
    a, b, c = (mesh.xyz[fc[:, i]] for i in range(3))
    area = 0.5 * np.cross(b - a, c - a)
    cen = (a + b + c) / 3.0
    flux = np.einsum("ij,ij->i", cen @ G.T + B0, area)
    vol = field.tet_gradients(mesh.xyz, mesh.tv)[1]
    assert rel(Q.div @ flux, np.trace(G) * vol) < 1e-12
    # a uniform field is divergence free
    assert np.abs(Q.div @ synth.uniform_face_flux(mesh.xyz, fc, B0)).max() < 1e-14


def test_div_of_curl_vanishes(mesh, Q):
    """(C e)_f = e_ab + e_bc - e_ac (the face-edge incidence of the field
    update) composed with the divergence is zero."""
    from oracle import field
    fe = field.face_edges(mesh)
    C = np.zeros((mesh.nf, mesh.ne))
    C[np.arange(mesh.nf), fe[:, 0]] += 1
    C[np.arange(mesh.nf), fe[:, 1]] += 1
    C[np.arange(mesh.nf), fe[:, 2]] -= 1
    assert np.abs(Q.div @ C).max() == 0.0


def test_sigma_is_eps_mg(mesh, Q):
    """Sigma = [*eps] D equals eps0 <W1_i, grad W0_j>, integrated directly:
    int W1_pq . g_j = V/4 (g_q - g_p) . g_j."""
    from oracle import field
    g, vol = field.tet_gradients(mesh.xyz, mesh.tv)
    te = mesh.tet_edges()
    Mg = np.zeros((mesh.ne, mesh.nv))
    for e, (p, q) in enumerate(field.LE):
        for j in range(4):
            np.add.at(Mg, (te[:, e], mesh.tv[:, j]),
                      vol / 4.0 * np.einsum("ta,ta->t", g[:, q] - g[:, p], g[:, j]))
    assert rel(Q.Sigma.toarray(), EPS0 * Mg) < 1e-12


def test_magnetic_projector(mesh, Q):
    from oracle import field
    rng = np.random.default_rng(3)
    b = rng.standard_normal(mesh.nf) + 1j * rng.standard_normal(mesh.nf)
    c = rng.standard_normal(mesh.nf)
    Pb = Q.project_b(b)
    scale = np.abs(b).max()
    assert np.abs(Q.div @ Pb).max() < 1e-12 * scale                # divergence free
    assert rel(Q.project_b(Pb), Pb) < 1e-12                         # idempotent
    assert abs(np.vdot(Q.project_b(c), b) - np.vdot(c, Pb)) < 1e-12 * np.abs(b).sum() * np.abs(c).max()   # symmetric
    fe = field.face_edges(mesh)
    e = rng.standard_normal(mesh.ne)
    ce = e[fe[:, 0]] + e[fe[:, 1]] - e[fe[:, 2]]
    assert rel(Q.project_b(ce), ce) < 1e-12                         # curls kept
    y = rng.standard_normal(mesh.nt)
    assert np.abs(Q.project_b(Q.div.T @ y)).max() < 1e-12 * np.abs(Q.div.T @ y).max()   # range of div^T killed


def test_electric_projectors(mesh, Q):
    rng = np.random.default_rng(5)
    d = (rng.standard_normal(mesh.ne) + 1j * rng.standard_normal(mesh.ne)) * 1e-11
    ps, pl, y = Q.project_e(d)
    assert rel(ps + pl, d) < 1e-15
    assert rel(Q.project_e(ps)[0], ps) < 1e-10                       # idempotent
    assert np.abs(Q.project_e(pl)[0]).max() < 1e-10 * np.abs(d).max()
    c = rng.standard_normal(mesh.ne) * 1e-11
    assert abs(np.vdot(Q.project_e(c)[0], d) - np.vdot(c, ps)) < 1e-10 * np.abs(d).sum() * np.abs(c).max()
    # Sigma^T P^Lambda d = 0: the solenoidal part has no discrete divergence
    assert np.abs(Q.Sigma.T @ pl).max() < 1e-10 * np.abs(Q.Sigma.T @ d).max()
    # a pure gradient flux density: E_ns is its potential (up to the constant)
    phi = rng.standard_normal(mesh.nv)
    ps2, pl2, y2 = Q.project_e(Q.Sigma @ phi)
    assert rel(y2, phi - phi.mean()) < 1e-9
    assert np.abs(pl2).max() < 1e-9 * np.abs(Q.Sigma @ phi).max()
    assert abs(y.sum()) < 1e-9 * np.abs(y).sum()                       # minimum norm: orthogonal to constants


MU0 = 1.25663706212e-6


def test_solenoidal_system_blocks_and_spectrum(ora):
    """Study of eq. sol_disc on the unit cube (3^3 and 4^3 unjittered cells).
    As printed, Z12 = C_b^T [curl] [*eps]^-1 P^Lambda_e [*eps] C_e reduces to
    C_b^T C C_e (the inverse only removes a gradient, which C annihilates),
    and the semi-discrete system's eigenvalues are not all real: with the
    Euclidean projectors it is not a lossless discretisation of the cavity.
    With the projectors orthogonal in the energy products it is: a real
    spectrum whose lowest modes (three degenerate ones at c sqrt(2)/2 for the
    unit cube, then two at c sqrt(3)/2) converge at second order."""
    from oracle import qh
    c0 = 1.0 / np.sqrt(EPS0 * MU0)
    errs = []
    for n in (3, 4):
        xyz, tv = synth.kuhn_mesh((n, n, n), (1.0, 1.0, 1.0), 0.0)
        m = ora.OracleMesh(xyz, tv)
        Z11, Z12, Z21, Z22, (Ce, Cb, C) = qh.solenoidal_blocks(m, EPS0, MU0, weighted=False)
        assert Ce.shape[1] == m.ne - m.nv + 1 and Cb.shape[1] == m.nf - m.nt
        assert np.abs(Z12 - Cb.T @ C @ Ce).max() < 1e-12
        ev = np.linalg.eigvals(np.linalg.solve(Z21, Z22) @ np.linalg.solve(Z11, Z12))
        assert np.abs(ev.imag).max() > 0.05 * np.abs(ev).max()
        ev = qh.solenoidal_spectrum(m, EPS0, MU0, weighted=True)
        assert np.abs(ev.imag).max() < 1e-10 * np.abs(ev).max() and ev.real.min() > 0
        f = np.sort(np.sqrt(ev.real)) / (2 * np.pi)
        f110, f111 = c0 * np.sqrt(2) / 2, c0 * np.sqrt(3) / 2
        assert np.all(np.abs(f[:3] / f110 - 1) < 0.02) and np.all(np.abs(f[3:5] / f111 - 1) < 0.03)
        errs.append(np.abs(f[:3] / f110 - 1).max())
    assert errs[0] / errs[1] > 1.5, errs           # (4/3)^2 = 1.78 for second order


def test_solenoidal_system_is_the_curl_curl_pencil_off_gradients(ora):
    """The solenoidal system with the energy-orthogonal projectors has the
    nonzero spectrum of the full edge-element pencil (K, [*eps]): its cotree
    unknowns are a basis of the [*eps]-orthogonal complement of the
    gradients, where K is nonsingular.  So the field step run on that
    complement (state solenoidal, source projected) is the same system
    without the tree-cotree gauge (unit cube, 3^3 cells, no boundary
    condition, as in the study above)."""
    import scipy.linalg as sl
    from oracle import field, qh
    xyz, tv = synth.kuhn_mesh((3, 3, 3), (1.0, 1.0, 1.0), 0.0)
    m = ora.OracleMesh(xyz, tv)
    ev = np.sort(qh.solenoidal_spectrum(m, EPS0, MU0, weighted=True).real)
    M, K, _ = field.assemble(m, EPS0, MU0)
    w = sl.eigh(K.toarray(), M.toarray(), eigvals_only=True)
    nz = np.sort(w[w > 1e-6 * w.max()])
    assert len(nz) == len(ev) == m.ne - m.nv + 1
    assert np.abs(nz / ev - 1).max() < 1e-10


MU0 = 1.25663706212e-6


def test_z13_is_the_curl_of_a_gradient(mesh):
    """Z13 = C_b^T [curl] [*eps]^-1 Sigma C_z: [*eps]^-1 Sigma is the
    node-to-edge incidence and the curl of a gradient vanishes, so the block
    is zero to rounding (Faraday's law gets no source from E_ns); Z23 =
    C_e^T [*eps] D C_z is not."""
    from oracle import qh
    Z13, Z23, Cz = qh.solenoidal_source_blocks(mesh, EPS0)
    assert Cz.shape == (mesh.nv, len(qh.inner_nodes(mesh)))
    assert np.abs(Z13).max() < 1e-12
    assert np.abs(Z23).max() > 1e-13


def test_printed_step_faraday_closed_form(mesh):
    """The dense trapezoidal step of eq. sol_disc as printed: the face field
    b = P^Lambda_b C_b B_s it produces satisfies Faraday's law on every face,
    b1 = ((1/dt - j w/2) b0 - C C_e (E0 + E1)/2) / (1/dt + j w/2): b and
    C C_e E are divergence-free and a divergence-free face field vanishing on
    the cotree faces vanishes.  Ampere's rows hold in the full-space form
    C_e^T (P^Lambda_e [*eps] e - C^T [*mu^-1] (b0 + b1)/2) = src_e with
    e = C_e (a E1 - conj(a) E0) and the projector from the sparse solves
    (not the dense pseudoinverse of the blocks)."""
    from oracle import qh
    rng = np.random.default_rng(4)
    et, ft = qh.spanning_trees(mesh)
    nec, nfc = int((~et).sum()), int((~ft).sum())
    Bs = (rng.standard_normal(nfc) + 1j * rng.standard_normal(nfc)) * 1e-6
    Es = (rng.standard_normal(nec) + 1j * rng.standard_normal(nec)) * 1e2
    src = (rng.standard_normal(nec) + 1j * rng.standard_normal(nec)) * 1e-1
    dt, w = 2e-11, 2 * np.pi * 1e9
    B1, E1 = qh.solenoidal_step(mesh, EPS0, MU0, dt, w, Bs, Es, src_e=src)
    b0, b1 = qh.solenoidal_b_field(mesh, EPS0, Bs), qh.solenoidal_b_field(mesh, EPS0, B1)
    a, ab = 1 / dt + 0.5j * w, 1 / dt - 0.5j * w
    C = qh.curl_incidence(mesh)
    e0, e1 = np.zeros(mesh.ne, complex), np.zeros(mesh.ne, complex)
    e0[~et], e1[~et] = Es, E1
    assert rel(b1, (ab * b0 - 0.5 * C @ (e0 + e1)) / a) < 1e-10
    Q = qh.QhOracle(mesh, EPS0)
    F = qh.face_mass(mesh, MU0)
    _, pl, _ = Q.project_e(Q.M @ (a * e1 - ab * e0))
    lhs = (pl - 0.5 * C.T @ F @ (b0 + b1))[~et]
    assert np.abs(lhs - src).max() < 1e-10 * np.abs(pl[~et]).max()


def test_printed_ampere_block_is_indefinite(ora):
    """Z21 = C_e^T P^Lambda_e [*eps] C_e (Euclidean projector) is not a mass
    matrix: from 6^3 cells of the unit cube on it has eigenvalues with a
    negative real part, while the energy-orthogonal form's Z21 is symmetric
    positive definite.  (On 3^3 and 4^3 cells all its eigenvalues still lie
    in the right half plane.)"""
    from oracle import qh
    for n, negative in ((4, False), (6, True)):
        xyz, tv = synth.kuhn_mesh((n, n, n), (1.0, 1.0, 1.0), 0.0)
        m = ora.OracleMesh(xyz, tv)
        _, _, Z21, _, _ = qh.solenoidal_blocks(m, EPS0, MU0, weighted=False)
        ev = np.linalg.eigvals(Z21 / np.abs(np.diag(Z21)).mean())
        assert (ev.real.min() < 0) == negative, (n, ev.real.min())
        if negative:
            _, _, W21, _, _ = qh.solenoidal_blocks(m, EPS0, MU0, weighted=True)
            assert np.abs(W21 - W21.T).max() < 1e-12 * np.abs(W21).max()
            assert np.linalg.eigvalsh(W21).min() > 0
