"""Pins of the field-update oracle: exactness properties of the Whitney edge
matrices and the energy conservation of the Newmark (1/2, 1/4) step."""
import numpy as np
import pytest

from paper_2208_12795_amd import synth

EPS0 = 8.8541878128e-12
MU0 = 1.25663706212e-6


@pytest.fixture(scope="module")
def fmesh(ora):
    xyz, tv = synth.kuhn_mesh((4, 3, 5), (1.0, 0.8, 1.2), 0.1, np.random.default_rng(31))
    return ora.OracleMesh(xyz, tv)


def total_volume(mesh):
    from oracle import field
    return field.tet_gradients(mesh.xyz, mesh.tv)[1].sum()


def test_mass_matrix_uniform_field_energy(fmesh):
    """W1 reproduces a uniform field exactly, so e^T M e = eps |E0|^2 volume."""
    from oracle import field
    M, K, bnd = field.assemble(fmesh, EPS0, MU0)
    ed = fmesh.edges()
    E0 = np.array([1.3, -0.4, 2.2])
    e = (fmesh.xyz[ed[:, 1]] - fmesh.xyz[ed[:, 0]]) @ E0
    assert np.isclose(e @ (M @ e), EPS0 * (E0 @ E0) * total_volume(fmesh), rtol=1e-12)
    assert abs(M - M.T).max() < 1e-12 * abs(M).max()
    assert np.linalg.eigvalsh(M.toarray()).min() > 0


def test_curl_matrix_null_space_and_uniform_curl(fmesh):
    """Gradients are curl free (K D phi = 0); the linear field E = B0 x r / 2 has
    curl B0, so e^T K e = |B0|^2 volume / mu (DoFs by the midpoint rule, exact
    for linear fields)."""
    from oracle import field
    M, K, bnd = field.assemble(fmesh, EPS0, MU0)
    ed = fmesh.edges()
    phi = np.random.default_rng(2).standard_normal(fmesh.nv)
    e = phi[ed[:, 1]] - phi[ed[:, 0]]
    assert np.abs(K @ e).max() < 1e-9 * abs(K).max() * np.abs(e).max()
    B0 = np.array([0.3, -1.1, 0.7])
    a, b = fmesh.xyz[ed[:, 0]], fmesh.xyz[ed[:, 1]]
    mid = 0.5 * (a + b)
    e = np.einsum("ij,ij->i", 0.5 * np.cross(B0, mid), b - a)
    assert np.isclose(e @ (K @ e), (B0 @ B0) * total_volume(fmesh) / MU0, rtol=1e-11)


def consistent_acceleration(F, u, v):
    """a with M a = -(2 j w M v + (K - w^2 M) u) on the interior edges (source free)."""
    import scipy.sparse.linalg as spla
    I = F.inner
    a = np.zeros_like(u)
    a[I] = -2j * F.w * v[I] + F.w ** 2 * u[I] - spla.spsolve(F.Mi, F.Ki @ u[I])
    return a


def test_newmark_conserves_energy(fmesh):
    """Source free, the average-acceleration step conserves
    0.5 v^H M v + 0.5 u^H (K - w^2 M) u (the gyroscopic term 2 j w M does no work)."""
    from oracle import field
    dt, w = 2e-11, 2 * np.pi * 1e9
    F = field.FieldOracle(fmesh, dt, w, EPS0, MU0)
    rng = np.random.default_rng(4)
    ne, nf = fmesh.ne, fmesh.nf
    u = (rng.standard_normal(ne) + 1j * rng.standard_normal(ne)) * ~F.bnd
    v = (rng.standard_normal(ne) + 1j * rng.standard_normal(ne)) * ~F.bnd * 1e9
    a = consistent_acceleration(F, u, v)
    b = np.zeros(nf, complex)
    H0 = F.energy(u, v)
    for k in range(15):
        u, v, a, b = F.step((k + 1) * dt, u, v, a, b)
    assert abs(F.energy(u, v) - H0) < 1e-9 * abs(H0)
    assert np.abs(u[F.bnd]).max() == 0.0


def test_faraday_face_update_matches_closed_form(fmesh):
    """A constant edge envelope with b(0) = j circ(e)/w is a fixed point of the
    trapezoidal face update (the discrete Faraday law at steady state)."""
    from oracle import field
    dt, w = 2e-11, 2 * np.pi * 1e9
    F = field.FieldOracle(fmesh, dt, w, EPS0, MU0)
    rng = np.random.default_rng(6)
    e = rng.standard_normal(fmesh.ne) + 1j * rng.standard_normal(fmesh.ne)
    fe = F.fe
    b0 = 1j * (e[fe[:, 0]] + e[fe[:, 1]] - e[fe[:, 2]]) / w
    ce = lambda x: x[fe[:, 0]] + x[fe[:, 1]] - x[fe[:, 2]]
    b1 = ((1 - 0.5j * w * dt) * b0 - 0.5 * dt * ce(e + e)) / (1 + 0.5j * w * dt)
    assert np.allclose(b1, b0, rtol=1e-13, atol=1e-13 * np.abs(b0).max())
    # the generator's Faraday-consistent envelope is the same b
    bs = synth.faraday_face_envelope(e, fmesh.edges(), fmesh.faces(), fmesh.nv, w)
    assert np.allclose(bs, b0, rtol=1e-14, atol=0)


def test_gmres_step_equals_direct_step(fmesh):
    """The iterative solve the oracle takes on large meshes (scipy's GMRES)
    gives the same Newmark step as the sparse direct solve, every state vector
    to 1e-13 relative."""
    from oracle import field
    dt, w = 2e-11, 2 * np.pi * 1e9
    F_lu = field.FieldOracle(fmesh, dt, w, EPS0, MU0, solver="lu")
    F_it = field.FieldOracle(fmesh, dt, w, EPS0, MU0, solver="gmres")
    rng = np.random.default_rng(4)
    ne, nf = fmesh.ne, fmesh.nf
    mask = ~F_lu.bnd
    u = (rng.standard_normal(ne) + 1j * rng.standard_normal(ne)) * mask
    v = (rng.standard_normal(ne) + 1j * rng.standard_normal(ne)) * mask * 1e9
    a = (rng.standard_normal(ne) + 1j * rng.standard_normal(ne)) * mask * 1e18
    b = (rng.standard_normal(nf) + 1j * rng.standard_normal(nf)) * 1e-9
    gdd = rng.standard_normal(ne) * 1e-10 * mask
    for x, y in zip(F_lu.step(dt, u, v, a, b, gdd), F_it.step(dt, u, v, a, b, gdd)):
        assert np.abs(x - y).max() <= 1e-13 * np.abs(x).max()
