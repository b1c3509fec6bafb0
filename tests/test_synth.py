"""Input generators: reference-grid point location and sampling sanity."""
import numpy as np

from paper_2208_12795_amd import synth


def test_reference_location_is_inside_and_exact():
    n, ext = (3, 2, 4), (1.5, 1.0, 2.0)
    xyz, tv = synth.kuhn_mesh(n, ext, 0.0, None)
    rng = np.random.default_rng(0)
    u = rng.random((20000, 3)) * np.array(ext)
    h = np.array(ext) / np.array(n)
    u[:50] = 0.25 * h                      # three-way tie of the fractional coordinates
    u[50:100, 0] = u[50:100, 1] / h[1] * h[0]   # two-way ties
    t, lam = synth.reference_located(u, n, ext)
    l4 = np.c_[1 - lam.sum(1), lam]
    assert l4.min() >= -1e-15
    x = np.einsum("ij,ijk->ik", l4, xyz[tv[t]])
    assert np.abs(x - u).max() < 1e-14


def test_uniform_particles_follow_volume():
    xyz, tv = synth.kuhn_mesh((4, 4, 4), (1.0, 1.0, 1.0), 0.1, np.random.default_rng(1))
    vol = np.abs(synth.tet_volumes(xyz, tv))
    tet, lam = synth.uniform_particles(xyz, tv, 400000, np.random.default_rng(2))
    assert tet.min() >= 0 and tet.max() < tv.shape[0]
    assert lam.min() >= 0 and (1 - lam.sum(1)).min() >= -1e-15
    cnt = np.bincount(tet, minlength=tv.shape[0])
    expect = 400000 * vol / vol.sum()
    chi2 = ((cnt - expect) ** 2 / expect).sum()
    assert chi2 < tv.shape[0] + 6 * np.sqrt(2 * tv.shape[0])


def test_workloads_are_reproducible():
    a = synth.make_workload(1)
    b = synth.make_workload(1)
    for x, y in ((a.tet, b.tet), (a.lam, b.lam), (a.vel, b.vel), (a.e_env, b.e_env), (a.xyz, b.xyz)):
        assert np.array_equal(x, y)
    assert a.tet.shape == (1000,) and a.tet_vert.shape == (750, 4)


def test_fixed_point_barycentrics_storage():
    """The compact mixed form's storage of barycentrics (uint32, 2^-32): the
    nearest grid point, lam_0 = 1 - sum never negative, exact round trip of
    grid values, and the edge cases (a vertex, a face, lam_0 slightly
    negative after rounding)."""
    import numpy as np
    from paper_2208_12795_amd.etpic import fixed_to_lam, lam_to_fixed
    rng = np.random.default_rng(3)
    g = rng.standard_exponential((100_000, 4))
    lam = (g / g.sum(1, keepdims=True))[:, 1:]
    lam[:6] = [[1.0, 0, 0], [0, 0, 0], [0.5, 0.5, 0], [1 / 3] * 3, [0.2, 0.3, 0.5 + 1e-12], [0.5, 0.5, 1e-13]]
    u = lam_to_fixed(lam)
    back = fixed_to_lam(u)
    uu = u.view(np.uint32).astype(np.int64)
    assert np.all(uu.sum(1) <= 1 << 32)
    assert np.all(np.abs(back - lam) <= 1.5 * 2.0 ** -32)
    assert np.array_equal(lam_to_fixed(back), u)
    assert np.all(1.0 - back.sum(1) >= 0.0)
