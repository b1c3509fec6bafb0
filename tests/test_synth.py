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
