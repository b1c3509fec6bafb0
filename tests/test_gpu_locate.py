"""GPU point location and positions (particle upload from Cartesian points)
against the Kuhn-grid reference location, the oracle's brute-force location
and the oracle's positions."""
import numpy as np
import pytest

from paper_2208_12795_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def E():
    from paper_2208_12795_amd import etpic
    return etpic


def empty_parts(E, torch, n):
    lam = torch.full((3, n), -7.0, dtype=torch.float64, device="cuda")
    vel = torch.zeros((3, n), dtype=torch.float64, device="cuda")
    tet = torch.full((n,), -9, dtype=torch.int32, device="cuda")
    return E.Particles(lam, vel, tet)


def to_dev(torch, x):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(x, np.float64).T)).cuda()


def kuhn_points(n_cells, extent, n, seed, jitter=0.1):
    """Jittered Kuhn mesh and n points with known (tet, lam): u uniform in the
    unjittered box, located by the grid rule, mapped to the jittered mesh."""
    rng = np.random.default_rng(seed)
    xyz, tv = synth.kuhn_mesh(n_cells, extent, jitter, rng)
    u = rng.random((n, 3)) * np.asarray(extent)
    tet, lam = synth.reference_located(u, n_cells, extent)
    return xyz, tv, tet, lam


def xyz_of(xyz, tv, tet, lam):
    l0 = 1.0 - lam.sum(axis=1)
    r = xyz[tv[tet]]
    return l0[:, None] * r[:, 0] + lam[:, 0:1] * r[:, 1] + lam[:, 1:2] * r[:, 2] + lam[:, 2:3] * r[:, 3]


@pytest.mark.parametrize("n_cells,extent,hint", [((40, 40, 40), (1.0, 1.0, 1.0), "none"),
                                                  ((32, 16, 16), (2.0, 1.0, 1.0), "none"),
                                                  ((32, 16, 16), (2.0, 1.0, 1.0), "exact"),
                                                  ((32, 16, 16), (2.0, 1.0, 1.0), "random")])
def test_locate_matches_kuhn_reference(E, torch_cuda, n_cells, extent, hint):
    torch = torch_cuda
    n = 1_000_003
    print(f"[locate] mesh {n_cells} extent {extent} hint {hint} N={n}", flush=True)
    xyz, tv, tet_ref, lam_ref = kuhn_points(n_cells, extent, n, seed=11)
    x = xyz_of(xyz, tv, tet_ref, lam_ref)
    ctx = E.Context(0)
    ctx.upload_mesh(xyz, tv)
    parts = empty_parts(E, torch, n)
    h = None
    if hint == "exact":
        h = torch.from_numpy(tet_ref.astype(np.int32)).cuda()
    elif hint == "random":
        h = torch.from_numpy(np.random.default_rng(3).integers(0, tv.shape[0], n).astype(np.int32)).cuda()
    ctx.locate(to_dev(torch, x), parts, hint=h)
    tet = parts.tet.cpu().numpy()
    lam = parts.lam.cpu().numpy().T
    lam4 = np.concatenate([1.0 - lam.sum(axis=1, keepdims=True), lam], axis=1)
    ref4 = np.concatenate([1.0 - lam_ref.sum(axis=1, keepdims=True), lam_ref], axis=1)
    off_face = ref4.min(axis=1) > 1e-9
    print(f"[locate] off-face {off_face.mean():.4f}, tet mismatches off-face {(tet != tet_ref)[off_face].sum()}", flush=True)
    assert np.array_equal(tet[off_face], tet_ref[off_face])
    assert np.abs(lam4[off_face] - ref4[off_face]).max() < 1e-12
    # every point (on faces too) is inside its tet and reproduces x
    assert (tet >= 0).all() and lam4.min() > -1e-12
    xr = xyz_of(xyz, tv, tet, lam)
    assert np.abs(xr - x).max() < 1e-14 * max(extent)
    ctx.close()


def test_locate_matches_bruteforce_small_mesh(E, torch_cuda, ora):
    """5^3 x 6 jittered mesh: the oracle's brute-force location of points drawn
    uniformly in the box (and the mesh's vertices and edge midpoints)."""
    torch = torch_cuda
    rng = np.random.default_rng(4)
    xyz, tv = synth.kuhn_mesh((5, 5, 5), (1.0, 1.0, 1.0), 0.1, rng)
    M = ora.OracleMesh(xyz, tv)
    ed = M.edges()
    pts = np.concatenate([rng.random((3000, 3)), xyz, 0.5 * (xyz[ed[:, 0]] + xyz[ed[:, 1]])])
    ctx = E.Context(0)
    ctx.upload_mesh(xyz, tv)
    parts = empty_parts(E, torch, pts.shape[0])
    ctx.locate(to_dev(torch, pts), parts)
    tet = parts.tet.cpu().numpy()
    lam = parts.lam.cpu().numpy().T
    lam4 = np.concatenate([1.0 - lam.sum(axis=1, keepdims=True), lam], axis=1)
    assert lam4.min() > -1e-12
    assert np.abs(xyz_of(xyz, tv, tet, lam) - pts).max() < 1e-14
    checked = 0
    for i in range(3000):
        t_ref, minlam = M.locate(pts[i])
        if minlam > 1e-9:
            assert tet[i] == t_ref, i
            checked += 1
    assert checked > 2900
    ctx.close()


def test_locate_reports_outside_points(E, torch_cuda):
    torch = torch_cuda
    xyz, tv, tet_ref, lam_ref = kuhn_points((8, 8, 8), (1.0, 1.0, 1.0), 1000, seed=5)
    x = xyz_of(xyz, tv, tet_ref, lam_ref)
    bad = np.array([3, 17, 500, 999])
    x[bad[0]] = (1.5, 0.5, 0.5)
    x[bad[1]] = (-1e-3, 0.2, 0.2)
    x[bad[2]] = (np.nan, 0.5, 0.5)
    x[bad[3]] = (0.5, 0.5, np.inf)
    ctx = E.Context(0)
    ctx.upload_mesh(xyz, tv)
    parts = empty_parts(E, torch, x.shape[0])
    rc = ctx.locate(to_dev(torch, x), parts, raise_on_error=False)
    assert rc == E.EPARTICLE
    tet = parts.tet.cpu().numpy()
    assert (tet[bad] == -1).all()
    good = np.setdiff1d(np.arange(x.shape[0]), bad)
    assert (tet[good] >= 0).all()
    with pytest.raises(E.EtpicError):
        ctx.locate(to_dev(torch, x), parts)
    ctx.close()


def test_positions_match_oracle_and_round_trip(E, torch_cuda, ora):
    """positions() against the oracle's x = sum lam_k r_k on the 5^3-cube workload
    particles, then locate(positions) gives back the same particles."""
    torch = torch_cuda
    w = synth.make_workload(1)
    M = ora.OracleMesh(w.xyz, w.tet_vert)
    ctx = E.Context(0)
    ctx.upload_mesh(w.xyz, w.tet_vert)
    parts = E.Particles.from_numpy(w.tet, w.lam, w.vel)
    x = ctx.positions(parts)
    ref = M.positions(w.tet, w.lam)
    assert np.abs(x.cpu().numpy().T - ref).max() < 1e-15
    back = empty_parts(E, torch, parts.n)
    ctx.locate(x, back)
    lam_b = back.lam.cpu().numpy().T
    l4 = np.concatenate([1.0 - w.lam.sum(axis=1, keepdims=True), w.lam], axis=1)
    off = l4.min(axis=1) > 1e-9
    assert np.array_equal(back.tet.cpu().numpy()[off], w.tet[off])
    assert np.abs(lam_b[off] - w.lam[off]).max() < 1e-13
    ctx.close()


def test_positions_and_locate_in_fixed_point_storage(E, torch_cuda, ora):
    """The compact mixed form's storage (barycentrics as uint32, 2^-32):
    positions() from the stored grid values against the oracle's positions of
    the same (exact) barycentrics, and locate() of those points stores the
    same grid values back up to one grid step (the point's barycentrics are
    recomputed in float64 and rounded to the grid again)."""
    torch = torch_cuda
    w = synth.make_workload(1)
    M = ora.OracleMesh(w.xyz, w.tet_vert)
    ctx = E.Context(0)
    ctx.upload_mesh(w.xyz, w.tet_vert)
    parts = E.Particles.from_numpy(w.tet, w.lam, w.vel, precision=E.MIXED_FIXED)
    t, lam, _, _ = parts.to_numpy()
    x = ctx.positions(parts)
    ref = M.positions(t, lam)
    assert np.abs(x.cpu().numpy().T - ref).max() < 1e-15
    back = E.Particles(torch.full((3, parts.n), -1, dtype=torch.int32, device="cuda"),
                       torch.zeros((3, parts.n), dtype=torch.float32, device="cuda"),
                       torch.full((parts.n,), -9, dtype=torch.int32, device="cuda"))
    assert back.precision == E.MIXED_FIXED
    ctx.locate(x, back)
    tb, lb, _, _ = back.to_numpy()
    l4 = np.concatenate([1.0 - lam.sum(axis=1, keepdims=True), lam], axis=1)
    off = l4.min(axis=1) > 1e-9
    assert np.array_equal(tb[off], t[off])
    assert np.abs(lb[off] - lam[off]).max() <= 2.0 ** -32 + 1e-15
    assert np.all(1.0 - lb.sum(axis=1) >= 0.0)
    ctx.close()
