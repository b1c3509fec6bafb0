"""The periodic re-sort folded into a step (etpic_sort_run_steps) against the
two calls it replaces (etpic_sort, then etpic_run_steps) and against the
oracle: every particle's state identical, the tets' groups at the same
places, the currents and charge equal to the atomics' rounding, the source
left untouched."""
import os
import sys

import numpy as np
import pytest

from paper_2208_12795_amd import synth

pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
from parity_util import assert_within, step_errors  # noqa: E402

NTH = max(1, min(16, os.cpu_count() or 1))


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


def by_id(state):
    t, l, v, i = state
    o = np.argsort(i)
    return t[o], l[o], v[o]


def two_ways(E, torch, w, precision, nsteps, dt, flags, step0=5):
    ctx = E.Context(0)
    ctx.upload_mesh(w.xyz, w.tet_vert)
    f = E.Fields.from_numpy(w.e_env, w.b_env, None, w.b_dc)
    sp = E.Species(w.q, w.m, w.w)
    src = E.Particles.from_numpy(w.tet, w.lam, w.vel, w.ids, precision=precision)
    before = src.to_numpy()
    rho0 = torch.zeros(ctx.n_vert, dtype=torch.float64, device="cuda")
    ctx.vertex_charge(src, sp, rho0)
    out = []
    for fused in (False, True):
        dst = src.empty_like()
        dG = torch.zeros(ctx.n_edge, dtype=torch.float64, device="cuda")
        rho = torch.zeros_like(rho0)
        if fused:
            ctx.sort_run_steps(src, dst, sp, f, step0, nsteps, dt, w.omega, dG, rho=rho, flags=flags)
        else:
            ctx.sort(src, dst)
            ctx.run_steps(dst, sp, f, step0, nsteps, dt, w.omega, dG, rho=rho, flags=flags)
        ctx.check()
        r, p = ctx.gauss_residual(dG, rho, rho0)
        assert r / p <= 1e-12, r / p
        out.append((dst.to_numpy(), dG.cpu().numpy(), rho.cpu().numpy()))
    after = src.to_numpy()
    for x, y in zip(before, after):
        assert np.array_equal(x, y)
    ctx.close()
    return before, out


@pytest.mark.parametrize("precision", [0, 1, 2])
@pytest.mark.parametrize("dt_scale,flags", [(1.0, "remap"), (60.0, "remap"), (60.0, "scan")])
def test_fused_sort_equals_sort_then_steps(E, torch_cuda, precision, dt_scale, flags):
    """300k unsorted electrons on the 40^3 mesh, 4 steps; dt x60 makes a few
    percent of them cross faces every step; "scan" walks the scatter step's
    walkers by a scan of all particles (the queue-overflow path)."""
    torch = torch_cuda
    fl = E.STEP_XCD_REMAP | (E.STEP_WALK_BY_SLICE if flags == "scan" else 0)
    w = synth.make_workload(2, n_particles=300_001)
    print(f"[sort-step] precision {precision} dt x{dt_scale} flags {flags}", flush=True)
    before, ((sa, ga, ra), (sb, gb, rb)) = two_ways(E, torch, w, precision, 4, w.dt * dt_scale, fl)
    t0 = before[0][np.argsort(before[3])]          # start tet by id
    ia, ib = sa[3], sb[3]
    assert np.array_equal(np.sort(ib), np.arange(len(ib)))
    # both outputs are grouped by start tet, the groups at the same places
    assert np.all(np.diff(t0[ib]) >= 0)
    assert np.array_equal(t0[ia], t0[ib])
    for x, y in zip(by_id(sa), by_id(sb)):
        assert np.array_equal(x, y)
    moved = (by_id(sb)[0] != t0).mean()
    print(f"[sort-step] particles that changed tet over the 4 steps: {moved:.4f}", flush=True)
    if dt_scale > 1:
        assert moved > 0.01
    assert np.abs(ga - gb).max() <= 1e-13 * np.abs(ga).max()
    assert np.abs(ra - rb).max() <= 1e-13 * np.abs(ra).max()


@pytest.mark.parametrize("slices", [4, 16])
@pytest.mark.parametrize("precision", [0, 1, 2])
def test_fused_sort_with_slices(E, torch_cuda, slices, precision):
    """The sliced particle kernels (several 64-particle slices per wavefront,
    the open run carried across slices) in their sorting form."""
    torch = torch_cuda
    w = synth.make_workload(2, n_particles=200_000)
    fl = E.STEP_XCD_REMAP | (E.STEP_SLICES_4 if slices == 4 else E.STEP_SLICES_16)
    before, ((sa, ga, _), (sb, gb, _)) = two_ways(E, torch, w, precision, 2, w.dt * 30, fl)
    t0 = before[0][np.argsort(before[3])]
    assert np.array_equal(t0[sa[3]], t0[sb[3]]) and np.all(np.diff(t0[sb[3]]) >= 0)
    for x, y in zip(by_id(sa), by_id(sb)):
        assert np.array_equal(x, y)
    assert np.abs(ga - gb).max() <= 1e-13 * np.abs(ga).max()


@pytest.mark.parametrize("precision,tol,case", [(0, 1e-12, "plain"), (1, 2e-5, "plain"), (0, 1e-12, "heavy"),
                                                (0, 1e-12, "heavy-scan"), (1, 2e-5, "heavy-scan"),
                                                (2, 2e-5, "plain"), (2, 2e-5, "heavy-scan")])
def test_fused_sort_step_matches_oracle(E, torch_cuda, ora, precision, tol, case):
    """One fused sort+step of the small workload (750 tets) against the
    oracle's step of the unsorted input, matched by id: 1000 electrons, or
    ("heavy") 4000 electrons 40x faster with dt 1e-8, so that most cross
    faces and many hit the walls, their walk found from the queue or by the
    scan of all particles."""
    torch = torch_cuda
    heavy = case != "plain"
    w = synth.make_workload(1, n_particles=4000 if heavy else None)
    dt = 1e-8 if heavy else w.dt
    if heavy:
        w.vel = w.vel * 40.0
    flags = E.STEP_XCD_REMAP | (E.STEP_WALK_BY_SLICE if case == "heavy-scan" else 0)
    perm = np.random.default_rng(5).permutation(w.tet.shape[0])
    tet, lam, vel, ids = w.tet[perm], w.lam[perm], w.vel[perm], w.ids[perm]
    ctx = E.Context(0)
    ctx.upload_mesh(w.xyz, w.tet_vert)
    f = E.Fields.from_numpy(w.e_env, w.b_env, None, w.b_dc)
    sp = E.Species(w.q, w.m, w.w)
    src = E.Particles.from_numpy(tet, lam, vel, ids, precision=precision)
    dst = src.empty_like()
    tin, lin, vin, iin = src.to_numpy()
    dG = torch.zeros(ctx.n_edge, dtype=torch.float64, device="cuda")
    ctx.sort_run_steps(src, dst, sp, f, 3, 1, dt, w.omega, dG, flags=flags)
    ctx.check()
    M = ora.OracleMesh(w.xyz, w.tet_vert)
    o = np.argsort(iin)
    t, l, v = tin[o].copy(), lin[o].copy(), vin[o].astype(np.float64)
    dGo = np.zeros(M.ne)
    rc, _ = M.step(t, l, v, q=w.q, m=w.m, w=w.w, step=3, dt=dt, omega=w.omega, e_env=w.e_env, b_env=w.b_env,
                   b_dc=w.b_dc, dG=dGo, nthreads=NTH)
    assert rc == 0
    tg, lg, vg = by_id(dst.to_numpy())
    err = step_errors(w.xyz, w.tet_vert, (tin[o], lin[o], vin[o]), (tg, lg, vg), (t, l, v), dG.cpu().numpy(), dGo,
                      lam_quantum=2.0 ** -31 if precision == E.MIXED_FIXED else 0.0)
    print(f"[sort-step] oracle {err}", flush=True)
    if heavy:
        assert (tg != tin[o]).mean() > 0.1
    assert err["tet_mismatch"] <= 2, err
    assert_within(err, tol, "fused sort step")
    ctx.close()


def test_fused_sort_argument_errors(E, torch_cuda):
    torch = torch_cuda
    w = synth.make_workload(1, n_particles=500)
    ctx = E.Context(0)
    ctx.upload_mesh(w.xyz, w.tet_vert)
    f = E.Fields.from_numpy(w.e_env, w.b_env, None, w.b_dc)
    sp = E.Species(w.q, w.m, w.w)
    src = E.Particles.from_numpy(w.tet, w.lam, w.vel, w.ids)
    dst = src.empty_like()
    dG = torch.zeros(ctx.n_edge, dtype=torch.float64, device="cuda")
    with pytest.raises(E.EtpicError):
        ctx.sort_run_steps(src, dst, sp, f, 0, 0, w.dt, w.omega, dG)
    with pytest.raises(E.EtpicError):
        ctx.sort_run_steps(src, src, sp, f, 0, 1, w.dt, w.omega, dG)
    no_ids = E.Particles.from_numpy(w.tet, w.lam, w.vel)
    with pytest.raises(E.EtpicError):
        ctx.sort_run_steps(no_ids, dst, sp, f, 0, 1, w.dt, w.omega, dG)
    with pytest.raises(E.EtpicError):
        ctx.sort_run_steps(src, dst, sp, f, 0, 1, w.dt, w.omega, None)
    ctx.check()
    ctx.close()
