"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Every case starts both sides from the same seeded state and compares one step
(v, positions, edge currents); multi-step cases also check the discrete
continuity law on the GPU every step.  Tolerances: float64 form 1e-12
relative, mixed form 2e-5 relative (positions beyond the float64 storage
quantum, see parity_util)."""
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


def fixed_quantum(E, precision):
    """absolute quantum of fixed-point barycentric storage (0 for float64 storage)"""
    return 2.0 ** -31 if precision == E.MIXED_FIXED else 0.0


def setup(E, torch, w, precision):
    ctx = E.Context(0)
    ctx.upload_mesh(w.xyz, w.tet_vert)
    assert np.array_equal(ctx.edges(), w.edges)
    assert np.array_equal(ctx.faces(), w.faces)
    parts = E.Particles.from_numpy(w.tet, w.lam, w.vel, w.ids, precision=precision)
    fields = E.Fields.from_numpy(w.e_env, w.b_env, None, w.b_dc)
    return ctx, parts, fields


def oracle_step(M, state, w, step, nthreads=1, omega=None, dt=None):
    tet, lam, vel = (np.ascontiguousarray(a).copy() for a in state)
    dG = np.zeros(M.ne)
    rc, _ = M.step(tet, lam, vel, q=w.q, m=w.m, w=w.w, step=step, dt=w.dt if dt is None else dt,
                   omega=w.omega if omega is None else omega, e_env=w.e_env, b_env=w.b_env, b_dc=w.b_dc, dG=dG,
                   nthreads=nthreads)
    return rc, (tet, lam, vel), dG


def run_case(E, torch, ora, w, steps, precision, tol, check_every=1, dt=None, flags=None):
    flags = E.STEP_XCD_REMAP if flags is None else flags
    print(f"[case] {w.name} N={w.tet.shape[0]} steps={steps} precision={precision} flags={flags}", flush=True)
    ctx, parts, fields = setup(E, torch, w, precision)
    M = ora.OracleMesh(w.xyz, w.tet_vert)
    sp = E.Species(w.q, w.m, w.w)
    dev = "cuda"
    rho_old = torch.zeros(ctx.n_vert, dtype=torch.float64, device=dev)
    ctx.vertex_charge(parts, sp, rho_old)
    worst = {}
    worst_gauss = 0.0
    dt = w.dt if dt is None else dt
    for s in range(steps):
        tin, lin, vin, _ = parts.to_numpy()
        dG = torch.zeros(ctx.n_edge, dtype=torch.float64, device=dev)
        ctx.gather_push_deposit(parts, sp, fields, s, dt, w.omega, dG, flags=flags)
        rho_new = torch.zeros_like(rho_old)
        ctx.vertex_charge(parts, sp, rho_new)
        r, p = ctx.gauss_residual(dG, rho_new, rho_old)
        worst_gauss = max(worst_gauss, r / p)
        assert r / p <= 1e-12, (s, r / p)
        if s % check_every == 0:
            rc, o, dGo = oracle_step(M, (tin, lin, vin), w, s, nthreads=NTH, dt=dt)
            assert rc == 0
            tg, lg, vg, _ = parts.to_numpy()
            err = step_errors(w.xyz, w.tet_vert, (tin, lin, vin), (tg, lg, vg), o, dG.cpu().numpy(), dGo,
                              lam_quantum=fixed_quantum(E, precision))
            assert err["tet_mismatch"] <= 2 + 1e-4 * len(tg), err
            assert_within(err, tol, f"step {s}")
            for k, v in err.items():
                worst[k] = max(worst.get(k, 0.0), v)
        rho_old = rho_new
    ctx.check()
    print(f"[case] {w.name} worst {worst} gauss {worst_gauss:.2e}", flush=True)
    ctx.close()
    return worst


@pytest.mark.parametrize("variant", ["remap", "no_remap"])
def test_small_config_fp64_every_step(E, torch_cuda, ora, variant):
    """1,000 electrons on the 750-tet unit cube, 100 steps, float64 form, with and
    without the XCD block remap."""
    flags = {"remap": E.STEP_XCD_REMAP, "no_remap": 0}[variant]
    run_case(E, torch_cuda, ora, synth.make_workload(1), 100, E.FP64, 1e-12, flags=flags)


def test_small_config_mixed(E, torch_cuda, ora):
    """Same case in the mixed form: float32 gather/push, float64 positions and deposit."""
    run_case(E, torch_cuda, ora, synth.make_workload(1), 30, E.MIXED, 2e-5)


def test_small_config_mixed_fixed(E, torch_cuda, ora):
    """The compact mixed form (barycentrics stored in 2^-32 fixed point) on the
    small workload, every step against the float64 oracle; continuity checked
    every step on the GPU (the deposit runs to the stored end points)."""
    run_case(E, torch_cuda, ora, synth.make_workload(1), 30, E.MIXED_FIXED, 2e-5)


@pytest.mark.parametrize("by_slice", [False, True])
@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 2e-5), (2, 2e-5)])
def test_crossing_heavy(E, torch_cuda, ora, precision, tol, by_slice):
    """Steps of 0.1-0.5 cell: most particles cross faces, several per step, and
    many hit the walls (reflection).  Walkers queued one by one, and by slice
    (the path taken when the particle queue overflows)."""
    w = synth.make_workload(1, n_particles=4000)
    w.vel = w.vel * 40.0
    flags = E.STEP_XCD_REMAP | (E.STEP_WALK_BY_SLICE if by_slice else 0)
    run_case(E, torch_cuda, ora, w, 12, precision, tol, dt=1e-8, flags=flags)


@pytest.mark.parametrize("presort", [False, True])
def test_ragged_and_multi_tile(E, torch_cuda, ora, presort):
    """A particle count that spans many 256-lane blocks with a ragged tail, on
    the 40^3 mesh (384k tets); unsorted (one slot per lane, several staging
    rounds per block) and sorted by tet (few slots per block)."""
    w = synth.make_workload(2, n_particles=200_003)
    if presort:
        order = np.argsort(w.tet, kind="stable")
        w.tet, w.lam, w.vel, w.ids = w.tet[order], w.lam[order], w.vel[order], w.ids[order]
    run_case(E, torch_cuda, ora, w, 3, E.FP64, 1e-12)


@pytest.mark.parametrize("slices", [1, 4, 16])
@pytest.mark.parametrize("precision,tol", [(0, 1e-12), (1, 2e-5), (2, 2e-5)])
def test_dense_tets_slices(E, torch_cuda, ora, slices, precision, tol):
    """About 400 particles per tet on the 750-tet cube, sorted by tet, so runs of
    one tet span several wavefronts; 1, 4 and 16 slices of 64 particles per
    wavefront (runs carried across slice boundaries).  Each step against the
    oracle (velocities, positions, currents) and the vertex charge deposited
    inside the step against a separate charge scatter after it."""
    torch = torch_cuda
    w = synth.make_workload(1, n_particles=300_007)
    order = np.argsort(w.tet, kind="stable")
    w.tet, w.lam, w.vel, w.ids = w.tet[order], w.lam[order], w.vel[order], w.ids[order]
    flags = E.STEP_XCD_REMAP | {1: E.STEP_SLICES_1, 4: E.STEP_SLICES_4, 16: E.STEP_SLICES_16}[slices]
    print(f"[dense] slices {slices} precision {precision}", flush=True)
    ctx, parts, fields = setup(E, torch, w, precision)
    M = ora.OracleMesh(w.xyz, w.tet_vert)
    sp = E.Species(w.q, w.m, w.w)
    for s in range(3):
        tin, lin, vin, _ = parts.to_numpy()
        dG = torch.zeros(ctx.n_edge, dtype=torch.float64, device="cuda")
        rho_step = torch.zeros(ctx.n_vert, dtype=torch.float64, device="cuda")
        ctx.gather_push_deposit(parts, sp, fields, s, w.dt, w.omega, dG, rho=rho_step, flags=flags)
        rho_after = torch.zeros_like(rho_step)
        ctx.vertex_charge(parts, sp, rho_after)
        assert torch.allclose(rho_step, rho_after, rtol=0, atol=1e-13 * rho_after.abs().max().item())
        rc, o, dGo = oracle_step(M, (tin, lin, vin.astype(np.float64)), w, s, nthreads=NTH)
        assert rc == 0
        tg, lg, vg, _ = parts.to_numpy()
        err = step_errors(w.xyz, w.tet_vert, (tin, lin, vin), (tg, lg, vg), o, dG.cpu().numpy(), dGo,
                          lam_quantum=fixed_quantum(E, precision))
        assert err["tet_mismatch"] <= 2 + 1e-4 * len(tg), err
        assert_within(err, tol, f"slices {slices} step {s}")
    ctx.check()
    ctx.close()


@pytest.mark.parametrize("n_particles,dense", [(300_007, True), (20_011, False)])
@pytest.mark.parametrize("precision", [1, 2])
def test_pipelined_slices(E, torch_cuda, ora, n_particles, dense, precision):
    """The float forms' two-slice kernel (the second slice's state requested
    before the first one's rows; runs carried across the slice boundary),
    forced by its flag: each step against the oracle, on runs of ~400
    particles per tet (sorted) and on a sparse set with a ragged last slice;
    continuity of the step's deposit against the charge moved.  float64 with
    the same flag runs one slice."""
    torch = torch_cuda
    w = synth.make_workload(1, n_particles=n_particles)
    if dense:
        order = np.argsort(w.tet, kind="stable")
        w.tet, w.lam, w.vel, w.ids = w.tet[order], w.lam[order], w.vel[order], w.ids[order]
    flags = E.STEP_XCD_REMAP | E.STEP_SLICES_2
    print(f"[pipe] N={n_particles} dense {dense} precision {precision}", flush=True)
    ctx, parts, fields = setup(E, torch, w, precision)
    M = ora.OracleMesh(w.xyz, w.tet_vert)
    sp = E.Species(w.q, w.m, w.w)
    for s in range(3):
        tin, lin, vin, _ = parts.to_numpy()
        dG = torch.zeros(ctx.n_edge, dtype=torch.float64, device="cuda")
        rho0 = torch.zeros(ctx.n_vert, dtype=torch.float64, device="cuda")
        rho1 = torch.zeros_like(rho0)
        ctx.vertex_charge(parts, sp, rho0)
        ctx.gather_push_deposit(parts, sp, fields, s, w.dt, w.omega, dG, flags=flags)
        assert ctx.last_push_slices() == 2
        ctx.vertex_charge(parts, sp, rho1)
        r, p = ctx.gauss_residual(dG, rho1, rho0)
        assert r <= 1e-12 * p, (r, p)
        rc, o, dGo = oracle_step(M, (tin, lin, vin.astype(np.float64)), w, s, nthreads=NTH)
        assert rc == 0
        tg, lg, vg, _ = parts.to_numpy()
        err = step_errors(w.xyz, w.tet_vert, (tin, lin, vin), (tg, lg, vg), o, dG.cpu().numpy(), dGo,
                          lam_quantum=fixed_quantum(E, precision))
        assert err["tet_mismatch"] <= 2 + 1e-4 * len(tg), err
        assert_within(err, 2e-5, f"pipe step {s}")
    ctx.check()
    ctx.close()
    ctx, parts, fields = setup(E, torch, w, E.FP64)
    dG = torch.zeros(ctx.n_edge, dtype=torch.float64, device="cuda")
    ctx.gather_push_deposit(parts, sp, fields, 0, w.dt, w.omega, dG, flags=flags)
    assert ctx.last_push_slices() == 1
    ctx.check()
    ctx.close()


def test_omega_zero_matches_regular(E, torch_cuda):
    """At w = 0 the GPU envelope run equals the GPU run with real DoFs Re(e~):
    the carrier factor is exactly one (reduction to the regular scheme)."""
    torch = torch_cuda
    w = synth.make_workload(1, omega=0.0)
    ctx, p1, f1 = setup(E, torch, w, E.FP64)
    p2 = p1.clone()
    f2 = E.Fields.from_numpy(np.zeros_like(w.e_env), w.b_env, w.e_env.real, w.b_dc)
    sp = E.Species(w.q, w.m, w.w)
    g1 = torch.zeros(ctx.n_edge, dtype=torch.float64, device="cuda")
    g2 = torch.zeros_like(g1)
    for s in range(5):
        ctx.gather_push_deposit(p1, sp, f1, s, w.dt, 0.0, g1)
        ctx.gather_push_deposit(p2, sp, f2, s, w.dt, 0.0, g2)
    a, b = p1.to_numpy(), p2.to_numpy()
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)
    # the currents are summed with float64 atomics in no fixed order
    assert torch.allclose(g1, g2, rtol=0, atol=1e-14 * g1.abs().max().item())


def test_sort_permutation_invariance(E, torch_cuda, ora):
    """Counting sort: output sorted by tet, a permutation of the input (ids carried),
    and a step after the sort gives the same currents as without it."""
    torch = torch_cuda
    w = synth.make_workload(2, n_particles=300_000)
    ctx, parts, fields = setup(E, torch, w, E.FP64)
    dst = parts.empty_like()
    ctx.sort(parts, dst)
    t0, l0, v0, i0 = parts.to_numpy()
    t1, l1, v1, i1 = dst.to_numpy()
    assert np.all(np.diff(t1) >= 0)
    assert np.array_equal(np.sort(i1), np.arange(len(i1)))
    assert np.array_equal(t1, t0[i1]) and np.array_equal(l1, l0[i1]) and np.array_equal(v1, v0[i1])
    sp = E.Species(w.q, w.m, w.w)
    g0 = torch.zeros(ctx.n_edge, dtype=torch.float64, device="cuda")
    g1 = torch.zeros_like(g0)
    ctx.gather_push_deposit(parts, sp, fields, 7, w.dt, w.omega, g0)
    ctx.gather_push_deposit(dst, sp, fields, 7, w.dt, w.omega, g1)
    assert torch.allclose(g0, g1, rtol=0, atol=1e-13 * g0.abs().max().item())
    ctx.check()


def test_sort_mixed_and_counts_histogram(E, torch_cuda):
    torch = torch_cuda
    w = synth.make_workload(1, n_particles=5000)
    ctx, parts, fields = setup(E, torch, w, E.MIXED)
    dst = parts.empty_like()
    ctx.sort(parts, dst)
    t1, l1, v1, i1 = dst.to_numpy()
    assert np.all(np.diff(t1) >= 0)
    assert np.array_equal(np.bincount(t1, minlength=ctx.n_tet), np.bincount(w.tet, minlength=ctx.n_tet))
    assert np.array_equal(v1.astype(np.float32), w.vel[i1].astype(np.float32))


def test_edge_cases(E, torch_cuda, ora):
    """Empty input; all particles in one tet (atomic contention); particles
    exactly on vertices and faces."""
    torch = torch_cuda
    w = synth.make_workload(1)
    ctx, _, fields = setup(E, torch, w, E.FP64)
    sp = E.Species(w.q, w.m, w.w)
    dG = torch.zeros(ctx.n_edge, dtype=torch.float64, device="cuda")
    empty = E.Particles.from_numpy(np.zeros(0, np.int32), np.zeros((0, 3)), np.zeros((0, 3)), np.zeros(0, np.int64))
    ctx.gather_push_deposit(empty, sp, fields, 0, w.dt, w.omega, dG)
    assert dG.abs().max().item() == 0.0
    M = ora.OracleMesh(w.xyz, w.tet_vert)
    rng = np.random.default_rng(9)
    n = 20000
    tet = np.full(n, 123, np.int32)
    g = rng.standard_exponential((n, 4))
    lam = (g / g.sum(1, keepdims=True))[:, 1:]
    lam[:8] = [[1, 0, 0], [0, 1, 0], [0, 0, 1], [0, 0, 0], [0.5, 0.5, 0], [0, 0.3, 0.7], [0.2, 0.3, 0.5], [1 / 3] * 3]
    vel = synth.maxwellian(n, 1e5, rng)
    parts = E.Particles.from_numpy(tet, lam, vel, np.arange(n))
    ctx.gather_push_deposit(parts, sp, fields, 4, w.dt, w.omega, dG)
    rc, o, dGo = oracle_step(M, (tet, np.ascontiguousarray(lam), vel), w, 4)
    tg, lg, vg, _ = parts.to_numpy()
    err = step_errors(w.xyz, w.tet_vert, (tet, lam, vel), (tg, lg, vg), o, dG.cpu().numpy(), dGo)
    assert_within(err, 1e-12, "one tet")
    ctx.check()


def ctx_tet_with_edge(w, e):
    """a tet that has edge e (from the generator's numbering)"""
    a, b = w.edges[e]
    tv = w.tet_vert
    return int(np.flatnonzero(np.any(tv == a, axis=1) & np.any(tv == b, axis=1))[0])


def test_device_errors_are_reported(E, torch_cuda, ora):
    """Host-forced error paths: a tet index out of range, a NaN field DoF and a
    displacement of ~1000 box lengths (hop cap) are flagged through
    etpic_check; the kernels still exit normally."""
    torch = torch_cuda
    w = synth.make_workload(1, n_particles=64)
    ctx, parts, fields = setup(E, torch, w, E.FP64)
    sp = E.Species(w.q, w.m, w.w)
    dG = torch.zeros(ctx.n_edge, dtype=torch.float64, device="cuda")
    bad = parts.clone()
    bad.tet[5] = ctx.n_tet + 3
    ctx.gather_push_deposit(bad, sp, fields, 0, w.dt, w.omega, dG)
    rc, word = ctx.check(raise_on_error=False)
    assert rc == E.EPARTICLE and word & E.DEV_BADTET
    rc, word = ctx.check(raise_on_error=False)
    assert rc == 0 and word == 0
    nan_f = E.Fields.from_numpy(np.where(np.arange(ctx.n_edge) == 7, np.nan, w.e_env), w.b_env, None, w.b_dc)
    hit = E.Particles.from_numpy(np.full(64, ctx_tet_with_edge(w, 7), np.int32), w.lam[:64], w.vel[:64])
    ctx.gather_push_deposit(hit, sp, nan_f, 0, w.dt, w.omega, dG)
    rc, word = ctx.check(raise_on_error=False)
    assert rc == E.ENAN and word & E.DEV_NAN
    fast = parts.clone()
    fast.vel.fill_(1e3)
    ctx.gather_push_deposit(fast, E.Species(w.q, w.m * 1e30, w.w), fields, 0, 1.0, 0.0, dG)
    rc, word = ctx.check(raise_on_error=False)
    assert rc == E.EWALK and word & E.DEV_HOPCAP
    with pytest.raises(E.EtpicError):
        ctx.gather_push_deposit(parts, E.Species(w.q, 0.0, w.w), fields, 0, w.dt, w.omega, dG)


def full_size_step(E, torch, ora, w, precision, tol, sort_first=True):
    """One step of the whole workload on the GPU (sorted by tet, as the benchmark
    runs it) against the oracle on the same state; plus the continuity residual."""
    ctx = E.Context(0)
    ctx.upload_mesh(w.xyz, w.tet_vert)
    parts = E.Particles.from_numpy(w.tet, w.lam, w.vel, w.ids, precision=precision)
    fields = E.Fields.from_numpy(w.e_env, w.b_env, None, w.b_dc)
    sp = E.Species(w.q, w.m, w.w)
    if sort_first:
        dst = parts.empty_like()
        ctx.sort(parts, dst)
        parts = dst
    tin, lin, vin, ids = parts.to_numpy()
    rho0 = torch.zeros(ctx.n_vert, dtype=torch.float64, device="cuda")
    rho1 = torch.zeros_like(rho0)
    dG = torch.zeros(ctx.n_edge, dtype=torch.float64, device="cuda")
    ctx.vertex_charge(parts, sp, rho0)
    ctx.gather_push_deposit(parts, sp, fields, 17, w.dt, w.omega, dG)
    ctx.vertex_charge(parts, sp, rho1)
    r, p = ctx.gauss_residual(dG, rho1, rho0)
    ctx.check()
    M = ora.OracleMesh(w.xyz, w.tet_vert)
    vin64 = vin.astype(np.float64)
    rc, o, dGo = oracle_step(M, (tin, lin, vin64), w, 17, nthreads=NTH)
    assert rc == 0
    tg, lg, vg, _ = parts.to_numpy()
    err = step_errors(w.xyz, w.tet_vert, (tin, lin, vin64), (tg, lg, vg), o, dG.cpu().numpy(), dGo,
                      lam_quantum=fixed_quantum(E, precision))
    print(f"[full-size {w.name} N={len(tg)} precision={precision}] {err} gauss {r / p:.2e}", flush=True)
    assert r / p <= 1e-12
    assert err["tet_mismatch"] <= 2 + 1e-5 * len(tg), err
    assert_within(err, tol, "full size")
    ctx.close()


def test_full_size_200_steps_checkpoints_and_drift(E, torch_cuda, ora):
    """The benchmark's run: 1e7 electrons on the 40^3 x 6 mesh, 200 float64 steps
    with the sort every 10 steps and the XCD remap.  At steps 0, 10, 100 and
    199 the GPU state is handed to the oracle for one step and compared with
    the GPU's next state; the continuity residual is checked at those steps.
    A sample of 20,000 particles (by id) is also run by the oracle for all 200
    steps from the initial state; the drift of the GPU trajectories from it is
    reported (not gated beyond a loose bound: rounding differences grow along
    chaotic orbits)."""
    torch = torch_cuda
    w = synth.make_workload(2)
    ctx = E.Context(0)
    ctx.upload_mesh(w.xyz, w.tet_vert)
    parts = E.Particles.from_numpy(w.tet, w.lam, w.vel, w.ids)
    spare = parts.empty_like()
    fields = E.Fields.from_numpy(w.e_env, w.b_env, None, w.b_dc)
    sp = E.Species(w.q, w.m, w.w)
    M = ora.OracleMesh(w.xyz, w.tet_vert)
    dG = torch.zeros(ctx.n_edge, dtype=torch.float64, device="cuda")
    rho0 = torch.zeros(ctx.n_vert, dtype=torch.float64, device="cuda")
    rho1 = torch.zeros_like(rho0)
    checks = {0, 10, 100, 199}
    for s in range(200):
        if s % 10 == 0:
            ctx.sort(parts, spare)
            parts, spare = spare, parts
        if s in checks:
            tin, lin, vin, _ = parts.to_numpy()
            dG.zero_()
            rho0.zero_()
            rho1.zero_()
            ctx.vertex_charge(parts, sp, rho0)
        ctx.gather_push_deposit(parts, sp, fields, s, w.dt, w.omega, dG)
        if s in checks:
            ctx.vertex_charge(parts, sp, rho1)
            r, p = ctx.gauss_residual(dG, rho1, rho0)
            rc, o, dGo = oracle_step(M, (tin, lin, vin), w, s, nthreads=NTH)
            assert rc == 0
            tg, lg, vg, _ = parts.to_numpy()
            err = step_errors(w.xyz, w.tet_vert, (tin, lin, vin), (tg, lg, vg), o, dG.cpu().numpy(), dGo)
            print(f"[200 steps] step {s}: {err} gauss {r / p:.2e}", flush=True)
            assert r / p <= 1e-12
            assert err["tet_mismatch"] <= 2 + 1e-5 * len(tg), err
            assert_within(err, 1e-12, f"step {s}")
    ctx.check()
    # trajectory drift of a sample, by particle id
    rng = np.random.default_rng(12)
    sample = np.sort(rng.choice(len(w.ids), 20_000, replace=False))
    t, l, v = w.tet[sample].copy(), w.lam[sample].copy(), w.vel[sample].copy()
    for s in range(200):
        rc, _ = M.step(t, l, v, q=w.q, m=w.m, w=w.w, step=s, dt=w.dt, omega=w.omega, e_env=w.e_env,
                       b_env=w.b_env, b_dc=w.b_dc, dG=np.zeros(M.ne), nthreads=NTH)
        assert rc == 0
    tg, lg, vg, ig = parts.to_numpy()
    pos = np.empty_like(ig)
    pos[ig] = np.arange(len(ig))
    k = pos[sample]
    xg = M.positions(tg[k], lg[k])
    xo = M.positions(t, l)
    x0 = M.positions(w.tet[sample], w.lam[sample])
    drift_x = np.abs(xg - xo).max() / np.abs(xo - x0).max()
    drift_v = np.abs(vg[k] - v).max() / np.abs(v).max()
    print(f"[200 steps] drift of 20,000 trajectories after 200 steps: position {drift_x:.2e} of the path "
          f"length scale, velocity {drift_v:.2e}", flush=True)
    assert drift_x < 1e-6 and drift_v < 1e-6
    ctx.close()


def test_full_size_fp64_40cube(E, torch_cuda, ora):
    """The benchmark workload at its real size: 40^3 x 6 tets, 1e7 electrons,
    float64, launch configuration of the benchmark (sorted, XCD remap)."""
    full_size_step(E, torch_cuda, ora, synth.make_workload(2), E.FP64, 1e-12)


def test_full_size_mixed_40cube_5e7(E, torch_cuda, ora):
    """Precision form at its real size: 40^3 x 6 tets, 5e7 electrons, float32
    gather/push with float64 positions and deposit, against the float64 oracle;
    then the compact form (fixed-point barycentrics) on the same workload."""
    w = synth.make_workload(3)
    full_size_step(E, torch_cuda, ora, w, E.MIXED, 2e-5)
    full_size_step(E, torch_cuda, ora, w, E.MIXED_FIXED, 2e-5)


def test_large_box_bunch_one_gpu_share(E, torch_cuda, ora):
    """The large mixed-precision workload's mesh and plasma at one GPU's share:
    2:1:1 box, 160x80x80 x 6 tets (6.1e6), 2.5e7 electrons (1/8 of 2e8: half a
    Gaussian bunch drifting at 1e7 m/s along x, half uniform background),
    B = 1 T along x; mixed and float64 forms against the float64 oracle."""
    w = synth.make_workload(5, n_particles=25_000_000)
    full_size_step(E, torch_cuda, ora, w, E.MIXED, 2e-5)
    full_size_step(E, torch_cuda, ora, w, E.MIXED_FIXED, 2e-5)
    full_size_step(E, torch_cuda, ora, w, E.FP64, 1e-12)
