"""GPU coarse field step at the fine step (three envelope snapshots, quadratic
Lagrange reconstruction at every fine time, fine Lorentz steps, path
integrals summed over the fine steps) against the oracle's coarse step."""
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


def gpu_snaps(E, w, snaps):
    return [E.Fields.from_numpy(e, b, None, w.b_dc) for e, b in snaps]


@pytest.mark.parametrize("config,n,fine,precision,tol", [(1, None, 8, 0, 1e-12), (1, None, 8, 1, 2e-5),
                                                        (2, 200_003, 4, 0, 1e-12), (2, 200_003, 4, 1, 2e-5)])
def test_coarse_step_matches_oracle(E, torch_cuda, ora, config, n, fine, precision, tol):
    torch = torch_cuda
    w = synth.make_workload(config, n_particles=n)
    order = np.argsort(w.tet, kind="stable")
    w.tet, w.lam, w.vel, w.ids = w.tet[order], w.lam[order], w.vel[order], w.ids[order]
    snaps = synth.envelope_snapshots(w, seed=config)
    t_c, dtc = 37 * fine * w.dt, fine * w.dt
    print(f"[coarse] config {config} N={w.tet.shape[0]} fine steps {fine} precision {precision}", flush=True)
    ctx = E.Context(0)
    ctx.upload_mesh(w.xyz, w.tet_vert)
    parts = E.Particles.from_numpy(w.tet, w.lam, w.vel, w.ids, precision=precision)
    sp = E.Species(w.q, w.m, w.w)
    tin, lin, vin, _ = parts.to_numpy()
    dG = torch.zeros(ctx.n_edge, dtype=torch.float64, device="cuda")
    rho0 = torch.zeros(ctx.n_vert, dtype=torch.float64, device="cuda")
    rho1 = torch.zeros_like(rho0)
    ctx.vertex_charge(parts, sp, rho0)
    ctx.coarse_step(parts, sp, gpu_snaps(E, w, snaps), t_c, dtc, fine, w.omega, dG, rho=rho1)
    r, p = ctx.gauss_residual(dG, rho1, rho0)
    ctx.check()
    M = ora.OracleMesh(w.xyz, w.tet_vert)
    t, l, v = tin.copy(), lin.copy(), vin.astype(np.float64)
    dGo = np.zeros(M.ne)
    rc = M.coarse_step(t, l, v, q=w.q, m=w.m, w=w.w, e_snaps=[s[0] for s in snaps], b_snaps=[s[1] for s in snaps],
                       t_coarse=t_c, dt_coarse=dtc, fine_steps=fine, omega=w.omega, b_dc=w.b_dc, dG=dGo,
                       nthreads=NTH)
    assert rc == 0
    tg, lg, vg, _ = parts.to_numpy()
    err = step_errors(w.xyz, w.tet_vert, (tin, lin, vin), (tg, lg, vg), (t, l, v), dG.cpu().numpy(), dGo)
    print(f"[coarse] {err} gauss {r / p:.2e}", flush=True)
    assert r / p <= 1e-12
    assert err["tet_mismatch"] <= 2 + 1e-4 * len(tg), err
    assert_within(err, tol, "coarse step")
    ctx.close()


def test_equal_snapshots_are_fine_steps(E, torch_cuda):
    """Three equal snapshots: the coarse step is the same as fine_steps calls of
    gather_push_deposit at the same times (weights sum to one)."""
    torch = torch_cuda
    w = synth.make_workload(1)
    fine = 5
    ctx = E.Context(0)
    ctx.upload_mesh(w.xyz, w.tet_vert)
    f = E.Fields.from_numpy(w.e_env, w.b_env, None, w.b_dc)
    sp = E.Species(w.q, w.m, w.w)
    p1 = E.Particles.from_numpy(w.tet, w.lam, w.vel, w.ids)
    p2 = p1.clone()
    g1 = torch.zeros(ctx.n_edge, dtype=torch.float64, device="cuda")
    g2 = torch.zeros_like(g1)
    n0 = 11
    ctx.coarse_step(p1, sp, [f, f, f], n0 * fine * w.dt, fine * w.dt, fine, w.omega, g1)
    for j in range(fine):
        ctx.gather_push_deposit(p2, sp, f, n0 * fine + j, w.dt, w.omega, g2)
    a, b = p1.to_numpy(), p2.to_numpy()
    assert np.array_equal(a[0], b[0])
    assert np.abs(a[1] - b[1]).max() < 1e-15
    assert np.abs(a[2] - b[2]).max() < 1e-14 * np.abs(b[2]).max()
    assert torch.allclose(g1, g2, rtol=0, atol=1e-13 * g2.abs().max().item())
    with pytest.raises(E.EtpicError):
        ctx.coarse_step(p1, sp, [f, f, f], 0.0, w.dt, 0, w.omega, g1)
    ctx.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_run_steps_equals_single_steps(E, torch_cuda, precision):
    """Ten steps in one call (the coefficient pass of the next step sharing a
    launch with the walk of this one) against ten single-step calls: the
    particle state is identical, the currents equal to the atomics' rounding,
    the charge after the last step matches a separate scatter, and the kernel
    timings cover every step."""
    torch = torch_cuda
    w = synth.make_workload(2, n_particles=300_000)
    order = np.argsort(w.tet, kind="stable")
    w.tet, w.lam, w.vel, w.ids = w.tet[order], w.lam[order], w.vel[order], w.ids[order]
    ctx = E.Context(0)
    ctx.upload_mesh(w.xyz, w.tet_vert)
    f = E.Fields.from_numpy(w.e_env, w.b_env, None, w.b_dc)
    sp = E.Species(w.q, w.m, w.w)
    p1 = E.Particles.from_numpy(w.tet, w.lam, w.vel, w.ids, precision=precision)
    p2 = p1.clone()
    g1 = torch.zeros(ctx.n_edge, dtype=torch.float64, device="cuda")
    g2 = torch.zeros_like(g1)
    rho = torch.zeros(ctx.n_vert, dtype=torch.float64, device="cuda")
    ctx.kernel_time(reset=True)
    ctx.run_steps(p1, sp, f, 3, 10, w.dt, w.omega, g1, rho=rho, flags=E.STEP_XCD_REMAP | E.STEP_TIMING_ALL)
    kt, nl = ctx.kernel_time(reset=True)
    assert nl == 10 and kt["steps_push"] == 10 and kt["steps_sort"] == 0
    assert min(kt["push"], kt["coef"], kt["walk"]) > 0.0 and kt["push_sort"] == 0.0
    for j in range(10):
        ctx.gather_push_deposit(p2, sp, f, 3 + j, w.dt, w.omega, g2)
    ctx.check()
    a, b = p1.to_numpy(), p2.to_numpy()
    for x, y in zip(a[:3], b[:3]):
        assert np.array_equal(x, y)
    assert torch.allclose(g1, g2, rtol=0, atol=1e-13 * g2.abs().max().item())
    rho2 = torch.zeros_like(rho)
    ctx.vertex_charge(p1, sp, rho2)
    assert torch.allclose(rho, rho2, rtol=0, atol=1e-13 * rho2.abs().max().item())
    ctx.close()


def test_step_timing_modes(E, torch_cuda):
    """STEP_TIMING times the particle kernel of every step and nothing else;
    STEP_TIMING_ALL also the coefficient, walk and edge-gather kernels; a
    sorting call books its first particle kernel apart.  Timing changes no
    result: the same steps without timing give identical particles."""
    torch = torch_cuda
    w = synth.make_workload(2, n_particles=200_000)
    ctx = E.Context(0)
    ctx.upload_mesh(w.xyz, w.tet_vert)
    f = E.Fields.from_numpy(w.e_env, w.b_env, None, w.b_dc)
    sp = E.Species(w.q, w.m, w.w)
    p = E.Particles.from_numpy(w.tet, w.lam, w.vel, w.ids)
    q = p.clone()
    g = torch.zeros(ctx.n_edge, dtype=torch.float64, device="cuda")
    ctx.kernel_time(reset=True)
    ctx.run_steps(p, sp, f, 0, 6, w.dt, w.omega, g, flags=E.STEP_XCD_REMAP | E.STEP_TIMING)
    kt, nl = ctx.kernel_time(reset=True)
    assert nl == 6 and kt["steps_push"] == 6 and kt["push"] > 0.0
    assert kt["coef"] == 0.0 and kt["walk"] == 0.0 and kt["push_sort"] == 0.0
    ctx.run_steps(q, sp, f, 0, 6, w.dt, w.omega, g, flags=E.STEP_XCD_REMAP)
    ctx.kernel_time(reset=True)
    assert ctx.kernel_time(reset=True)[1] == 0
    for x, y in zip(p.to_numpy(), q.to_numpy()):
        assert np.array_equal(x, y)
    dst = p.empty_like()
    ctx.sort_run_steps(p, dst, sp, f, 6, 4, w.dt, w.omega, g, flags=E.STEP_XCD_REMAP | E.STEP_TIMING_ALL)
    kt, nl = ctx.kernel_time(reset=True)
    assert nl == 4 and kt["steps_sort"] == 1 and kt["steps_push"] == 3
    assert min(kt["push"], kt["push_sort"], kt["coef"], kt["walk"]) > 0.0
    ctx.check()
    ctx.close()
