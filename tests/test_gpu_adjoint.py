"""GPU adjoint of the float64 particle steps against the oracle's reverse mode
and against central finite differences of the GPU forward run."""
import os
import time

import numpy as np
import pytest

from paper_2208_12795_amd import synth

pytestmark = pytest.mark.gpu

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


def gpu_setup(E, w):
    ctx = E.Context(0)
    ctx.upload_mesh(w.xyz, w.tet_vert)
    parts = E.Particles.from_numpy(w.tet, w.lam, w.vel, w.ids)
    fields = E.Fields.from_numpy(w.e_env, w.b_env, None, w.b_dc)
    return ctx, parts, fields


def gpu_grad(E, torch, ctx, parts, fields, w, nsteps, every, seed_fn):
    """forward (checkpointed) + backward through the C ABI; returns (v_final, grad_e, vbar0, xbar0)."""
    sp = E.Species(w.q, w.m, w.w)
    work = parts.clone()
    ws = torch.empty(ctx.adjoint_workspace_bytes(work.n, nsteps, every), dtype=torch.uint8, device="cuda")
    ctx.forward_checkpointed(work, sp, fields, 0, nsteps, w.dt, w.omega, every, ws)
    vfin = work.vel.clone()
    vbar = seed_fn(vfin).contiguous()
    xbar = torch.zeros_like(vbar)
    g = torch.zeros((ctx.n_edge, 2), dtype=torch.float64, device="cuda")
    ctx.backward(work.n, sp, fields, 0, nsteps, w.dt, w.omega, every, ws, vbar, xbar, g)
    ctx.check()
    gz = g[:, 0].cpu().numpy() + 1j * g[:, 1].cpu().numpy()
    return vfin.cpu().numpy().T, gz, vbar.cpu().numpy().T, xbar.cpu().numpy().T


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


@pytest.mark.parametrize("every", [1, 3, 5, 20])
def test_adjoint_matches_oracle_small(E, torch_cuda, ora, every):
    """1,000 electrons, 20 steps, several checkpoint spacings (ragged last segment
    for 3): envelope gradient and initial-state adjoints against the oracle's
    reverse mode with the same seed (m w v_final)."""
    torch = torch_cuda
    w = synth.make_workload(1)
    ctx, parts, fields = gpu_setup(E, w)
    K = 20
    vfin, g, vb0, xb0 = gpu_grad(E, torch, ctx, parts, fields, w, K, every, lambda v: w.m * w.w * v)
    M = ora.OracleMesh(w.xyz, w.tet_vert)
    rc, go, vbo, xbo = M.vjp(w.tet, w.lam, w.vel, q=w.q, m=w.m, w=w.w, step0=0, nsteps=K, dt=w.dt, omega=w.omega,
                             e_env=w.e_env, b_env=w.b_env, b_dc=w.b_dc, vbar=w.m * w.w * vfin, nthreads=NTH)
    assert rc == 0
    print(f"[adjoint small every={every}] grad rel {rel(g, go):.2e} vbar0 {rel(vb0, vbo):.2e} xbar0 {rel(xb0, xbo):.2e}")
    assert rel(g, go) < 1e-10
    assert np.linalg.norm(g - go) / np.linalg.norm(go) < 1e-10
    assert rel(vb0, vbo) < 1e-10
    assert rel(xb0, xbo) < 1e-10
    ctx.close()


def test_adjoint_with_crossings_and_walls(E, torch_cuda, ora):
    """Steps of a sizeable fraction of a cell: face crossings and wall reflections
    enter the adjoint through the reflection Jacobian."""
    torch = torch_cuda
    w = synth.make_workload(1, n_particles=2000)
    w.vel = w.vel * 40.0
    w.dt = 1e-9
    ctx, parts, fields = gpu_setup(E, w)
    K = 10
    vfin, g, vb0, xb0 = gpu_grad(E, torch, ctx, parts, fields, w, K, 4, lambda v: w.m * w.w * v)
    M = ora.OracleMesh(w.xyz, w.tet_vert)
    rc, go, vbo, xbo = M.vjp(w.tet, w.lam, w.vel, q=w.q, m=w.m, w=w.w, step0=0, nsteps=K, dt=w.dt, omega=w.omega,
                             e_env=w.e_env, b_env=w.b_env, b_dc=w.b_dc, vbar=w.m * w.w * vfin, nthreads=NTH)
    assert rc == 0
    print(f"[adjoint crossings] grad rel {rel(g, go):.2e} vbar0 {rel(vb0, vbo):.2e} xbar0 {rel(xb0, xbo):.2e}")
    assert rel(g, go) < 1e-9 and rel(vb0, vbo) < 1e-9 and rel(xb0, xbo) < 1e-9
    ctx.close()


def test_autograd_differentiation_workload(E, torch_cuda, ora):
    """Differentiation workload: 20^3 x 6 tets, 2e6 electrons, 20 steps,
    checkpoint every 5.  Gradient of the kinetic energy at step 20 with respect
    to the complex edge envelope through torch.autograd: against the oracle's
    gradient (all edges) and against central differences (h = 1e-6 V, real and
    imaginary parts) on 50 random edges, evaluated in factored form."""
    torch = torch_cuda
    from paper_2208_12795_amd.autograd import particle_steps
    w = synth.make_workload(4)
    ctx, parts, fields = gpu_setup(E, w)
    sp = E.Species(w.q, w.m, w.w)
    K, every = 20, 5
    z = torch.tensor(w.e_env, dtype=torch.complex128, device="cuda", requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    v = particle_steps(z, ctx, parts, sp, fields.b_env, b_dc=fields.b_dc, nsteps=K, dt=w.dt, omega=w.omega,
                       checkpoint_every=every)
    ke = 0.5 * w.m * w.w * (v * v).sum()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ke.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    print(f"[adjoint 20^3 x 6, 2e6] forward {1e3 * (t1 - t0):.1f} ms, backward {1e3 * (t2 - t1):.1f} ms, "
          f"ratio {(t2 - t1) / (t1 - t0):.2f}")
    g = z.grad.cpu().numpy()
    # oracle gradient, same seed
    vfin = v.detach().cpu().numpy().T
    M = ora.OracleMesh(w.xyz, w.tet_vert)
    rc, go, _, _ = M.vjp(w.tet, w.lam, w.vel, q=w.q, m=w.m, w=w.w, step0=0, nsteps=K, dt=w.dt, omega=w.omega,
                         e_env=w.e_env, b_env=w.b_env, b_dc=w.b_dc, vbar=w.m * w.w * vfin, nthreads=NTH)
    assert rc == 0
    print(f"[adjoint 20^3 x 6, 2e6] vs oracle: max rel {rel(g, go):.2e}")
    assert rel(g, go) < 1e-10
    # the oracle's tangent-linear (forward mode) along a dense random direction
    # and single-edge directions: dKE = Re(g).Re(de) + Im(g).Im(de)
    rng_d = np.random.default_rng(2023)
    dirs = [rng_d.standard_normal(ctx.n_edge) + 1j * rng_d.standard_normal(ctx.n_edge)]
    for e, unit in zip(rng_d.choice(ctx.n_edge, 4, replace=False), (1.0, 1j, 1.0, 1j)):
        d1 = np.zeros(ctx.n_edge, complex)
        d1[e] = unit
        dirs.append(d1)
    for de in dirs:
        rc, dv, _ = M.jvp(w.tet, w.lam, w.vel, q=w.q, m=w.m, step0=0, nsteps=K, dt=w.dt, omega=w.omega,
                          e_env=w.e_env, b_env=w.b_env, b_dc=w.b_dc, de=de, nthreads=NTH)
        assert rc == 0
        fwd = float((w.m * w.w * vfin * dv).sum())
        mine = float((g.real * de.real).sum() + (g.imag * de.imag).sum())
        scale = float((np.abs(g) * np.abs(de)).sum())
        print(f"[adjoint 20^3 x 6, 2e6] tangent-linear check: forward {fwd:.6e} adjoint {mine:.6e} "
              f"rel {abs(fwd - mine) / scale:.2e}")
        assert abs(fwd - mine) <= 1e-10 * scale
    # central differences of the GPU forward run
    rng = np.random.default_rng(2022)
    probes = rng.choice(ctx.n_edge, 50, replace=False)
    base = torch.view_as_real(z.detach()).contiguous()

    def final_v(ee):
        work = parts.clone()
        f = E.Fields(ee, fields.b_env, None, fields.b_dc)
        dG = torch.zeros(ctx.n_edge, dtype=torch.float64, device="cuda")
        for s in range(K):
            ctx.gather_push_deposit(work, sp, f, s, w.dt, w.omega, dG)
        return work.vel

    # A DoF change of h moves a particle's velocity by ~70 h m/s per volt, i.e.
    # ~1e4-1e6 ulps at h = 1e-6 V, so the float64 rounding of the two forward
    # runs leaves ~1e-4 relative noise in v+ - v- (and 100x less at h = 1e-4 V).
    # Errors are measured against |g| + the median |g| of the probes, so edges
    # with near-cancelling contributions do not dominate.
    gp = np.concatenate([g[probes].real, g[probes].imag])
    floor = np.median(np.abs(gp))
    for h, med_tol, max_tol in ((1e-6, 1e-4, 3e-3), (1e-4, 2e-6, 5e-5)):
        errs = []
        for e in probes:
            for comp in (0, 1):
                ep, em = base.clone(), base.clone()
                ep[e, comp] += h
                em[e, comp] -= h
                vp, vm = final_v(ep), final_v(em)
                fd = (0.5 * w.m * w.w * ((vp - vm) * (vp + vm)).sum()).item() / (2 * h)
                gg = g[e].real if comp == 0 else g[e].imag
                errs.append(abs(fd - gg) / (abs(gg) + floor))
        errs = np.array(errs)
        print(f"[adjoint 20^3 x 6, 2e6] FD h={h:g} V on 50 edges x (re, im): median {np.median(errs):.2e} "
              f"worst {errs.max():.2e}")
        assert np.median(errs) < med_tol and errs.max() < max_tol
    ctx.close()


def test_autograd_composes_with_torch(E, torch_cuda):
    """The returned gradient composes with torch's own complex autograd:
    d/dz [KE(z) + sum |z|^2] = grad KE + 2 z."""
    torch = torch_cuda
    from paper_2208_12795_amd.autograd import particle_steps
    w = synth.make_workload(1, n_particles=400)
    ctx, parts, fields = gpu_setup(E, w)
    sp = E.Species(w.q, w.m, w.w)
    z = torch.tensor(w.e_env, dtype=torch.complex128, device="cuda", requires_grad=True)
    v = particle_steps(z, ctx, parts, sp, fields.b_env, b_dc=fields.b_dc, nsteps=7, dt=w.dt, omega=w.omega,
                       checkpoint_every=3)
    (0.5 * w.m * w.w * (v * v).sum()).backward()
    g1 = z.grad.clone()
    z.grad = None
    v = particle_steps(z, ctx, parts, sp, fields.b_env, b_dc=fields.b_dc, nsteps=7, dt=w.dt, omega=w.omega,
                       checkpoint_every=3)
    scale = 1e-30
    (0.5 * w.m * w.w * (v * v).sum() + scale * (z.abs() ** 2).sum()).backward()
    assert torch.allclose(z.grad, g1 + 2 * scale * z.detach(), rtol=1e-12, atol=1e-12 * g1.abs().max().item())
    ctx.close()
