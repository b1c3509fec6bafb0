"""The allocation-free continuity residual (etpic_gauss_residual_noalloc)
against etpic_gauss_residual, through the C ABI: the same two maxima bit for
bit (both take the maximum of the same per-vertex values), on two calls in a
row, the second on a smaller mesh, then again on the first; a non-finite
input is an error on both."""
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


def stepped(E, torch, w, step=0):
    """(ctx, dG, rho_new, rho_old) of one float64 step of workload w"""
    ctx = E.Context(0)
    ctx.upload_mesh(w.xyz, w.tet_vert)
    parts = E.Particles.from_numpy(w.tet, w.lam, w.vel, w.ids)
    fields = E.Fields.from_numpy(w.e_env, w.b_env, None, w.b_dc)
    sp = E.Species(w.q, w.m, w.w)
    r0 = torch.zeros(ctx.n_vert, dtype=torch.float64, device="cuda")
    r1 = torch.zeros_like(r0)
    dG = torch.zeros(ctx.n_edge, dtype=torch.float64, device="cuda")
    ctx.vertex_charge(parts, sp, r0)
    ctx.gather_push_deposit(parts, sp, fields, step, w.dt, w.omega, dG)
    ctx.vertex_charge(parts, sp, r1)
    return ctx, dG, r1, r0


def test_noalloc_residual_equals_residual(torch_cuda):
    from paper_2208_12795_amd import etpic as E
    torch = torch_cuda
    big = synth.make_workload(2, n_particles=2_000_000)     # 68,921 vertices
    small = synth.make_workload(1)                           # 216 vertices
    print(f"[no-alloc] meshes nv {big.xyz.shape[0]} then {small.xyz.shape[0]}", flush=True)
    cb, gb, r1b, r0b = stepped(E, torch, big)
    cs, gs, r1s, r0s = stepped(E, torch, small)
    for ctx, g, r1, r0 in ((cb, gb, r1b, r0b), (cs, gs, r1s, r0s), (cb, gb, r1b, r0b)):
        ref = ctx.gauss_residual(g, r1, r0)
        got = ctx.gauss_residual_noalloc(g, r1, r0)
        print(f"[no-alloc] nv {ctx.n_vert}: {got} vs {ref}", flush=True)
        assert got == ref
        assert got[0] <= 1e-12 * got[1]
        # a planted violation, then arbitrary arrays: still the same numbers
        bad = g.clone()
        bad[ctx.n_edge // 2] += 1e-9 * got[1]
        assert ctx.gauss_residual_noalloc(bad, r1, r0) == ctx.gauss_residual(bad, r1, r0)
        rng = np.random.default_rng(ctx.n_vert)
        a = [torch.from_numpy(rng.standard_normal(n)).cuda() for n in (ctx.n_edge, ctx.n_vert, ctx.n_vert)]
        assert ctx.gauss_residual_noalloc(*a) == ctx.gauss_residual(*a)
    nan = gs.clone()
    nan[3] = float("nan")
    with pytest.raises(E.EtpicError) as ei:
        cs.gauss_residual_noalloc(nan, r1s, r0s)
    assert ei.value.code == E.ENAN
    assert cs.gauss_residual_noalloc(gs, r1s, r0s) == cs.gauss_residual(gs, r1s, r0s)
    cb.check()
    cs.check()
    cb.close()
    cs.close()
