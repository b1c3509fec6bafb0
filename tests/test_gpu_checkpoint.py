"""Checkpoint and resume of the particle state through a host file
(etpic_checkpoint_write / _read): a run stopped at a checkpoint and resumed
from it in new arrays continues exactly as the run that did not stop (the
particle state bit for bit, the currents to the rounding of the atomics'
order), in every precision, with and without ids; recovery from a step that
raised a device error restores the last checkpoint; mismatched arrays, another
mesh and a corrupted file are refused."""
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


@pytest.fixture(scope="module")
def setup(E, torch_cuda):
    w = synth.make_workload(2, n_particles=300_000)
    ctx = E.Context(0)
    ctx.upload_mesh(w.xyz, w.tet_vert)
    f = E.Fields.from_numpy(w.e_env, w.b_env, None, w.b_dc)
    sp = E.Species(w.q, w.m, w.w)
    yield w, ctx, f, sp
    ctx.close()


def canonical(parts):
    """(tet, lam, v, ids) in a fixed particle order: by id, or without ids by
    the whole state.  The counting sort places the runs of one tet in the order
    their cursor atomics land, so two equal runs may hold the same particles
    in different orders."""
    tet, lam, vel, ids = parts.to_numpy()
    if ids is not None:
        o = np.argsort(ids, kind="stable")
    else:
        o = np.lexsort((*vel.T, *lam.T, tet))
    return tet[o], lam[o], vel[o], None if ids is None else ids[o]


def run_blocks(E, torch, ctx, parts, sp, f, w, step0, nblocks, dG):
    """nblocks sort+10-step blocks from step0; returns the particles"""
    spare = parts.empty_like()
    for b in range(nblocks):
        ctx.sort_run_steps(parts, spare, sp, f, step0 + 10 * b, 10, w.dt, w.omega, dG)
        parts, spare = spare, parts
    return parts


@pytest.mark.parametrize("precision", [0, 1, 2])
@pytest.mark.parametrize("with_ids", [True, False])
def test_resume_continues_the_run(E, torch_cuda, setup, tmp_path, precision, with_ids):
    torch = torch_cuda
    w, ctx, f, sp = setup
    parts = E.Particles.from_numpy(w.tet, w.lam, w.vel, w.ids if with_ids else None, precision=precision)
    dG = torch.zeros(ctx.n_edge, dtype=torch.float64, device="cuda")
    parts = run_blocks(E, torch, ctx, parts, sp, f, w, 0, 1, dG)
    path = str(tmp_path / f"ck_{precision}_{with_ids}.bin")
    ctx.checkpoint_write(parts, 10, path)
    info = E.checkpoint_info(path)
    assert info == {"n": parts.n, "precision": precision, "step": 10, "has_id": with_ids}
    # the run that goes on
    g_ref = torch.zeros_like(dG)
    ref = run_blocks(E, torch, ctx, parts, sp, f, w, 10, 2, g_ref)
    ctx.check()
    # the run resumed from the file, in new arrays
    back, step = ctx.checkpoint_load(path)
    assert step == 10 and back.precision == precision and (back.ids is not None) == with_ids
    g_res = torch.zeros_like(dG)
    res = run_blocks(E, torch, ctx, back, sp, f, w, step, 2, g_res)
    ctx.check()
    for a, b in zip(canonical(ref), canonical(res)):
        if a is None:
            assert b is None
        else:
            assert np.array_equal(a, b)
    tol = 1e-13 * g_ref.abs().max().item()
    assert torch.allclose(g_res, g_ref, rtol=0, atol=tol)
    print(f"[checkpoint] precision {precision} ids {with_ids}: {parts.n} particles, file "
          f"{info}", flush=True)


def test_recovery_after_a_device_error(E, torch_cuda, setup, tmp_path):
    """A step whose displacements span ~100 box lengths (time step 1e-4 s,
    the fields switched off by a huge mass) trips the walk's hop cap (the
    device status reports it); the run is restored from its last checkpoint
    and continues as if the bad step had never been taken."""
    torch = torch_cuda
    w, ctx, f, sp = setup
    parts = E.Particles.from_numpy(w.tet, w.lam, w.vel, w.ids)
    dG = torch.zeros(ctx.n_edge, dtype=torch.float64, device="cuda")
    parts = run_blocks(E, torch, ctx, parts, sp, f, w, 0, 1, dG)
    path = str(tmp_path / "recover.bin")
    ctx.checkpoint_write(parts, 10, path)
    clean = run_blocks(E, torch, ctx, parts.clone(), sp, f, w, 10, 1, torch.zeros_like(dG))
    ctx.check()
    bad = parts.clone()
    ctx.run_steps(bad, E.Species(w.q, w.m * 1e30, w.w), f, 10, 1, 1e-4, 0.0, torch.zeros_like(dG))
    rc, word = ctx.check(raise_on_error=False)
    assert rc == E.EWALK and word & E.DEV_HOPCAP
    step = ctx.checkpoint_read(bad, path)
    assert step == 10
    again = run_blocks(E, torch, ctx, bad, sp, f, w, step, 1, torch.zeros_like(dG))
    ctx.check()
    for a, b in zip(canonical(clean), canonical(again)):
        assert np.array_equal(a, b)


def test_mismatches_are_refused(E, torch_cuda, setup, tmp_path):
    torch = torch_cuda
    w, ctx, f, sp = setup
    parts = E.Particles.from_numpy(w.tet[:5000], w.lam[:5000], w.vel[:5000], w.ids[:5000])
    path = str(tmp_path / "m.bin")
    ctx.checkpoint_write(parts, 3, path)

    def code(fn):
        with pytest.raises(E.EtpicError) as ei:
            fn()
        return ei.value.code

    # another precision, count, or id presence
    mixed = E.Particles.from_numpy(w.tet[:5000], w.lam[:5000], w.vel[:5000], w.ids[:5000], precision=E.MIXED)
    assert code(lambda: ctx.checkpoint_read(mixed, path)) == E.EINVAL
    fewer = E.Particles.from_numpy(w.tet[:4000], w.lam[:4000], w.vel[:4000], w.ids[:4000])
    assert code(lambda: ctx.checkpoint_read(fewer, path)) == E.EINVAL
    no_ids = E.Particles.from_numpy(w.tet[:5000], w.lam[:5000], w.vel[:5000], None)
    assert code(lambda: ctx.checkpoint_read(no_ids, path)) == E.EINVAL
    # another mesh (one vertex moved by one unit in the last place)
    xyz2 = w.xyz.copy()
    k = int(np.flatnonzero(np.all((xyz2 > 0.01) & (xyz2 < 0.99), axis=1))[0])
    xyz2[k, 0] = np.nextafter(xyz2[k, 0], 1.0)
    ctx2 = E.Context(0)
    ctx2.upload_mesh(xyz2, w.tet_vert)
    assert code(lambda: ctx2.checkpoint_read(parts.clone(), path)) == E.EMESH
    ctx2.close()
    # a flipped bit in the velocities: EIO, arrays partly overwritten
    raw = bytearray(open(path, "rb").read())
    raw[136 + 4 * 5000 + 3 * 8 * 5000 + 123] ^= 0x10
    bad = str(tmp_path / "bad.bin")
    open(bad, "wb").write(bytes(raw))
    assert code(lambda: ctx.checkpoint_read(parts.clone(), bad)) == E.EIO
    # writing over an existing checkpoint replaces it whole
    ctx.checkpoint_write(parts, 4, path)
    assert E.checkpoint_info(path)["step"] == 4


def test_empty_particle_set_round_trip(E, torch_cuda, setup, tmp_path):
    """No particles: the file is a header alone and reads back as such."""
    torch = torch_cuda
    w, ctx, f, sp = setup
    empty = E.Particles.from_numpy(w.tet[:0], w.lam[:0], w.vel[:0], None)
    path = str(tmp_path / "empty.bin")
    ctx.checkpoint_write(empty, 42, path)
    import os
    assert os.path.getsize(path) == 136
    assert E.checkpoint_info(path) == {"n": 0, "precision": 0, "step": 42, "has_id": False}
    back, step = ctx.checkpoint_load(path)
    assert step == 42 and back.n == 0
