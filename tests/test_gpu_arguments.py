"""The binding checks every device vector it hands to the library (CUDA
memory, dtype, contiguity, exact element count) and refuses a wrong one with
EINVAL before anything is launched; the context stays usable afterwards."""
import numpy as np
import pytest

from paper_2208_12795_amd import synth

pytestmark = pytest.mark.gpu

EPS0 = 8.8541878128e-12
MU0 = 1.25663706212e-6


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
    w = synth.make_workload(1)
    ctx = E.Context(0)
    ctx.upload_mesh(w.xyz, w.tet_vert)
    f = E.Fields.from_numpy(w.e_env, w.b_env, None, w.b_dc)
    sp = E.Species(w.q, w.m, w.w)
    yield w, ctx, f, sp
    ctx.close()


def einval(E, fn, name):
    with pytest.raises(E.EtpicError) as ei:
        fn()
    assert ei.value.code == E.EINVAL and name in str(ei.value), str(ei.value)


def test_particle_step_vectors(E, torch_cuda, setup):
    torch = torch_cuda
    w, ctx, f, sp = setup
    parts = E.Particles.from_numpy(w.tet, w.lam, w.vel)
    ne, nv = ctx.n_edge, ctx.n_vert
    z = lambda n, dt=torch.float64: torch.zeros(n, dtype=dt, device="cuda")
    before = parts.clone()
    einval(E, lambda: ctx.gather_push_deposit(parts, sp, f, 0, w.dt, w.omega, z(ne - 1)), "dG")
    einval(E, lambda: ctx.gather_push_deposit(parts, sp, f, 0, w.dt, w.omega, z(ne, torch.float32)), "dG")
    einval(E, lambda: ctx.gather_push_deposit(parts, sp, f, 0, w.dt, w.omega, torch.zeros(ne, dtype=torch.float64)),
           "dG")
    einval(E, lambda: ctx.gather_push_deposit(parts, sp, f, 0, w.dt, w.omega, z(ne), rho=z(nv + 1)), "rho")
    einval(E, lambda: ctx.run_steps(parts, sp, f, 0, 2, w.dt, w.omega, z(2 * ne)[::2]), "dG")
    spare = parts.empty_like()
    einval(E, lambda: ctx.sort_run_steps(parts, spare, sp, f, 0, 2, w.dt, w.omega, z(ne + 5)), "dG")
    einval(E, lambda: ctx.vertex_charge(parts, sp, z(nv - 1)), "rho")
    einval(E, lambda: ctx.gauss_residual(z(ne), z(nv), z(nv - 2)), "rho_old")
    einval(E, lambda: ctx.positions(parts, torch.zeros((3, parts.n - 1), dtype=torch.float64, device="cuda")), "xyz")
    einval(E, lambda: ctx.locate(torch.zeros((parts.n, 3), dtype=torch.float64, device="cuda"), parts), "xyz")
    # nothing ran: the particles are as they were, and the context still works
    for a, b in zip(before.to_numpy(), parts.to_numpy()):
        assert (a is None and b is None) or np.array_equal(a, b)
    dG = z(ne)
    ctx.gather_push_deposit(parts, sp, f, 0, w.dt, w.omega, dG)
    ctx.check()
    assert torch.count_nonzero(dG).item() > 0


def test_field_and_solver_vectors(E, torch_cuda, setup):
    torch = torch_cuda
    w, ctx, f, sp = setup
    ne, nf, nv = ctx.n_edge, ctx.n_face, ctx.n_vert
    c = lambda n: torch.zeros((n, 2), dtype=torch.float64, device="cuda")
    ctx.field_setup(w.dt, w.omega, EPS0, MU0)
    einval(E, lambda: ctx.field_spmv(c(ne), c(ne - 1), 1.0, 1.0), "y")
    einval(E, lambda: ctx.field_step(w.dt, c(ne), c(ne), c(ne), c(nf - 1)), "b")
    ctx.ns_setup(EPS0)
    einval(E, lambda: ctx.ns_solve(None, None, 0.0, 0.0, c(nv + 1), None), "x_out")
    einval(E, lambda: ctx.ns_correct(c(ne), c(ne), G=torch.zeros(ne - 1, dtype=torch.float64, device="cuda")), "G")
    einval(E, lambda: ctx.sol_source(torch.zeros(ne, dtype=torch.float64, device="cuda"),
                                     torch.zeros(ne, dtype=torch.float32, device="cuda")), "gs_out")


def test_projector_and_cotree_vectors(E, torch_cuda):
    torch = torch_cuda
    xyz, tv = synth.kuhn_mesh((3, 3, 3), (1.0, 1.0, 1.0), 0.0)
    Q = E.QhProjectors(xyz, tv, EPS0)
    Z = E.CotreeSystem(Q, xyz, tv, MU0)
    c = lambda n: torch.zeros((n, 2), dtype=torch.float64, device="cuda")
    try:
        einval(E, lambda: Q.project_b(c(Q.n_face), c(Q.n_face - 1)), "b_out")
        einval(E, lambda: Q.project_e(c(Q.n_edge), e_ns=c(Q.n_vert - 1)), "e_ns")
        # block 13 maps the nodes off the wall to the cotree faces: an output of
        # node length is refused (cotree edges and faces are equally many on a
        # simply connected mesh, so blocks 12 and 22 could not show it)
        assert Z.n_inner_node != Z.n_cotree_face
        einval(E, lambda: Z.apply(13, c(Z.n_inner_node), c(Z.n_inner_node)), "y")
        einval(E, lambda: Z.b_field(c(Z.n_cotree_face), c(Q.n_face + 1)), "b_out")
        einval(E, lambda: Z.step(1e-11, 0.0, c(Q.n_face), c(Z.n_cotree_edge), src=c(Z.n_cotree_edge - 1)), "src")
        Z.apply(13, c(Z.n_inner_node), c(Z.n_cotree_face))   # the right lengths still work
    finally:
        Z.close()
        Q.close()


def test_particle_and_field_arrays(E, torch_cuda, setup):
    """Particle arrays of the wrong length, dtype or shape, and field arrays
    that do not match the mesh, are refused before any launch."""
    torch = torch_cuda
    w, ctx, f, sp = setup
    good = E.Particles.from_numpy(w.tet, w.lam, w.vel)
    dG = torch.zeros(ctx.n_edge, dtype=torch.float64, device="cuda")
    n = good.n
    bad = {
        "vel": E.Particles(good.lam, good.vel[:, : n - 1].contiguous(), good.tet),
        "lam": E.Particles(good.lam.float(), good.vel, good.tet),
        "tet": E.Particles(good.lam, good.vel, good.tet.long()),
        "ids": E.Particles(good.lam, good.vel, good.tet, torch.arange(n + 1, device="cuda")),
    }
    for name, parts in bad.items():
        einval(E, lambda: ctx.gather_push_deposit(parts, sp, f, 0, w.dt, w.omega, dG), name)
    # the compact storage needs float32 velocities
    fixed = E.Particles.from_numpy(w.tet, w.lam, w.vel, precision=E.MIXED_FIXED)
    einval(E, lambda: ctx.gather_push_deposit(E.Particles(fixed.lam, good.vel, fixed.tet), sp, f, 0, w.dt,
                                              w.omega, dG), "vel")
    short_b = E.Fields(f.e_env, f.b_env[:-1].contiguous(), f.e_dc, f.b_dc)
    einval(E, lambda: ctx.gather_push_deposit(good, sp, short_b, 0, w.dt, w.omega, dG), "b_env")
    assert torch.count_nonzero(dG).item() == 0
