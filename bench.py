#!/usr/bin/env python3
"""Throughput of the envelope-tracking particle-mesh step on one MI355X.

A step is one pass of the particle path over all particles: the per-tet
carrier-rotated field coefficients (k_tet_coef), the particle kernel (gather,
Boris push, in-tet path-integral deposit with same-tet sums before the edge
atomics; k_push), the walk of the particles that left their tet (k_walk), and
the counting sort by tet every `--sort-every` steps (amortised, inside the
timed region).  The steps between two sorts go through one multi-step call,
in which the walk of a step and the coefficient pass of the next share one
kernel launch.  Default workload: the 40^3 x 6 jittered Kuhn mesh (384,000
tets) with 10,000,000 electrons (Maxwellian, 1e6 m/s), an 8-mode envelope on a
10 GHz carrier, B = 0.5 T, dt = 1e-12 s; `--workload large-box` runs the 2:1:1
160x80x80 x 6 mesh with 2e8 electrons (bunch + background, B = 1 T along x).
Inputs are resident in HBM before the timed region starts, and before each
form's warmup steps ~50 ms of untimed streaming over its particle arrays lets
the GPU's clocks settle (without it the first timed steps of a short run are
~3 % slower).

Prints ONE JSON line.  `value` is the float64 form; the mixed form (float32
gather/push on barycentrics, float64 positions and deposit) is reported under
"mixed", and the compact mixed form (the same arithmetic, barycentrics stored
as 32-bit fixed point, so 52 instead of 76 bytes of particle state move per
step) under "mixed_fixed".  The roofline figure is for the dominant kernel (the particle
kernel), timed with HIP events recorded on its launch stream; beside it the
rate its access pattern alone reaches (a stream probe over the same particle
arrays), a device copy, and the whole step's algorithmic bytes over the time
per step.  After the timed steps a few single steps are run with the
continuity residual of each, timed apart ("logged").  Side entries (not in
`value`): the precision workload (same mesh, 5e7 electrons) and the large box
(2e8 electrons on 6.1M tets), all three forms, each with its own roofline,
and on the large box a run of 1,000 mixed-form steps (re-sort every 10) with
the continuity residual computed and checked after every step; the
field update, the Gauss-law solve and loops, the projectors, the multi-rate
and downshifted steps, the adjoint; and the float64 oracle on the host's
cores (`cpu_baseline`).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# vector-ALU issue ceiling: 256 CUs x 4 SIMDs, one 64-lane wavefront instruction
# per 4 cycles of a 16-lane SIMD, at 2.4 GHz (wavefront instructions per second)
VALU_PEAK_PER_S = 256 * 4 * 2.4e9 / 4
# Algorithmic bytes of the particle kernel (what it must move per unit):
#  per particle-step: state read (tet 4 B, lam 3x8, v 3x8) and written back
#                     (lam 3x8, v 3x8): 100 B in float64; v is float32 in the
#                     mixed form: 76 B; with the barycentrics also in 32-bit
#                     fixed point (compact mixed form): 4 + 2 x (12 + 12) = 52 B.
#                     (The tet id is rewritten only for the particles that
#                     leave their tet, by the walk kernel.)
#  per tet and step : its coefficient row (24 reals), gradient row (9 reals) and
#                     edge ids (6 x 4 B), read once: 288 B (float64), 156 B (mixed)
#  per edge and step: the current accumulator read + written once (16 B)
BYTES_PER_PARTICLE = {"fp64": 100, "mixed": 76, "mixed_fixed": 52}
# per tet and launch: the step's coefficient row (A_0, beta, C_0, b: 10 reals),
# the gradient row (grad l_1..3: 9 reals), the six edge ids (24 B) and the
# geometry row (r_k - r_0, k = 1..3: 9 reals); reals float64, or float32 in
# both mixed forms
BYTES_PER_TET = {"fp64": 248, "mixed": 136, "mixed_fixed": 136}
BYTES_PER_EDGE = 16
KERNEL_NAME = {"fp64": "k_push<double>", "mixed": "k_push<float>", "mixed_fixed": "k_push_fixed"}
# Algorithmic bytes of a whole step (what the method must move per particle-step
# and per tet, independent of how the kernels split the work): the particle
# state read and written, tet included (2 x (lam 24 + v 24 + tet 4) = 104 B in
# float64, 2 x (24 + 12 + 4) = 80 B with float32 velocities); per tet and step
# its field DoFs, geometry and ids (~320 B); and the periodic sort amortised:
# per particle and sort its state and id read and written plus key and offset
# (2 x (52 + 8) + 8 = 128 B in float64, 2 x (40 + 8) + 8 = 104 B mixed).
# The compact mixed form stores the barycentrics as 32-bit fixed point:
# 2 x (12 + 12 + 4) = 56 B per particle-step, 2 x (28 + 8) + 8 = 80 B per sort.
STEP_BYTES_PER_PARTICLE = {"fp64": 104, "mixed": 80, "mixed_fixed": 56}
STEP_BYTES_PER_TET = 320
SORT_BYTES_PER_PARTICLE = {"fp64": 128, "mixed": 104, "mixed_fixed": 80}
REAL = {"fp64": "double", "mixed": "float", "mixed_fixed": "float"}
FORM_DTYPE = {"fp64": "f64", "mixed": "f32 gather/push, f64 deposit",
              "mixed_fixed": "f32 gather/push, f64 deposit, barycentrics stored as u32 (2^-32 fixed point)"}


def precision_of(E, form):
    return {"fp64": E.FP64, "mixed": E.MIXED, "mixed_fixed": E.MIXED_FIXED}[form]
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "k_push_hbm_traffic_40cube_1e7.md")
TRAFFIC_SUMMARY_LARGE = os.path.join(ROOT, "profiles", "k_push_hbm_traffic_large_box_2e8.md")
VALU_SUMMARY = os.path.join(ROOT, "profiles", "k_push_valu_issue_40cube_1e7.md")
VALU_SUMMARY_LARGE = os.path.join(ROOT, "profiles", "k_push_valu_issue_large_box_2e8.md")
TRAFFIC_SUMMARY_PRECISION = os.path.join(ROOT, "profiles", "k_push_hbm_traffic_40cube_5e7.md")
VALU_SUMMARY_PRECISION = os.path.join(ROOT, "profiles", "k_push_valu_issue_40cube_5e7.md")
# counter summaries (HBM traffic, VALU issue) of each workload's particle kernels
PROFILE_SUMMARIES = {"40cube": (TRAFFIC_SUMMARY, VALU_SUMMARY),
                     "precision": (TRAFFIC_SUMMARY_PRECISION, VALU_SUMMARY_PRECISION),
                     "large-box": (TRAFFIC_SUMMARY_LARGE, VALU_SUMMARY_LARGE)}
COPY_CALIB_BYTES = 1 << 30
SPIN_UP_MS = 50.0
CPU_SAMPLE_MAX = 10_000_000
WORKLOADS = {
    "40cube": (2, "40^3x6 jittered Kuhn tet mesh (384,000 tets), 1e7 electrons (Maxwellian 1e6 m/s), "
                  "8-mode envelope on a 10 GHz carrier, B 0.5 T, dt 1e-12 s"),
    "precision": (3, "40^3x6 jittered Kuhn tet mesh (384,000 tets), 5e7 electrons (Maxwellian 1e6 m/s), "
                     "8-mode envelope on a 10 GHz carrier, B 0.5 T, dt 1e-12 s"),
    "large-box": (5, "2:1:1 box, 160x80x80x6 jittered Kuhn tets (6,144,000), 2e8 electrons: half a Gaussian "
                     "bunch (sigma 0.1, drift 1e7 m/s along x), half uniform background (1e6 m/s), 8-mode "
                     "envelope on a 10 GHz carrier, B 1 T along x, dt 1e-12 s"),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_name(form, slices):
    if slices <= 1:
        return KERNEL_NAME[form]
    if slices == 2:   # two pipelined slices per wavefront (float forms)
        return f"k_push_pipe<{'true' if form == 'mixed_fixed' else 'false'}>"
    if form == "mixed_fixed":
        return f"k_push_slices_fixed<{slices}, false>"
    return f"k_push_slices<{REAL[form]}, {slices}, false>"


def logged_steps(E, torch, ctx, parts, sp, fields, w, step0, nlog):
    """nlog single steps, each followed by the continuity residual of that
    step (vertex charge before and after, D^T dG - drho): the largest relative
    residual, and the mean time of a step and of its residual, each timed with
    events on the stream apart from the other."""
    rho_a = torch.zeros(ctx.n_vert, dtype=torch.float64, device="cuda")
    rho_b = torch.zeros_like(rho_a)
    dG = torch.zeros(ctx.n_edge, dtype=torch.float64, device="cuda")
    ctx.vertex_charge(parts, sp, rho_a)
    worst, step_ms, res_ms = 0.0, 0.0, 0.0
    for k in range(nlog):
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        dG.zero_()
        rho_b.zero_()
        ev[0].record()
        ctx.gather_push_deposit(parts, sp, fields, step0 + k, w.dt, w.omega, dG, flags=E.STEP_XCD_REMAP)
        ev[1].record()
        ctx.vertex_charge(parts, sp, rho_b)
        r, p = ctx.gauss_residual(dG, rho_b, rho_a)
        ev[2].record()
        torch.cuda.synchronize()
        worst = max(worst, r / p)
        step_ms += ev[0].elapsed_time(ev[1])
        res_ms += ev[1].elapsed_time(ev[2])
        rho_a, rho_b = rho_b, rho_a
    return {"steps": nlog, "gauss_rel_max": worst, "step_ms": step_ms / max(nlog, 1),
            "charge_and_residual_ms": res_ms / max(nlog, 1),
            "note": "single steps, each followed by the vertex charge and the continuity residual of that step "
                    "(timed apart from the step)"}


def spin_up(torch, ctx, parts, min_ms=SPIN_UP_MS):
    """Untimed streaming over the particle arrays (the stream probe, which
    leaves them as they are) until min_ms of device time have passed: the
    GPU's clocks settle under sustained load, and a handful of warmup steps
    alone leaves the first timed steps ~3 % slower."""
    done = 0.0
    while done < min_ms:
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(10):
            ctx.stream_probe(parts)
        e1.record()
        torch.cuda.synchronize()
        done += e0.elapsed_time(e1)
    return done


def run_form(E, torch, ctx, w, precision, steps, warmup, sort_every, fields, nlog=0, stream_reps=10):
    sp = E.Species(w.q, w.m, w.w)
    parts = E.Particles.from_numpy(w.tet, w.lam, w.vel, w.ids, precision=precision)
    spare = parts.empty_like()
    dG = torch.zeros(ctx.n_edge, dtype=torch.float64, device="cuda")
    # initial sort, clocks settled, then warmup
    ctx.sort(parts, spare)
    parts, spare = spare, parts
    spin_ms = spin_up(torch, ctx, parts)
    step = 0
    for _ in range(warmup):
        ctx.gather_push_deposit(parts, sp, fields, step, w.dt, w.omega, dG)
        step += 1
    torch.cuda.synchronize()
    ctx.kernel_time(reset=True)
    # --- timed region: exactly `steps` steps
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    block = sort_every if sort_every else steps
    k = 0
    while k < steps:
        nb = min(block, steps - k)
        # the steps between two sorts in one call; the re-sort's scatter is
        # folded into the first of them
        if sort_every:
            ctx.sort_run_steps(parts, spare, sp, fields, step, nb, w.dt, w.omega, dG,
                               flags=E.STEP_XCD_REMAP | E.STEP_TIMING)
            parts, spare = spare, parts
        else:
            ctx.run_steps(parts, sp, fields, step, nb, w.dt, w.omega, dG, flags=E.STEP_XCD_REMAP | E.STEP_TIMING)
        step += nb
        k += nb
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = ev0.elapsed_time(ev1)
    kt, launches = ctx.kernel_time(reset=True)
    slices = ctx.last_push_slices()
    ctx.check()
    # per-kernel breakdown, after the timed region: one sort block with every
    # kernel of the step timed (each timed dispatch idles the stream for a few
    # microseconds after it, so the timed region times the particle kernel only)
    nbd = min(block, 10)
    if sort_every:
        ctx.sort_run_steps(parts, spare, sp, fields, step, nbd, w.dt, w.omega, dG,
                           flags=E.STEP_XCD_REMAP | E.STEP_TIMING_ALL)
        parts, spare = spare, parts
    else:
        ctx.run_steps(parts, sp, fields, step, nbd, w.dt, w.omega, dG, flags=E.STEP_XCD_REMAP | E.STEP_TIMING_ALL)
    step += nbd
    kb, nbl = ctx.kernel_time(reset=True)
    # the particle kernel's access pattern alone over the same arrays
    ctx.stream_probe(parts)
    torch.cuda.synchronize()
    s0, s1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s0.record()
    for _ in range(stream_reps):
        ctx.stream_probe(parts)
    s1.record()
    torch.cuda.synchronize()
    stream_ms = s0.elapsed_time(s1) / stream_reps
    # sort alone
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    nsort = 5
    for _ in range(nsort):
        ctx.sort(parts, spare)
        parts, spare = spare, parts
    e1.record()
    torch.cuda.synchronize()
    sort_ms = e0.elapsed_time(e1) / nsort
    # continuity residual (timed separately): rho before / after one more step
    rho0 = torch.zeros(ctx.n_vert, dtype=torch.float64, device="cuda")
    rho1 = torch.zeros_like(rho0)
    dGs = torch.zeros_like(dG)
    ctx.vertex_charge(parts, sp, rho0)
    ctx.gather_push_deposit(parts, sp, fields, step, w.dt, w.omega, dGs)
    torch.cuda.synchronize()
    g0 = torch.cuda.Event(enable_timing=True)
    g1 = torch.cuda.Event(enable_timing=True)
    g0.record()
    ctx.vertex_charge(parts, sp, rho1)
    r, p = ctx.gauss_residual(dGs, rho1, rho0)
    g1.record()
    torch.cuda.synchronize()
    gauss_ms = g0.elapsed_time(g1)
    n = parts.n
    logged = logged_steps(E, torch, ctx, parts, sp, fields, w, step + 1, nlog) if nlog else None
    return {
        "slices": slices,
        "spin_up_ms": round(spin_ms, 1),
        "stream_ms": stream_ms,
        "logged": logged,
        "ms_per_step": total_ms / steps,
        "wall_s": wall,
        "kernel_ms": kt["push"] / max(kt["steps_push"], 1),
        "sort_step_kernel_ms": kt["push_sort"] / max(kt["steps_sort"], 1),
        "coef_ms": kb["coef"] / max(nbl, 1),
        "walk_ms": kb["walk"] / max(nbl, 1),
        "timing_note": "kernel_ms: particle kernel of the in-place steps; sort_step_kernel_ms: the one of the "
                       "first step after each re-sort, which also scatters the particles to their sorted places "
                       "(both from HIP events bound to the kernel's dispatches over the timed region); walk_ms "
                       "and coef_ms per step from a block of %d steps after the timed region with every kernel "
                       "timed: walk_ms covers the walk and, except before a sort, the next step's coefficient "
                       "pass (one launch), and the edge gather of the per-tet sums at the end of the block; "
                       "coef_ms averages the stand-alone passes over the steps" % nbd,
        "launches": launches,
        "sort_ms": sort_ms,
        "gauss_rel": r / p,
        "gauss_ms": gauss_ms,
        "value": n * steps / (total_ms * 1e-3),
    }


def field_update_timing(E, torch, ctx, w, reps=20):
    """Side path, timed separately: the implicit envelope field step on the
    bench mesh (Jacobi-preconditioned COCG with the CSR SpMV).  A random
    interior state is advanced once; SpMV bandwidth from its algorithmic bytes
    (column index 4 B + M and K values 8 B each per nonzero; row pointer 4 B,
    x read and y written 16 B each per row)."""
    eps0, mu0 = 8.8541878128e-12, 1.25663706212e-6
    nnz = ctx.field_setup(w.dt, w.omega, eps0, mu0)
    ne, nf = ctx.n_edge, ctx.n_face
    g = torch.Generator(device="cuda").manual_seed(5)
    x = torch.randn((ne, 2), dtype=torch.float64, device="cuda", generator=g)
    y = torch.empty_like(x)
    ctx.field_spmv(x, y, 1.0 + 0.1j, 1e-3)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ctx.field_spmv(x, y, 1.0 + 0.1j, 1e-3)
    e1.record()
    torch.cuda.synchronize()
    spmv_ms = e0.elapsed_time(e1) / reps
    spmv_bytes = 20 * nnz + 36 * ne
    u = torch.randn((ne, 2), dtype=torch.float64, device="cuda", generator=g)
    v = torch.randn((ne, 2), dtype=torch.float64, device="cuda", generator=g) * 1e9
    a = torch.zeros((ne, 2), dtype=torch.float64, device="cuda")
    b = torch.zeros((nf, 2), dtype=torch.float64, device="cuda")
    # one untimed step, then the timed one (from the state the first left)
    ctx.field_step(w.dt, u, v, a, b, None, tol=1e-10, max_iter=1000, raise_on_error=False)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rc, iters, res = ctx.field_step(2 * w.dt, u, v, a, b, None, tol=1e-10, max_iter=1000, raise_on_error=False)
    torch.cuda.synchronize()
    step_ms = 1e3 * (time.perf_counter() - t0)
    return {"n_edges": ne, "nnz": nnz, "spmv_ms": spmv_ms, "spmv_GBs": spmv_bytes / (spmv_ms * 1e-3) / 1e9,
            "step_ms": step_ms, "cocg_iterations": iters, "rel_residual": res, "status": rc,
            "note": "side path, not in value; the second Newmark step from a random interior state, tol 1e-10"}


def ns_solve_timing(E, torch, ctx, w, reps=3):
    """Side path, timed separately: the non-solenoidal (Gauss-law) solve on the
    bench mesh, its source the charge of the workload's particles (float64
    Jacobi-preconditioned CG on the nodal operator, to a 1e-10 relative
    residual).  Algorithmic bytes per iteration: the product reads the column
    index and value of every stored entry (12 B) and per row the row pointer,
    z, p and q (28 B) and writes p and q (16 B); the update reads p, q, x, r
    and the preconditioner (40 B) and writes x, r and z (24 B)."""
    eps0 = 8.8541878128e-12
    nnz, n_wall = ctx.ns_setup(eps0)
    nv, ne = ctx.n_vert, ctx.n_edge
    parts = E.Particles.from_numpy(w.tet, w.lam, w.vel, w.ids)
    rho0 = torch.zeros(nv, dtype=torch.float64, device="cuda")
    ctx.vertex_charge(parts, E.Species(w.q, w.m, w.w), rho0)
    del parts
    x = torch.zeros((nv, 2), dtype=torch.float64, device="cuda")
    e = torch.zeros((ne, 2), dtype=torch.float64, device="cuda")
    rc, iters, res = ctx.ns_solve(None, rho0, 0.0, w.omega, x, e, tol=1e-10, max_iter=5000, raise_on_error=False)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        t0 = time.perf_counter()
        rc, iters, res = ctx.ns_solve(None, rho0, 0.0, w.omega, x, e, tol=1e-10, max_iter=5000,
                                      raise_on_error=False)
        torch.cuda.synchronize()
        ms.append(1e3 * (time.perf_counter() - t0))
    solve_ms = min(ms)
    # Gauss-law correction of an edge envelope (the field step's mass: set up
    # by the field-update timing with the same eps), two real solves
    gc = torch.Generator(device="cuda").manual_seed(3)
    u = torch.randn((ne, 2), dtype=torch.float64, device="cuda", generator=gc)
    eo = torch.empty_like(u)
    ctx.ns_correct(u, eo, None, rho0, 0.0, w.omega, tol=1e-10, max_iter=5000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, corr_it, _ = ctx.ns_correct(u, eo, None, rho0, 0.0, w.omega, tol=1e-10, max_iter=5000)
    torch.cuda.synchronize()
    corr_ms = 1e3 * (time.perf_counter() - t0)
    bytes_iter = 12 * nnz + 108 * nv
    per_iter = solve_ms / max(iters, 1)
    # the loop closed through the solve: the workload's electrons over a
    # neutralising background (rho0 = 0, G from zero), fields of the workload
    # added, 5 steps each preceded by a warm-started solve
    unsorted = E.Particles.from_numpy(w.tet, w.lam, w.vel, w.ids)
    parts = unsorted.empty_like()
    ctx.sort(unsorted, parts)
    del unsorted
    fields = E.Fields.from_numpy(w.e_env, w.b_env, None, w.b_dc)
    G = torch.zeros(ne, dtype=torch.float64, device="cuda")
    edc = torch.zeros(ne, dtype=torch.float64, device="cuda")
    sp = E.Species(w.q, w.m, w.w)
    ctx.ns_run_steps(parts, sp, 0, 1, w.dt, w.omega, G, edc, ext=fields, tol=1e-10)
    torch.cuda.synchronize()
    # the electromagnetic loop: particle step, field step, Gauss correction
    # (the field state of the field-update timing's setup: dt and omega of the
    # workload), 5 steps from rest
    uu = torch.zeros((ne, 2), dtype=torch.float64, device="cuda")
    vv, aa, ee = torch.zeros_like(uu), torch.zeros_like(uu), torch.zeros_like(uu)
    bb = torch.zeros((ctx.n_face, 2), dtype=torch.float64, device="cuda")
    GG = torch.zeros(ne, dtype=torch.float64, device="cuda")
    HH = torch.zeros(2 * ne, dtype=torch.float64, device="cuda")
    em_parts = parts.clone()
    ctx.em_steps(em_parts, sp, 0, 1, uu, vv, aa, bb, ee, GG, HH, tol=1e-10, max_iter=5000)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    em_it = ctx.em_steps(em_parts, sp, 1, 5, uu, vv, aa, bb, ee, GG, HH, tol=1e-10, max_iter=5000, warm=True)
    torch.cuda.synchronize()
    em_ms = 1e3 * (time.perf_counter() - t0) / 5
    del em_parts
    # the same loop in the form of the split: field step on the solenoidal
    # part (source projected, one real solve) plus the field of eq.
    # ns_equation (one real solve)
    for t_ in (uu, vv, aa, ee, bb, GG, HH):
        t_.zero_()
    em_parts = parts.clone()
    ctx.em_steps(em_parts, sp, 0, 1, uu, vv, aa, bb, ee, GG, HH, tol=1e-10, max_iter=5000, split=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    split_it = ctx.em_steps(em_parts, sp, 1, 5, uu, vv, aa, bb, ee, GG, HH, tol=1e-10, max_iter=5000, warm=True,
                            split=True)
    torch.cuda.synchronize()
    split_ms = 1e3 * (time.perf_counter() - t0) / 5
    del em_parts
    loop = {}
    for per in (1, 10):
        t0 = time.perf_counter()
        it = ctx.ns_run_steps(parts, sp, 1, 20, w.dt, w.omega, G, edc, ext=fields, tol=1e-10, warm=True,
                              steps_per_solve=per)
        torch.cuda.synchronize()
        loop[per] = (1e3 * (time.perf_counter() - t0) / 20, it / (20 // per))
    del parts
    return {"n_nodes": nv, "wall_nodes": n_wall, "nnz": nnz, "solve_ms": solve_ms, "cg_iterations": iters,
            "ms_per_iteration": per_iter, "bytes_per_iteration": bytes_iter,
            "GBs_per_iteration": bytes_iter / (per_iter * 1e-3) / 1e9, "rel_residual": res, "status": rc,
            "correction_ms": corr_ms, "correction_cg_iterations": corr_it,
            "em_loop_ms_per_step": em_ms, "em_loop_iterations_per_step": em_it / 5,
            "split_loop_ms_per_step": split_ms, "split_loop_iterations_per_step": split_it / 5,
            "loop_ms_per_step": loop[1][0], "loop_cg_iterations_per_solve": loop[1][1],
            "loop10_ms_per_step": loop[10][0], "loop10_cg_iterations_per_solve": loop[10][1],
            "note": "side path, not in value; wall time of the whole solve (one host read of the iteration "
                    "scalars per 10 iterations included), best of %d; loop: 20 particle steps of all %d "
                    "electrons (sorted by tet once) with a warm-started solve before every step (loop) or "
                    "every 10th (loop10), mean per step; em_loop: particle step, implicit field step and "
                    "Gauss correction per step, mean of 5; split_loop: the same with the field step on the "
                    "solenoidal part (projected source) plus the Gauss-law field" % (reps, w.tet.shape[0])}


def qh_projector_timing(E, torch, w, reps=3):
    """Side path, timed separately: the quasi-Helmholtz projectors on the bench
    mesh, to a 1e-10 relative residual.  P^Lambda_b of the workload's face
    envelope plus a random part (CG on div div^T over the tets); P^Sigma_e /
    P^Lambda_e of random edge DoFs (CG on Sigma^T Sigma over the nodes, four
    passes per iteration)."""
    eps0 = 8.8541878128e-12
    P = E.QhProjectors(w.xyz, w.tet_vert, eps0)
    g = torch.Generator(device="cuda").manual_seed(11)
    b = torch.from_numpy(np.ascontiguousarray(np.stack([w.b_env.real, w.b_env.imag], axis=1))).cuda()
    b = b + 1e-3 * b.abs().max() * torch.randn(b.shape, dtype=torch.float64, device="cuda", generator=g)
    bo = torch.empty_like(b)
    d = 1e-11 * torch.randn((P.n_edge, 2), dtype=torch.float64, device="cuda", generator=g)
    ds, dl = torch.empty_like(d), torch.empty_like(d)
    out = {}
    for name, call in (("project_b", lambda: P.project_b(b, bo, tol=1e-10, raise_on_error=False)),
                       ("project_e", lambda: P.project_e(d, ds, dl, None, tol=1e-10, raise_on_error=False))):
        call()
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            t0 = time.perf_counter()
            rc, it, res = call()
            torch.cuda.synchronize()
            ms.append(1e3 * (time.perf_counter() - t0))
        out[name] = {"ms": min(ms), "cg_iterations": it, "ms_per_iteration": min(ms) / max(it, 1),
                     "rel_residual": res, "status": rc}
    out["n_tets"], out["n_nodes"] = P.n_tet, P.n_vert
    out["note"] = "side path, not in value; wall time of the whole projection, best of %d" % reps
    P.close()
    return out


def coarse_step_timing(E, torch, synth, ctx, w, fine=10, reps=5):
    """Multi-rate form: one coarse field step of `fine` fine steps with the
    envelope reconstructed from three snapshots (quadratic in time) at every
    fine step; float64, particles sorted, same workload as the metric."""
    snaps = [E.Fields.from_numpy(e, b, None, w.b_dc) for e, b in synth.envelope_snapshots(w, seed=2)]
    sp = E.Species(w.q, w.m, w.w)
    parts = E.Particles.from_numpy(w.tet, w.lam, w.vel, w.ids)
    spare = parts.empty_like()
    ctx.sort(parts, spare)
    parts = spare
    dG = torch.zeros(ctx.n_edge, dtype=torch.float64, device="cuda")
    dtc = fine * w.dt
    ctx.coarse_step(parts, sp, snaps, dtc, dtc, fine, w.omega, dG)
    torch.cuda.synchronize()
    ctx.kernel_time(reset=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for r in range(reps):
        ctx.coarse_step(parts, sp, snaps, (2 + r) * dtc, dtc, fine, w.omega, dG,
                        flags=E.STEP_XCD_REMAP | E.STEP_TIMING)
    e1.record()
    torch.cuda.synchronize()
    kt, launches = ctx.kernel_time(reset=True)
    ctx.coarse_step(parts, sp, snaps, (2 + reps) * dtc, dtc, fine, w.omega, dG,
                    flags=E.STEP_XCD_REMAP | E.STEP_TIMING_ALL)
    kb, nbl = ctx.kernel_time(reset=True)
    ctx.check()
    ms = e0.elapsed_time(e1) / (reps * fine)
    return {"fine_steps_per_coarse": fine, "ms_per_fine_step": ms, "value": parts.n / (ms * 1e-3),
            "coef_ms": kb["coef"] / max(nbl, 1), "walk_coef_ms": kb["walk"] / max(nbl, 1),
            "push_ms": kt["push"] / max(kt["steps_push"], 1),
            "note": "float64, three envelope snapshots interpolated at every fine step; no sort inside"}


# downshifted step without dc edge DoFs, see ds_step_timing
DS_BYTES_PER_PARTICLE = {"fp64": 556, "mixed": 304}
DS_BYTES_PER_TET = {"fp64": 576 + 96, "mixed": 576 + 64}   # complex-envelope rows and the push row


def ds_step_timing(E, torch, ctx, w, form="fp64", nsteps=10, reps=3):
    """Downshifted form (carrier-exact velocity quadrature of envelope samples
    interpolated over three steps, Adams-Bashforth positions), same workload and
    step as the metric, particles sorted once, calls of `nsteps` steps after a
    3-step ramp.  Algorithmic bytes per particle-step of its particle kernel,
    float64: read tet 4, lam 24, v 24, three earlier velocities 72, two E
    samples (Re, Im) 96, two B samples (Re, Im, dc) 144; write lam 24, v 24,
    one velocity 24, one E sample 48, one B sample 72: 556 B.  Mixed (float32
    velocities and samples): 196 read + 108 written = 304 B."""
    sp = E.Species(w.q, w.m, w.w)
    f = E.Fields.from_numpy(w.e_env, w.b_env, None, w.b_dc)
    parts = E.Particles.from_numpy(w.tet, w.lam, w.vel, w.ids, precision=E.FP64 if form == "fp64" else E.MIXED)
    spare = parts.empty_like()
    ctx.sort(parts, spare)
    parts = spare
    hist = ctx.ds_history(parts)
    dG = torch.zeros(ctx.n_edge, dtype=torch.float64, device="cuda")
    ctx.ds_steps(parts, hist, sp, f, 0, 3, 0, w.dt, w.omega, dG)
    torch.cuda.synchronize()
    ctx.kernel_time(reset=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for r in range(reps):
        ctx.ds_steps(parts, hist, sp, f, 3 + r * nsteps, nsteps, 3 + r * nsteps, w.dt, w.omega, dG,
                     flags=E.STEP_XCD_REMAP | E.STEP_TIMING)
    e1.record()
    torch.cuda.synchronize()
    kt, launches = ctx.kernel_time(reset=True)
    s0 = 3 + reps * nsteps
    ctx.ds_steps(parts, hist, sp, f, s0, nsteps, s0, w.dt, w.omega, dG, flags=E.STEP_XCD_REMAP | E.STEP_TIMING_ALL)
    kb, nbl = ctx.kernel_time(reset=True)
    ctx.check()
    ms = e0.elapsed_time(e1) / (reps * nsteps)
    push_ms = kt["push"] / max(kt["steps_push"], 1)
    nbytes = DS_BYTES_PER_PARTICLE[form] * parts.n + DS_BYTES_PER_TET[form] * w.tet_vert.shape[0] + 16 * ctx.n_edge
    ach = nbytes / (push_ms * 1e-3) / 1e9
    del hist
    return {"ms_per_step": ms, "value": parts.n / (ms * 1e-3), "push_ms": push_ms,
            "walk_ms": kb["walk"] / max(nbl, 1), "coef_env_ms": kb["coef"],
            "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(ach / HBM_PEAK_GBS, 4),
                         "kernel": "k_push_ds<double, false>" if form == "fp64" else "k_push_ds<float, false>",
                         "bytes_per_launch": nbytes},
            "note": f"{form} downshifted step (side path, not in value); the complex-envelope rows are built "
                    "once per call"}


def adjoint_timing(E, torch, synth):
    """Differentiation workload: 20^3 x 6 tets, 2e6 electrons, 20 float64 steps
    with a checkpoint every 5, then the reverse sweep (gradient of the final
    kinetic energy with respect to the complex edge envelope)."""
    w = synth.make_workload(4)
    ctx = E.Context(0)
    ctx.upload_mesh(w.xyz, w.tet_vert)
    fields = E.Fields.from_numpy(w.e_env, w.b_env, None, w.b_dc)
    sp = E.Species(w.q, w.m, w.w)
    parts = E.Particles.from_numpy(w.tet, w.lam, w.vel, w.ids)
    spare = parts.empty_like()
    ctx.sort(parts, spare)
    parts = spare
    K, every = 20, 5
    ws = torch.empty(ctx.adjoint_workspace_bytes(parts.n, K, every), dtype=torch.uint8, device="cuda")
    res = {}
    for rep in range(2):   # the first pass warms up
        work = parts.clone()
        torch.cuda.synchronize()
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record()
        ctx.forward_checkpointed(work, sp, fields, 0, K, w.dt, w.omega, every, ws)
        e1.record()
        vbar = (w.m * w.w) * work.vel.clone()
        xbar = torch.zeros_like(vbar)
        grad = torch.zeros((ctx.n_edge, 2), dtype=torch.float64, device="cuda")
        ctx.backward(parts.n, sp, fields, 0, K, w.dt, w.omega, every, ws, vbar, xbar, grad)
        e2.record()
        torch.cuda.synchronize()
        res = {"forward_ms": e0.elapsed_time(e1), "backward_ms": e1.elapsed_time(e2)}
    ctx.check()
    ctx.close()
    res["backward_over_forward"] = res["backward_ms"] / res["forward_ms"]
    res["workload"] = "20^3x6 tets, 2e6 electrons, 20 float64 steps, checkpoint every 5"
    return res


def copy_bandwidth(torch, nbytes=1 << 31, reps=10):
    """Device-to-device copy rate (bytes read + written per second): the
    practical streaming ceiling next to the nominal HBM peak."""
    src = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del src, dst
    return 2 * nbytes / (ms * 1e-3) / 1e9


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, nthreads, steps, stride):
    import oracle
    M = oracle.OracleMesh(w.xyz, w.tet_vert)
    tet, lam, vel = (np.ascontiguousarray(a[::stride]) for a in (w.tet, w.lam, w.vel))
    dG = np.zeros(M.ne)
    t0 = time.perf_counter()
    cpu0 = time.process_time()
    for s in range(steps):
        rc, _ = M.step(tet, lam, vel, q=w.q, m=w.m, w=w.w, step=s, dt=w.dt, omega=w.omega, e_env=w.e_env,
                       b_env=w.b_env, b_dc=w.b_dc, dG=dG, nthreads=nthreads)
    wall = time.perf_counter() - t0
    cpu = time.process_time() - cpu0
    return tet.shape[0] * steps / wall, wall, cpu


def alu_roofline(valu_path, name, kernel_ms):
    """The particle kernel against the vector-ALU issue ceiling: its VALU
    wavefront instructions per launch (counted by rocprofv3 on this source and
    workload, from the committed summary) over its mean duration measured here;
    None without a matching summary."""
    if valu_path is None:
        return None
    from paper_2208_12795_amd import rocprof_summary
    v = rocprof_summary.read_valu(valu_path, name)
    if v is None:
        return None
    insts, busy = v
    ach = insts / (kernel_ms * 1e-3)
    return {"bound": "alu", "achieved": round(ach / 1e9, 1), "peak": round(VALU_PEAK_PER_S / 1e9, 1),
            "unit": "G VALU wavefront instructions/s", "frac": round(ach / VALU_PEAK_PER_S, 4),
            "valu_insts_per_launch": insts, "valu_busy_pct_profiled": busy}


def roofline(res, form, n_p, n_t, n_e, sort_every, copy_gbs, traffic_path=None, valu_path=None):
    """Roofline entry of one form's run: the dominant kernel (the particle
    kernel: its algorithmic bytes per launch over its mean duration from HIP
    events on its launch stream), the attainable rate of its access pattern
    alone (stream probe) and of a device copy, and the whole step's
    algorithmic bytes over the measured time per step; with a VALU summary, the
    same kernel against the vector-ALU issue ceiling (the binding one for the
    compact mixed form)."""
    r = res[form]
    name = kernel_name(form, r["slices"])
    bytes_launch = BYTES_PER_PARTICLE[form] * n_p + BYTES_PER_TET[form] * n_t + BYTES_PER_EDGE * n_e
    ach = bytes_launch / (r["kernel_ms"] * 1e-3) / 1e9
    stream_gbs = BYTES_PER_PARTICLE[form] * n_p / (r["stream_ms"] * 1e-3) / 1e9
    traffic = None
    if traffic_path is not None:
        from paper_2208_12795_amd import rocprof_summary
        traffic = rocprof_summary.read_traffic(traffic_path, name)
    step_bytes = STEP_BYTES_PER_PARTICLE[form] * n_p + STEP_BYTES_PER_TET * n_t
    if sort_every:
        step_bytes += SORT_BYTES_PER_PARTICLE[form] * n_p / sort_every
    step_gbs = step_bytes / (r["ms_per_step"] * 1e-3) / 1e9
    return {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic, "kernel": name,
            "bytes_per_launch": bytes_launch, "kernel_ms": round(r["kernel_ms"], 5),
            "stream_GBs": round(stream_gbs, 1), "frac_of_stream": round(ach / stream_gbs, 4),
            "copy_GBs": round(copy_gbs, 1), "frac_of_copy": round(ach / copy_gbs, 4),
            "alu": alu_roofline(valu_path, name, r["kernel_ms"]),
            "whole_step": {"bytes_per_step": int(step_bytes), "ms_per_step": round(r["ms_per_step"], 5),
                           "achieved": round(step_gbs, 1), "frac": round(step_gbs / HBM_PEAK_GBS, 4),
                           "note": "algorithmic bytes of the whole step (state %d B per particle, %d B per "
                                   "tet, sort amortised) over the measured time per step"
                                   % (STEP_BYTES_PER_PARTICLE[form], STEP_BYTES_PER_TET)}}


def logged_run(E, torch, ctx, w, fields, form, nsteps, sort_every):
    """nsteps single steps of one form, re-sorted every sort_every steps (the
    sort folded into that step), each followed by the vertex charge and the
    continuity residual of that step: the largest relative residual over the
    run, and the mean time of a step and of its residual, each from events on
    the stream apart from the other (the residual's host read synchronises
    every step, so the steps do not overlap)."""
    sp = E.Species(w.q, w.m, w.w)
    parts = E.Particles.from_numpy(w.tet, w.lam, w.vel, w.ids, precision=precision_of(E, form))
    spare = parts.empty_like()
    ctx.sort(parts, spare)
    parts, spare = spare, parts
    dG = torch.zeros(ctx.n_edge, dtype=torch.float64, device="cuda")
    rho_a = torch.zeros(ctx.n_vert, dtype=torch.float64, device="cuda")
    rho_b = torch.zeros_like(rho_a)
    ctx.vertex_charge(parts, sp, rho_a)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    worst, step_ms, res_ms = 0.0, 0.0, 0.0
    t0 = time.perf_counter()
    for k in range(nsteps):
        dG.zero_()
        rho_b.zero_()
        ev[0].record()
        if sort_every and k % sort_every == 0:
            ctx.sort_run_steps(parts, spare, sp, fields, k, 1, w.dt, w.omega, dG, flags=E.STEP_XCD_REMAP)
            parts, spare = spare, parts
        else:
            ctx.gather_push_deposit(parts, sp, fields, k, w.dt, w.omega, dG, flags=E.STEP_XCD_REMAP)
        ev[1].record()
        ctx.vertex_charge(parts, sp, rho_b)
        r, p = ctx.gauss_residual(dG, rho_b, rho_a)
        ev[2].record()
        ev[2].synchronize()
        worst = max(worst, r / p)
        step_ms += ev[0].elapsed_time(ev[1])
        res_ms += ev[1].elapsed_time(ev[2])
        rho_a, rho_b = rho_b, rho_a
    wall = time.perf_counter() - t0
    ctx.check()
    n = parts.n
    del parts, spare
    torch.cuda.empty_cache()
    return {"form": form, "steps": nsteps, "sort_every": sort_every, "gauss_rel_max": worst,
            "step_ms": step_ms / nsteps, "charge_and_residual_ms": res_ms / nsteps, "wall_s": round(wall, 2),
            "value": n / (step_ms / nsteps * 1e-3),
            "note": "every step followed by the vertex charge and the continuity residual of that step; value is "
                    "particle-steps/s over the mean step time without the residual"}


def config_entry(E, torch, synth, key, steps, warmup, sort_every, nlog, copy_gbs,
                 forms=("fp64", "mixed", "mixed_fixed"), logged_steps_run=0, logged_form="mixed"):
    """A second workload measured beside the metric's: both forms, its own
    roofline entries and a logged phase of single steps with the continuity
    residual of every step timed apart; with logged_steps_run, also a run of
    that many single steps of logged_form with the residual after every one."""
    cfg, desc = WORKLOADS[key]
    t0 = time.perf_counter()
    w = synth.make_workload(cfg, progress=lambda m: log(f"[bench] {key}: generated {m}"))
    gen_s = time.perf_counter() - t0
    log(f"[bench] {key}: workload generated in {gen_s:.1f}s: N_p={w.tet.shape[0]} N_t={w.tet_vert.shape[0]}")
    ctx = E.Context(0)
    ctx.upload_mesh(w.xyz, w.tet_vert)
    fields = E.Fields.from_numpy(w.e_env, w.b_env, None, w.b_dc)
    res = {}
    for form in forms:
        res[form] = run_form(E, torch, ctx, w, precision_of(E, form), steps, warmup, sort_every, fields,
                             nlog=nlog)
        log(f"[bench] {key} {form}: {json.dumps(res[form])}")
        torch.cuda.empty_cache()
    n_p, n_t, n_e = w.tet.shape[0], w.tet_vert.shape[0], ctx.n_edge
    out = {"workload": desc + ", sort every %d steps" % sort_every, "n_particles": n_p, "n_tets": n_t,
           "n_edges": n_e, "steps": steps, "warmup": warmup, "generation_s": round(gen_s, 1)}
    for form in forms:
        r = res[form]
        out[form] = {"value": r["value"], "ms_per_step": r["ms_per_step"], "sort_ms": r["sort_ms"],
                     "dtype": FORM_DTYPE[form],
                     "gauss_rel": r["gauss_rel"], "logged": r["logged"],
                     "roofline": roofline(res, form, n_p, n_t, n_e, sort_every, copy_gbs,
                                          *PROFILE_SUMMARIES.get(key, (None, None)))}
    for form in ("mixed", "mixed_fixed"):
        if "fp64" in res and form in res:
            out[form]["speedup_vs_fp64"] = res[form]["value"] / res["fp64"]["value"]
    if logged_steps_run:
        out["logged_run"] = logged_run(E, torch, ctx, w, fields, logged_form, logged_steps_run, sort_every)
        log(f"[bench] {key} logged run: {json.dumps(out['logged_run'])}")
    ctx.close()
    del w
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="40cube",
                    help="40cube: the throughput workload (default); precision: the same mesh with 5e7 "
                         "electrons; large-box: the 2:1:1 bunch workload")
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--particles", type=int, default=None, help="override the particle count (default 1e7)")
    ap.add_argument("--sort-every", type=int, default=10)
    ap.add_argument("--forms", default="fp64,mixed,mixed_fixed")
    ap.add_argument("--log-steps", type=int, default=10,
                    help="single steps with the continuity residual of each, after the timed run")
    ap.add_argument("--precision-steps", type=int, default=20,
                    help="steps of the 5e7-particle side entry (0: skip it)")
    ap.add_argument("--large-box-logged-steps", type=int, default=1000,
                    help="single mixed-form steps of the large box, each followed by the continuity residual "
                         "(0: skip)")
    ap.add_argument("--large-box-steps", type=int, default=100,
                    help="steps of the 2e8-particle large-box side entry (0: skip it)")
    ap.add_argument("--cpu-steps", type=int, default=3)
    ap.add_argument("--cpu-threads", type=int, default=0, help="0 = every core this process may run on")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-side", action="store_true",
                    help="skip the side measurements (field update, adjoint, the other workloads)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run a plain 1 GiB device-to-device copy (reference for HBM byte counters)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}, WORLD_SIZE {world}); "
              "the multi-GPU path is a design, not built", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2208_12795_amd import etpic as E
    from paper_2208_12795_amd import synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.calibrate_copy:
        src = torch.empty(COPY_CALIB_BYTES // 8, dtype=torch.float64, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        c0 = torch.cuda.Event(enable_timing=True)
        c1 = torch.cuda.Event(enable_timing=True)
        c0.record()
        dst.copy_(src)
        c1.record()
        torch.cuda.synchronize()
        copy_gbs = 2 * COPY_CALIB_BYTES / (c0.elapsed_time(c1) * 1e-3) / 1e9
        log(f"[bench] copy calibration: {COPY_CALIB_BYTES} B read + written in {c0.elapsed_time(c1):.3f} ms "
            f"({copy_gbs:.0f} GB/s)")
        del src, dst
    else:
        # (not in a counter run: the calibration copy must stay the run's largest copy)
        copy_gbs = copy_bandwidth(torch)
    log(f"[bench] device copy: {copy_gbs:.0f} GB/s")
    t0 = time.perf_counter()
    cfg, desc = WORKLOADS[args.workload]
    w = synth.make_workload(cfg, n_particles=args.particles)
    log(f"[bench] workload generated in {time.perf_counter() - t0:.1f}s: N_p={w.tet.shape[0]} N_t={w.tet_vert.shape[0]}")
    ctx = E.Context(0)
    ctx.upload_mesh(w.xyz, w.tet_vert)
    fields = E.Fields.from_numpy(w.e_env, w.b_env, None, w.b_dc)
    res = {}
    for form in args.forms.split(","):
        res[form] = run_form(E, torch, ctx, w, precision_of(E, form), args.steps, args.warmup, args.sort_every, fields,
                             nlog=args.log_steps)
        log(f"[bench] {form}: {json.dumps(res[form])}")
    n_p, n_t, n_e = w.tet.shape[0], w.tet_vert.shape[0], ctx.n_edge
    traffic_path, valu_path = (PROFILE_SUMMARIES.get(args.workload, (None, None)) if args.particles is None
                               else (None, None))

    main_form = "fp64" if "fp64" in res else next(iter(res))
    r = res[main_form]
    line = {
        "metric": "particle-steps/s (gather+push+deposit), FP64 vs FP32-mixed, % of HBM peak",
        "value": r["value"],
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_form == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": desc + ", sort every %d steps" % args.sort_every,
                   "n_particles": n_p, "n_tets": n_t, "n_edges": n_e, "parallelism": "single GPU"},
        "roofline": roofline(res, main_form, n_p, n_t, n_e, args.sort_every, copy_gbs, traffic_path, valu_path),
        "sort_ms": r["sort_ms"],
        "gauss_rel": r["gauss_rel"],
        "gauss_ms": r["gauss_ms"],
        "logged": r["logged"],
    }
    for form in ("mixed", "mixed_fixed"):
        if form in res and main_form != form:
            m = res[form]
            line[form] = {"value": m["value"], "ms_per_step": m["ms_per_step"], "dtype": FORM_DTYPE[form],
                          "speedup_vs_fp64": m["value"] / r["value"],
                          "roofline": roofline(res, form, n_p, n_t, n_e, args.sort_every, copy_gbs, traffic_path,
                                               valu_path),
                          "gauss_rel": m["gauss_rel"], "logged": m["logged"]}
    if not args.no_side and args.workload == "40cube":
        line["field_update"] = field_update_timing(E, torch, ctx, w)
        log(f"[bench] field update: {json.dumps(line['field_update'])}")
        line["ns_solve"] = ns_solve_timing(E, torch, ctx, w)
        log(f"[bench] non-solenoidal solve: {json.dumps(line['ns_solve'])}")
        line["qh_projectors"] = qh_projector_timing(E, torch, w)
        log(f"[bench] quasi-Helmholtz projectors: {json.dumps(line['qh_projectors'])}")
        line["coarse_step"] = coarse_step_timing(E, torch, synth, ctx, w)
        log(f"[bench] coarse step: {json.dumps(line['coarse_step'])}")
        line["downshifted_step"] = ds_step_timing(E, torch, ctx, w)
        line["downshifted_step"]["mixed"] = ds_step_timing(E, torch, ctx, w, form="mixed")
        log(f"[bench] downshifted step: {json.dumps(line['downshifted_step'])}")
        line["adjoint"] = adjoint_timing(E, torch, synth)
        log(f"[bench] adjoint: {json.dumps(line['adjoint'])}")
    if not args.no_cpu_baseline:
        nth = args.cpu_threads or len(os.sched_getaffinity(0))
        stride = max(1, n_p // CPU_SAMPLE_MAX)
        val, wall, cpu = cpu_baseline(w, nth, args.cpu_steps, stride)
        which = f"all {n_p} particles" if stride == 1 else f"every {stride}th of the {n_p} particles"
        one_stride = max(stride, n_p // 1_000_000)
        one, wall1, _ = cpu_baseline(w, 1, 1, one_stride)
        line["cpu_baseline"] = {"value": val, "unit": "particle-steps/s", "cores": nth, "kind": "oracle",
                                "sample": f"{which}, first {args.cpu_steps} steps (float64 oracle, "
                                          f"OpenMP over particles, {nth} threads); wall {wall:.1f}s, "
                                          f"cpu {cpu:.1f}s",
                                "nproc": os.cpu_count(), "affinity_cores": len(os.sched_getaffinity(0)),
                                "cpu_model": cpu_model(),
                                "single_thread_value": one,
                                "single_thread_sample": f"every {one_stride}th particle, first step, 1 thread; "
                                                        f"wall {wall1:.1f}s"}
    ctx.close()
    del w
    if not args.no_side and args.workload == "40cube":
        if args.precision_steps:
            line["precision"] = config_entry(E, torch, synth, "precision", args.precision_steps, 2,
                                             args.sort_every, args.log_steps, copy_gbs)
            log(f"[bench] precision: {json.dumps(line['precision'])}")
        if args.large_box_steps:
            line["large_box"] = config_entry(E, torch, synth, "large-box", args.large_box_steps, 2,
                                             args.sort_every, args.log_steps, copy_gbs,
                                             forms=("mixed_fixed", "mixed", "fp64"),
                                             logged_steps_run=args.large_box_logged_steps)
            log(f"[bench] large box: {json.dumps(line['large_box'])}")
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
