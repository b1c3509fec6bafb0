"""Comparison helpers of the parity tests (GPU path vs FP64 oracle).

Tolerance reading.  Velocities and edge currents are fresh results of a step
and are compared relative to their own scale.  Positions are stored as float64
barycentrics, and a step moves them by ~1e-5 of their magnitude, so the stored
end point of *any* float64 implementation carries a quantum of one unit in the
last place of lambda.  The position error is therefore measured beyond that
quantum (2 ulp of lambda per coordinate), relative to the largest barycentric
increment of the step.  A particle that crossed a face has, in addition, been
re-expressed in its new tet's barycentric frame at the crossing point; each
coordinate of that point is rounded there (an absolute quantum of a few units
of float64 epsilon, whatever the implementation: the kernel sets the exit
coordinate to zero and rescales, the oracle solves for the point's
barycentrics by Cramer's rule), so for crossed particles the quantum also
holds 4 epsilon absolute per coordinate.  Barycentrics stored in fixed point
(the compact mixed form, a grid of 2^-32) carry that grid's quantum instead:
lam_quantum = 2^-31 absolute (rounding to the grid, and the largest coordinate
giving up the excess when the three sum past one).
"""
import numpy as np

ULP1 = np.finfo(np.float64).eps  # ulp of numbers in [1, 2)


def positions(xyz, tv, tet, lam):
    l0 = 1.0 - lam.sum(axis=1)
    r = xyz[tv[tet]]
    return l0[:, None] * r[:, 0] + lam[:, 0:1] * r[:, 1] + lam[:, 1:2] * r[:, 2] + lam[:, 2:3] * r[:, 3]


def step_errors(xyz, tv, state_in, gpu, ora, dG_gpu, dG_ora, lam_quantum=0.0):
    """state_in/gpu/ora = (tet, lam[N,3], vel[N,3]); returns a dict of errors.
    lam_quantum: absolute quantum of the GPU's stored barycentrics beyond
    float64 (2^-31 for fixed-point storage)."""
    t0, l0, v0 = state_in
    tg, lg, vg = gpu
    to, lo, vo = ora
    out = {}
    out["v_rel"] = float(np.abs(vg - vo).max() / max(np.abs(vo).max(), 1e-300)) if len(vo) else 0.0
    same = tg == to
    out["tet_mismatch"] = int((~same).sum())
    dl = np.abs(lo - l0)[same & (to == t0)]
    scale = dl.max() if dl.size else 0.0
    if same.any():
        quantum = 2.0 * ULP1 * np.maximum(np.abs(lg[same]), np.abs(lo[same]))
        crossed = ((tg != t0) | (to != t0))[same]
        quantum[crossed] += 4.0 * ULP1
        quantum += lam_quantum
        excess = np.maximum(np.abs(lg[same] - lo[same]) - quantum, 0.0)
        out["lam_rel"] = float(excess.max() / scale) if scale > 0 else float(excess.max())
    else:
        out["lam_rel"] = 0.0
    if (~same).any():
        xg = positions(xyz, tv, tg[~same], lg[~same])
        xo = positions(xyz, tv, to[~same], lo[~same])
        dx = np.abs(positions(xyz, tv, to, lo) - positions(xyz, tv, t0, l0)).max()
        h = np.abs(xyz[tv[:, 1]] - xyz[tv[:, 0]]).max()
        out["x_mismatch_rel"] = float((np.abs(xg - xo).max() - 8 * ULP1 * np.abs(xyz).max() - 4 * lam_quantum * h) / dx)
    else:
        out["x_mismatch_rel"] = 0.0
    nrm2 = np.linalg.norm(dG_ora)
    out["dG_rel2"] = float(np.linalg.norm(dG_gpu - dG_ora) / nrm2) if nrm2 > 0 else float(np.abs(dG_gpu).max())
    mx = np.abs(dG_ora).max() if dG_ora.size else 0.0
    out["dG_relinf"] = float(np.abs(dG_gpu - dG_ora).max() / mx) if mx > 0 else float(np.abs(dG_gpu).max())
    return out


def assert_within(err, tol, what=""):
    bad = {k: v for k, v in err.items() if k in ("v_rel", "lam_rel", "x_mismatch_rel", "dG_rel2", "dG_relinf")
           and v > tol}
    assert not bad, f"{what}: {bad} > {tol} (all: {err})"
