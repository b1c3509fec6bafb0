"""Seeded synthetic workloads for the envelope-tracking particle step.

This module only *makes inputs*: a jittered Kuhn tetrahedral mesh, electron
macroparticles given as (tet, barycentric) pairs with Maxwellian velocities,
and envelope field degrees of freedom.  It holds none of the particle step's
arithmetic (no field gather, push, walk or deposit) and is shared, as a pure
input source, by the CPU oracle (tests only) and by the GPU path.

Conventions fixed here and relied on by both consumers:

* tet rows list their four vertex ids in ascending order; the particle's
  barycentrics (lam1, lam2, lam3) refer to local vertices 1..3 of that order,
  lam0 = 1 - lam1 - lam2 - lam3;
* edges are vertex pairs (a < b) numbered lexicographically, oriented a -> b;
* faces are vertex triples (a < b < c) numbered lexicographically, oriented by
  the normal (r_b - r_a) x (r_c - r_a);
* the complex envelope DoF of an edge is the line integral of the complex
  envelope field along it (the Whitney 1-form DoF); the face DoF is the flux
  through the oriented face (the Whitney 2-form DoF).  Field expansion in these
  bases: Formulation, discretization in space and time.
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np

Q_E = -1.602176634e-19       # electron charge [C]
M_E = 9.1093837015e-31       # electron mass [kg]
SEED_BASE = 220812795

PERMS = list(itertools.permutations(range(3)))   # Kuhn tet k <-> axis order PERMS[k]


# --------------------------------------------------------------------------- mesh
def kuhn_mesh(n, extent=(1.0, 1.0, 1.0), jitter=0.1, rng=None):
    """Box [0,Lx]x[0,Ly]x[0,Lz] cut into nx*ny*nz cells, each split into the six
    Kuhn tets (one per axis permutation: the monotone vertex path 000 -> 111).

    Interior vertices are displaced by U(-jitter*h, +jitter*h) per axis; boundary
    vertices stay on the box so the domain is exactly the box.
    Returns (xyz float64[N_n,3], tet_vert int32[N_t,4] ascending)."""
    nx, ny, nz = (int(v) for v in n)
    lx, ly, lz = (float(v) for v in extent)
    hx, hy, hz = lx / nx, ly / ny, lz / nz
    i = np.arange(nx + 1, dtype=np.float64)
    j = np.arange(ny + 1, dtype=np.float64)
    k = np.arange(nz + 1, dtype=np.float64)
    K, J, I = np.meshgrid(k, j, i, indexing="ij")     # vertex id = i + (nx+1)(j + (ny+1)k)
    xyz = np.stack([I.ravel() * hx, J.ravel() * hy, K.ravel() * hz], axis=1)
    if jitter and rng is not None:
        ii, jj, kk = I.ravel(), J.ravel(), K.ravel()
        interior = (ii > 0) & (ii < nx) & (jj > 0) & (jj < ny) & (kk > 0) & (kk < nz)
        d = rng.uniform(-jitter, jitter, size=(xyz.shape[0], 3)) * np.array([hx, hy, hz])
        xyz[interior] += d[interior]
    sx, sy, sz = 1, nx + 1, (nx + 1) * (ny + 1)
    step = np.array([sx, sy, sz], dtype=np.int64)
    ci, cj, ck = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    # cell order: ci fastest  -> cell = ci + nx*(cj + ny*ck)
    ci = ci.transpose(2, 1, 0).ravel()
    cj = cj.transpose(2, 1, 0).ravel()
    ck = ck.transpose(2, 1, 0).ravel()
    base = ci * sx + cj * sy + ck * sz
    tets = np.empty((base.size, 6, 4), dtype=np.int64)
    for p, perm in enumerate(PERMS):
        v0 = base
        v1 = v0 + step[perm[0]]
        v2 = v1 + step[perm[1]]
        v3 = v2 + step[perm[2]]
        tets[:, p, :] = np.stack([v0, v1, v2, v3], axis=1)   # strictly increasing
    return xyz, tets.reshape(-1, 4).astype(np.int32)


def mesh_edges(tet_vert, n_vert):
    """Canonical edge list: unique (a<b) pairs in lexicographic order."""
    tv = tet_vert.astype(np.int64)
    pairs = tv[:, [[0, 1], [0, 2], [0, 3], [1, 2], [1, 3], [2, 3]]].reshape(-1, 2)
    keys = np.unique(pairs[:, 0] * n_vert + pairs[:, 1])
    return np.stack([keys // n_vert, keys % n_vert], axis=1).astype(np.int32)


def mesh_faces(tet_vert, n_vert):
    """Canonical face list: unique (a<b<c) triples in lexicographic order."""
    tv = tet_vert.astype(np.int64)
    tri = tv[:, [[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]]].reshape(-1, 3)
    keys = np.unique((tri[:, 0] * n_vert + tri[:, 1]) * n_vert + tri[:, 2])
    c = keys % n_vert
    ab = keys // n_vert
    return np.stack([ab // n_vert, ab % n_vert, c], axis=1).astype(np.int32)


def _cross_cols(a, b):
    """row-wise cross product of [N,3] arrays, column by column (large N)"""
    return np.stack([a[:, 1] * b[:, 2] - a[:, 2] * b[:, 1],
                     a[:, 2] * b[:, 0] - a[:, 0] * b[:, 2],
                     a[:, 0] * b[:, 1] - a[:, 1] * b[:, 0]], axis=1)


def tet_volumes(xyz, tet_vert):
    """Signed volumes (geometry of the generated mesh; used for sampling)."""
    r0 = xyz[tet_vert[:, 0]]
    a, b, c = xyz[tet_vert[:, 1]] - r0, xyz[tet_vert[:, 2]] - r0, xyz[tet_vert[:, 3]] - r0
    return (a * _cross_cols(b, c)).sum(axis=1) / 6.0


# --------------------------------------------------------------------- particles
def uniform_particles(xyz, tet_vert, n, rng):
    """Positions uniform in the domain: tet chosen with probability |vol| (by
    rejection against the largest volume), barycentrics ~ Dirichlet(1,1,1,1)
    (uniform inside a tet)."""
    vol = np.abs(tet_volumes(xyz, tet_vert))
    acc = vol / vol.max()
    nt = tet_vert.shape[0]
    tet = np.empty(0, dtype=np.int64)
    while tet.size < n:
        m = int((n - tet.size) / acc.mean() * 1.05) + 64
        cand = rng.integers(0, nt, m)
        tet = np.concatenate([tet, cand[rng.random(m) < acc[cand]]])
    tet = tet[:n].astype(np.int32)
    g = rng.standard_exponential((n, 4))
    g /= g.sum(axis=1, keepdims=True)
    return tet, np.ascontiguousarray(g[:, 1:])


def reference_located(u, n, extent):
    """(tet, lam1..3) of points u[N,3] given in the *unjittered* box coordinates.

    In the unjittered Kuhn grid the containing tet is read off the cell index and
    the descending order of the fractional coordinates.  The same (tet, lam) in
    the jittered mesh is the image of u under the piecewise-linear jitter map."""
    nx, ny, nz = (int(v) for v in n)
    h = np.asarray(extent, dtype=np.float64) / np.array([nx, ny, nz])
    s = u / h
    cell = np.floor(s).astype(np.int64)
    cell = np.clip(cell, 0, np.array([nx - 1, ny - 1, nz - 1]))
    f = np.clip(s - cell, 0.0, 1.0)
    # descending order of the three fractional coordinates (ties: lower axis first)
    f0, f1, f2 = f[:, 0], f[:, 1], f[:, 2]
    ge01, ge02, ge12 = f0 >= f1, f0 >= f2, f1 >= f2
    first = np.where(ge01 & ge02, 0, np.where(~ge01 & ge12, 1, 2))     # largest, lowest axis on ties
    last = np.where(ge02 & ge12, 2, np.where(ge01, 1, 0))               # smallest, highest axis on ties
    mid = 3 - first - last
    order = np.stack([first, mid, last], axis=1)
    lut = np.full(27, -1, dtype=np.int64)
    for i, p in enumerate(PERMS):
        lut[p[0] * 9 + p[1] * 3 + p[2]] = i
    pidx = lut[order[:, 0] * 9 + order[:, 1] * 3 + order[:, 2]]
    fs = np.take_along_axis(f, order, axis=1)
    lam = np.stack([1.0 - fs[:, 0], fs[:, 0] - fs[:, 1], fs[:, 1] - fs[:, 2], fs[:, 2]], axis=1)
    cid = cell[:, 0] + nx * (cell[:, 1] + ny * cell[:, 2])
    tet = (cid * 6 + pidx).astype(np.int32)
    return tet, np.ascontiguousarray(lam[:, 1:])


def maxwellian(n, vth, rng, drift=(0.0, 0.0, 0.0)):
    """Each component ~ N(drift_c, vth_c^2)."""
    vth = np.broadcast_to(np.asarray(vth, dtype=np.float64), (3,))
    return rng.standard_normal((n, 3)) * vth + np.asarray(drift, dtype=np.float64)


# ------------------------------------------------------------------------ fields
def phasor_edge_dofs(xyz, edges, amp, rng):
    """e_e = amp * |edge| * exp(j*phi_e), phi_e ~ U[0, 2pi)  (line-integral units: V)."""
    d = xyz[edges[:, 1]] - xyz[edges[:, 0]]
    length = np.sqrt((d * d).sum(axis=1))
    phi = rng.uniform(0.0, 2.0 * np.pi, size=edges.shape[0])
    return amp * length * np.exp(1j * phi)


def _phi1(z):
    small = np.abs(z) < 1e-3
    out = np.empty_like(z)
    zs = z[small]
    out[small] = 1.0 + zs / 2.0 + zs * zs / 6.0 + zs * zs * zs / 24.0
    zl = z[~small]
    out[~small] = np.expm1(zl) / zl if np.isrealobj(zl) else (np.exp(zl) - 1.0) / zl
    return out


def mode_edge_dofs(xyz, edges, amp, extent, rng, n_modes=8):
    """Smooth random envelope E(r) = sum_m a_m exp(j k_m.r), a_m complex normal
    3-vectors, k_m = 2pi (nx/Lx, ny/Ly, nz/Lz) with n in {-2..2}^3 minus 0,
    scaled so that max over vertices |E| = amp.  DoF = exact line integral."""
    L = np.asarray(extent, dtype=np.float64)
    cand = np.array([c for c in itertools.product(range(-2, 3), repeat=3) if any(c)], dtype=np.float64)
    pick = rng.choice(cand.shape[0], size=n_modes, replace=False)
    kvec = 2.0 * np.pi * cand[pick] / L
    a = (rng.standard_normal((n_modes, 3)) + 1j * rng.standard_normal((n_modes, 3))) / np.sqrt(2.0)
    ev = np.zeros((xyz.shape[0], 3), dtype=np.complex128)
    for m in range(n_modes):
        ev += a[m] * np.exp(1j * (xyz @ kvec[m]))[:, None]
    scale = amp / np.sqrt((np.abs(ev) ** 2).sum(axis=1)).max()
    ra = xyz[edges[:, 0]]
    d = xyz[edges[:, 1]] - ra
    dof = np.zeros(edges.shape[0], dtype=np.complex128)
    for m in range(n_modes):
        z = 1j * (d @ kvec[m])
        dof += (d @ a[m]) * np.exp(1j * (ra @ kvec[m])) * _phi1(z)
    return scale * dof


def uniform_face_flux(xyz, faces, b0):
    """Flux of a uniform B0 through each oriented face: B0 . (r_b-r_a)x(r_c-r_a)/2."""
    ra = xyz[faces[:, 0]]
    area = 0.5 * _cross_cols(xyz[faces[:, 1]] - ra, xyz[faces[:, 2]] - ra)
    return area @ np.asarray(b0, dtype=np.float64)


def edge_ids(edges, n_vert, a, b):
    keys = edges[:, 0].astype(np.int64) * n_vert + edges[:, 1]
    q = a.astype(np.int64) * n_vert + b
    idx = np.searchsorted(keys, q)
    assert np.all(keys[idx] == q)
    return idx


def faraday_face_envelope(e_env, edges, faces, n_vert, omega):
    """Face envelope consistent with a constant edge envelope under the envelope
    Faraday law (curl E~ = -(j w + d/dt) B~):  b~ = j * circ(e~) / w, where the
    circulation around face (a,b,c) is e_ab + e_bc - e_ac.  Zero at w = 0."""
    if omega == 0.0:
        return np.zeros(faces.shape[0], dtype=np.complex128)
    a, b, c = faces[:, 0], faces[:, 1], faces[:, 2]
    circ = (e_env[edge_ids(edges, n_vert, a, b)] + e_env[edge_ids(edges, n_vert, b, c)]
            - e_env[edge_ids(edges, n_vert, a, c)])
    return 1j * circ / omega


# ------------------------------------------------------------------------ configs
@dataclass
class Workload:
    name: str
    n: tuple
    extent: tuple
    xyz: np.ndarray
    tet_vert: np.ndarray
    edges: np.ndarray
    faces: np.ndarray
    tet: np.ndarray          # int32 [N_p]
    lam: np.ndarray          # float64 [N_p, 3]  (lam1, lam2, lam3)
    vel: np.ndarray          # float64 [N_p, 3]  v^{n-1/2}
    ids: np.ndarray          # int64 [N_p]
    e_env: np.ndarray        # complex128 [N_e]
    b_env: np.ndarray        # complex128 [N_f]
    b_dc: np.ndarray         # float64 [N_f]
    omega: float
    dt: float
    steps: int
    sort_every: int
    q: float = Q_E
    m: float = M_E
    w: float = 1.0
    extra: dict = field(default_factory=dict)

    @property
    def n_vert(self):
        return self.xyz.shape[0]


WORKLOAD_TABLE = {
    # unit cube 5^3 x 6, 1e3 e-, vth 1e5, B 0.1 T z, random unit phasors 1e3 V/m, 1 GHz, dt 1e-11, 100 steps
    1: dict(name="cube5x6-1e3", n=(5, 5, 5), extent=(1.0, 1.0, 1.0), n_p=1000, vth=1e5, b0=(0.0, 0.0, 0.1),
            fields="phasor", amp=1e3, freq=1e9, dt=1e-11, steps=100, sort_every=0),
    # 40^3 x 6, 1e7 e-, vth 1e6, 8-mode envelope, 10 GHz, B 0.5 T z, dt 1e-12, 200 steps, sort every 10
    2: dict(name="cube40x6-1e7", n=(40, 40, 40), extent=(1.0, 1.0, 1.0), n_p=10_000_000, vth=1e6, b0=(0.0, 0.0, 0.5),
            fields="modes", amp=1e3, freq=1e10, dt=1e-12, steps=200, sort_every=10),
    # same mesh, 5e7 particles (mixed-precision form)
    3: dict(name="cube40x6-5e7", n=(40, 40, 40), extent=(1.0, 1.0, 1.0), n_p=50_000_000, vth=1e6, b0=(0.0, 0.0, 0.5),
            fields="modes", amp=1e3, freq=1e10, dt=1e-12, steps=200, sort_every=10),
    # 20^3 x 6, 2e6 e-, physics of the 40^3 case, 20 steps (differentiation form)
    4: dict(name="cube20x6-2e6", n=(20, 20, 20), extent=(1.0, 1.0, 1.0), n_p=2_000_000, vth=1e6, b0=(0.0, 0.0, 0.5),
            fields="modes", amp=1e3, freq=1e10, dt=1e-12, steps=20, sort_every=0),
    # 2:1:1 box, 160x80x80 x 6, bunch + background, B 1 T x, 10 GHz, 1000 steps
    5: dict(name="box160x80x80x6-2e8", n=(160, 80, 80), extent=(2.0, 1.0, 1.0), n_p=200_000_000, vth=1e6, b0=(1.0, 0.0, 0.0),
            fields="modes", amp=1e3, freq=1e10, dt=1e-12, steps=1000, sort_every=10, bunch=True),
}


def rngs(k):
    ss = np.random.SeedSequence(SEED_BASE + k).spawn(4)
    return [np.random.Generator(np.random.PCG64(s)) for s in ss]   # mesh, pos, vel, fields


def make_workload(k, n_particles=None, n_cells=None, omega=None, b0=None, amp=None, progress=None):
    """Workload k with optional overrides (smaller particle count / mesh):
    1 = 5^3 x 6 tets, unit cube, 1e3 electrons; 2 = 40^3 x 6, 1e7; 3 = 40^3 x 6,
    5e7; 4 = 20^3 x 6, 2e6; 5 = 160 x 80 x 80 x 6, 2:1:1 box, 2e8 (bunch and
    background).  progress(msg), if given, is called after each phase."""
    import time as _time
    t_start = _time.perf_counter()

    def done(what):
        if progress is not None:
            progress(f"{what} ({_time.perf_counter() - t_start:.1f}s)")
    c = dict(WORKLOAD_TABLE[k])
    if n_cells is not None:
        c["n"] = tuple(n_cells)
    n_p = int(c["n_p"] if n_particles is None else n_particles)
    r_mesh, r_pos, r_vel, r_fld = rngs(k)
    xyz, tv = kuhn_mesh(c["n"], c["extent"], 0.1, r_mesh)
    nv = xyz.shape[0]
    edges = mesh_edges(tv, nv)
    faces = mesh_faces(tv, nv)
    done("mesh")
    if c.get("bunch"):
        nb = n_p // 2
        ctr = 0.5 * np.asarray(c["extent"])
        u = np.empty((0, 3))
        while u.shape[0] < nb:
            cand = ctr + 0.1 * r_pos.standard_normal((nb - u.shape[0], 3))
            ok = np.all((cand > 0) & (cand < np.asarray(c["extent"])), axis=1)
            u = np.concatenate([u, cand[ok]])
        tb, lb = reference_located(u, c["n"], c["extent"])
        done("bunch positions")
        tu, lu = uniform_particles(xyz, tv, n_p - nb, r_pos)
        done("background positions")
        vb = maxwellian(nb, (5e4, 1e5, 1e5), r_vel, drift=(1e7, 0.0, 0.0))
        vu = maxwellian(n_p - nb, c["vth"], r_vel)
        tet = np.concatenate([tb, tu]); lam = np.concatenate([lb, lu]); vel = np.concatenate([vb, vu])
    else:
        tet, lam = uniform_particles(xyz, tv, n_p, r_pos)
        vel = maxwellian(n_p, c["vth"], r_vel)
    done("particles")
    w = 2.0 * np.pi * c["freq"] if omega is None else float(omega)
    a = c["amp"] if amp is None else amp
    if c["fields"] == "phasor":
        e_env = phasor_edge_dofs(xyz, edges, a, r_fld)
    else:
        e_env = mode_edge_dofs(xyz, edges, a, c["extent"], r_fld)
    b_env = faraday_face_envelope(e_env, edges, faces, nv, w)
    b_dc = uniform_face_flux(xyz, faces, c["b0"] if b0 is None else b0)
    done("fields")
    return Workload(name=c["name"], n=c["n"], extent=c["extent"], xyz=xyz, tet_vert=tv,
                    edges=edges, faces=faces, tet=tet.astype(np.int32),
                    lam=np.ascontiguousarray(lam, dtype=np.float64),
                    vel=np.ascontiguousarray(vel, dtype=np.float64),
                    ids=np.arange(n_p, dtype=np.int64), e_env=e_env, b_env=b_env, b_dc=b_dc,
                    omega=w, dt=c["dt"], steps=c["steps"], sort_every=c["sort_every"])


def envelope_snapshots(w, seed=1, count=3, drift=0.3):
    """`count` envelope snapshots (edge, face) for coarse field times: the
    workload's edge envelope plus `drift` times independent 8-mode envelopes of
    the same amplitude (seeded), each with its Faraday-consistent face envelope."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_BASE, 77, seed]))
    amp = np.abs(w.e_env).max()
    edges, faces = w.edges, w.faces
    out = []
    for _ in range(count):
        extra = mode_edge_dofs(w.xyz, edges, 1.0, w.extent, rng)
        e = w.e_env + drift * amp * extra / np.abs(extra).max()
        out.append((e, faraday_face_envelope(e, edges, faces, w.n_vert, w.omega)))
    return out


def as_interleaved(z):
    """complex128[N] -> float64[N,2] (re, im) contiguous, the device layout."""
    return np.ascontiguousarray(np.stack([z.real, z.imag], axis=1))


# --------------------------------------------------------------- cold plasma
EPS0 = 8.8541878128e-12
E_CHARGE = -1.602176634e-19
E_MASS = 9.1093837015e-31


@dataclass
class ColdPlasma:
    """Electrons at rest in the unjittered box [0, L]^3, displaced from
    uniform random places u0 by xi = a grad psi, psi = sin(kx) sin(ky)
    sin(kz), k = pi / L, with a neutralising background (the charge of the
    undisplaced electrons, with the opposite sign).  The macroparticle weight
    sets the electron density n so that the plasma frequency is omega_p."""
    n: tuple
    extent: tuple
    xyz: np.ndarray
    tet_vert: np.ndarray
    tet0: np.ndarray        # undisplaced places
    lam0: np.ndarray
    tet: np.ndarray         # displaced places
    lam: np.ndarray
    vel: np.ndarray
    ids: np.ndarray
    q: float
    m: float
    w: float
    density: float          # electrons per m^3
    a: float                # displacement scale [m^2]
    omega_p: float


def cold_plasma(n_cells, n_particles, amp=1e-3, omega_p=2 * np.pi * 1e9, L=0.1, seed=1):
    """Cold-plasma oscillation input; amp * L / pi is the largest displacement
    component over grad psi / k (a = amp * L^2 / pi^2)."""
    rng = np.random.default_rng(np.random.SeedSequence([SEED_BASE, 91, seed]))
    n = (int(n_cells),) * 3
    ext = (L, L, L)
    xyz, tv = kuhn_mesh(n, ext, 0.0)
    u0 = rng.random((int(n_particles), 3)) * L
    k = np.pi / L
    a = amp * L * L / np.pi ** 2
    s, c = np.sin(k * u0), np.cos(k * u0)
    grad = k * np.stack([c[:, 0] * s[:, 1] * s[:, 2], s[:, 0] * c[:, 1] * s[:, 2], s[:, 0] * s[:, 1] * c[:, 2]], axis=1)
    u = u0 + a * grad
    t0, l0 = reference_located(u0, n, ext)
    t1, l1 = reference_located(u, n, ext)
    dens = omega_p ** 2 * EPS0 * E_MASS / E_CHARGE ** 2
    w = dens * L ** 3 / int(n_particles)
    return ColdPlasma(n=n, extent=ext, xyz=xyz, tet_vert=tv, tet0=t0, lam0=l0, tet=t1, lam=l1,
                      vel=np.zeros((int(n_particles), 3)), ids=np.arange(int(n_particles), dtype=np.int64),
                      q=E_CHARGE, m=E_MASS, w=w, density=dens, a=a, omega_p=omega_p)
