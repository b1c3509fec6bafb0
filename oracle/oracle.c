/*
 * FP64 CPU oracle for the envelope-tracking particle-mesh step
 * (Ramachandran et al., "An Envelope Tracking Approach for Particle in Cell
 * Simulations").  TEST INFRASTRUCTURE ONLY: it is linked by the test-suite, by
 * the smoke check and by the CPU-baseline leg of the benchmark, never by the
 * product path.  It shares no code with the GPU library.
 *
 * Plain, slow, scalar C, one particle at a time, in the order the method takes
 * its steps:
 *   1. fields at the particle: Whitney edge (E) and face (B) expansions
 *      (Formulation, "Discretization in Space and Time", the E~/B~ expansion),
 *      with the envelope modulated by the carrier and the real part taken
 *      (Particle Push section: dv/dt = q/m Re{E~ e^{j w t}} + v x Re{B~ e^{j w t}});
 *   2. a Lorentz update at the fine step (the "simpler" scheme of the Particle
 *      Push section) -- the textbook Boris rotation, non-relativistic;
 *   3. the straight-line path of the step walked through the mesh;
 *   4. the path integral of the Whitney 1-forms along each piece, i.e. the
 *      edge DoFs g_l = <W1_l, G> of G = q * sum_p int dr (eq. g_def and the
 *      piecewise sum of eq. G_integral).
 * The section's other scheme -- the velocity update that integrates the carrier
 * exactly against interpolated envelope samples, with Adams-Bashforth positions
 * (eq. newtons) -- is the downshifted step at the end of the file.
 * Each function cites the passage it follows.
 *
 * Conventions (shared definitions, own implementation): tet rows are ascending
 * vertex ids; local edge order (0,1),(0,2),(0,3),(1,2),(1,3),(2,3); local face k
 * is opposite local vertex k; global edges (a<b) and faces (a<b<c) are numbered
 * lexicographically; face orientation (r_b-r_a)x(r_c-r_a).
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORA_HOP_CAP 64

typedef struct ora_mesh {
    int64_t nv, nt, ne, nf;
    double *xyz;       /* nv*3 */
    int32_t *tv;       /* nt*4, ascending */
    int32_t *edges;    /* ne*2 */
    int32_t *faces;    /* nf*3 */
    int32_t *tet_edge; /* nt*6 */
    int32_t *tet_face; /* nt*4, face opposite local vertex k */
    int32_t *nbr;      /* nt*4, tet across face k or -1 */
} ora_mesh;

static const int LE[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
static const int LF[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};

static int cmp_i64(const void *a, const void *b) {
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

static int64_t find_key(const int64_t *keys, int64_t n, int64_t k) {
    int64_t lo = 0, hi = n - 1;
    while (lo <= hi) {
        int64_t mid = (lo + hi) / 2;
        if (keys[mid] == k) return mid;
        if (keys[mid] < k) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

static double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
static void cross3(const double *a, const double *b, double *c) {
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static void sub3(const double *a, const double *b, double *c) { c[0] = a[0] - b[0]; c[1] = a[1] - b[1]; c[2] = a[2] - b[2]; }

void ora_mesh_free(ora_mesh *m) {
    if (!m) return;
    free(m->xyz); free(m->tv); free(m->edges); free(m->faces);
    free(m->tet_edge); free(m->tet_face); free(m->nbr);
    free(m);
}

/* Mesh sets N, E, F, T and their incidences (Appendix A, first paragraph).
 * Returns 0 on success, -1 bad input, -4 degenerate tet or non-manifold face. */
int ora_mesh_build(int64_t nv, const double *xyz, int64_t nt, const int32_t *tv, ora_mesh **out) {
    *out = NULL;
    if (nv <= 0 || nt <= 0) return -1;
    ora_mesh *m = (ora_mesh *)calloc(1, sizeof(ora_mesh));
    m->nv = nv; m->nt = nt;
    m->xyz = (double *)malloc(sizeof(double) * 3 * nv);
    memcpy(m->xyz, xyz, sizeof(double) * 3 * nv);
    m->tv = (int32_t *)malloc(sizeof(int32_t) * 4 * nt);
    memcpy(m->tv, tv, sizeof(int32_t) * 4 * nt);
    for (int64_t t = 0; t < nt; ++t) {
        const int32_t *v = tv + 4 * t;
        for (int k = 0; k < 4; ++k)
            if (v[k] < 0 || v[k] >= nv || (k > 0 && v[k] <= v[k - 1])) { ora_mesh_free(m); return -1; }
        double a[3], b[3], c[3], bc[3];
        sub3(xyz + 3 * v[1], xyz + 3 * v[0], a);
        sub3(xyz + 3 * v[2], xyz + 3 * v[0], b);
        sub3(xyz + 3 * v[3], xyz + 3 * v[0], c);
        cross3(b, c, bc);
        double vol6 = dot3(a, bc);
        double la = sqrt(dot3(a, a)), lb = sqrt(dot3(b, b)), lc = sqrt(dot3(c, c));
        if (!(fabs(vol6) > 1e-12 * la * lb * lc)) { ora_mesh_free(m); return -4; }
    }
    /* edges */
    int64_t *ek = (int64_t *)malloc(sizeof(int64_t) * 6 * nt);
    for (int64_t t = 0; t < nt; ++t)
        for (int e = 0; e < 6; ++e)
            ek[6 * t + e] = (int64_t)tv[4 * t + LE[e][0]] * nv + tv[4 * t + LE[e][1]];
    qsort(ek, 6 * nt, sizeof(int64_t), cmp_i64);
    int64_t ne = 0;
    for (int64_t i = 0; i < 6 * nt; ++i)
        if (i == 0 || ek[i] != ek[i - 1]) ek[ne++] = ek[i];
    m->ne = ne;
    m->edges = (int32_t *)malloc(sizeof(int32_t) * 2 * ne);
    for (int64_t i = 0; i < ne; ++i) { m->edges[2 * i] = (int32_t)(ek[i] / nv); m->edges[2 * i + 1] = (int32_t)(ek[i] % nv); }
    m->tet_edge = (int32_t *)malloc(sizeof(int32_t) * 6 * nt);
    for (int64_t t = 0; t < nt; ++t)
        for (int e = 0; e < 6; ++e)
            m->tet_edge[6 * t + e] = (int32_t)find_key(ek, ne, (int64_t)tv[4 * t + LE[e][0]] * nv + tv[4 * t + LE[e][1]]);
    free(ek);
    /* faces */
    int64_t *fk = (int64_t *)malloc(sizeof(int64_t) * 4 * nt);
    for (int64_t t = 0; t < nt; ++t)
        for (int f = 0; f < 4; ++f)
            fk[4 * t + f] = ((int64_t)tv[4 * t + LF[f][0]] * nv + tv[4 * t + LF[f][1]]) * nv + tv[4 * t + LF[f][2]];
    qsort(fk, 4 * nt, sizeof(int64_t), cmp_i64);
    int64_t nf = 0;
    for (int64_t i = 0; i < 4 * nt; ++i)
        if (i == 0 || fk[i] != fk[i - 1]) fk[nf++] = fk[i];
    m->nf = nf;
    m->faces = (int32_t *)malloc(sizeof(int32_t) * 3 * nf);
    for (int64_t i = 0; i < nf; ++i) {
        int64_t k = fk[i];
        m->faces[3 * i + 2] = (int32_t)(k % nv); k /= nv;
        m->faces[3 * i + 1] = (int32_t)(k % nv); k /= nv;
        m->faces[3 * i + 0] = (int32_t)k;
    }
    m->tet_face = (int32_t *)malloc(sizeof(int32_t) * 4 * nt);
    int64_t *owner0 = (int64_t *)malloc(sizeof(int64_t) * nf);
    int64_t *owner1 = (int64_t *)malloc(sizeof(int64_t) * nf);
    for (int64_t i = 0; i < nf; ++i) owner0[i] = owner1[i] = -1;
    int bad = 0;
    for (int64_t t = 0; t < nt; ++t)
        for (int f = 0; f < 4; ++f) {
            int64_t key = ((int64_t)tv[4 * t + LF[f][0]] * nv + tv[4 * t + LF[f][1]]) * nv + tv[4 * t + LF[f][2]];
            int64_t id = find_key(fk, nf, key);
            m->tet_face[4 * t + f] = (int32_t)id;
            if (owner0[id] < 0) owner0[id] = t;
            else if (owner1[id] < 0) owner1[id] = t;
            else bad = 1;
        }
    m->nbr = (int32_t *)malloc(sizeof(int32_t) * 4 * nt);
    for (int64_t t = 0; t < nt; ++t)
        for (int f = 0; f < 4; ++f) {
            int64_t id = m->tet_face[4 * t + f];
            int64_t o = owner0[id] == t ? owner1[id] : owner0[id];
            m->nbr[4 * t + f] = (int32_t)o;
        }
    free(owner0); free(owner1); free(fk);
    if (bad) { ora_mesh_free(m); return -4; }
    *out = m;
    return 0;
}

void ora_mesh_counts(const ora_mesh *m, int64_t *out4) { out4[0] = m->nv; out4[1] = m->ne; out4[2] = m->nf; out4[3] = m->nt; }
void ora_mesh_edges(const ora_mesh *m, int32_t *out) { memcpy(out, m->edges, sizeof(int32_t) * 2 * m->ne); }
void ora_mesh_faces(const ora_mesh *m, int32_t *out) { memcpy(out, m->faces, sizeof(int32_t) * 3 * m->nf); }
void ora_mesh_tet_edges(const ora_mesh *m, int32_t *out) { memcpy(out, m->tet_edge, sizeof(int32_t) * 6 * m->nt); }
void ora_mesh_tet_faces(const ora_mesh *m, int32_t *out) { memcpy(out, m->tet_face, sizeof(int32_t) * 4 * m->nt); }
void ora_mesh_neighbours(const ora_mesh *m, int32_t *out) { memcpy(out, m->nbr, sizeof(int32_t) * 4 * m->nt); }

/* Barycentric gradients of tet T.  lambda_k is affine, 0 on the face opposite
 * vertex k and 1 at vertex k, so its gradient is a face normal n scaled by
 * 1/(n.(r_k - r_a)) for any point r_a of that face (W0 = barycentric, App. A). */
void ora_grad(const ora_mesh *m, int64_t T, double g[4][3]) {
    const int32_t *v = m->tv + 4 * T;
    for (int k = 0; k < 4; ++k) {
        const double *ra = m->xyz + 3 * v[LF[k][0]], *rb = m->xyz + 3 * v[LF[k][1]], *rc = m->xyz + 3 * v[LF[k][2]];
        const double *rk = m->xyz + 3 * v[k];
        double ab[3], ac[3], n[3], ak[3];
        sub3(rb, ra, ab); sub3(rc, ra, ac); cross3(ab, ac, n); sub3(rk, ra, ak);
        double s = 1.0 / dot3(n, ak);
        g[k][0] = n[0] * s; g[k][1] = n[1] * s; g[k][2] = n[2] * s;
    }
}

/* Cartesian -> barycentric by Cramer's rule (ratio of signed volumes). */
void ora_bary(const ora_mesh *m, int64_t T, const double *x, double lam[4]) {
    const int32_t *v = m->tv + 4 * T;
    for (int k = 0; k < 4; ++k) {
        const double *ra = m->xyz + 3 * v[LF[k][0]], *rb = m->xyz + 3 * v[LF[k][1]], *rc = m->xyz + 3 * v[LF[k][2]];
        const double *rk = m->xyz + 3 * v[k];
        double ab[3], ac[3], n[3], ak[3], ax[3];
        sub3(rb, ra, ab); sub3(rc, ra, ac); cross3(ab, ac, n); sub3(rk, ra, ak); sub3(x, ra, ax);
        lam[k] = dot3(n, ax) / dot3(n, ak);
    }
}

/* barycentric -> Cartesian: x = sum_k lambda_k r_k */
void ora_point(const ora_mesh *m, int64_t T, const double lam[4], double *x) {
    const int32_t *v = m->tv + 4 * T;
    x[0] = x[1] = x[2] = 0.0;
    for (int k = 0; k < 4; ++k)
        for (int c = 0; c < 3; ++c) x[c] += lam[k] * m->xyz[3 * v[k] + c];
}

/* Whitney edge functions of tet T at barycentric point lam (Formulation, the
 * E~ expansion, lowest-order edge elements): W1_ij = l_i grad l_j - l_j grad l_i. */
void ora_whitney1(const ora_mesh *m, int64_t T, const double lam[4], double W[6][3]) {
    double g[4][3];
    ora_grad(m, T, g);
    for (int e = 0; e < 6; ++e) {
        int i = LE[e][0], j = LE[e][1];
        for (int c = 0; c < 3; ++c) W[e][c] = lam[i] * g[j][c] - lam[j] * g[i][c];
    }
}

/* Whitney face functions (the B~ expansion): for face (i<j<k)
 * W2 = 2 (l_i gl_j x gl_k + l_j gl_k x gl_i + l_k gl_i x gl_j). */
void ora_whitney2(const ora_mesh *m, int64_t T, const double lam[4], double W[4][3]) {
    double g[4][3];
    ora_grad(m, T, g);
    for (int f = 0; f < 4; ++f) {
        int i = LF[f][0], j = LF[f][1], k = LF[f][2];
        double jk[3], ki[3], ij[3];
        cross3(g[j], g[k], jk); cross3(g[k], g[i], ki); cross3(g[i], g[j], ij);
        for (int c = 0; c < 3; ++c) W[f][c] = 2.0 * (lam[i] * jk[c] + lam[j] * ki[c] + lam[k] * ij[c]);
    }
}

typedef struct {
    const double *e_env; /* ne*2 (re,im) */
    const double *e_dc;  /* ne or NULL */
    const double *b_env; /* nf*2 */
    const double *b_dc;  /* nf or NULL */
} ora_fields_t;

/* Physical fields at (T, lam) and carrier phase (c, s) = (cos wt, sin wt):
 * E = Re{ sum_e e~_e W1_e e^{jwt} } + sum_e e_dc,e W1_e, and likewise B with W2.
 * Edge-by-edge sums, no pre-contraction. */
static void fields_at(const ora_mesh *m, int64_t T, const double lam[4], double c, double s,
                      const ora_fields_t *F, double E[3], double B[3]) {
    double W1[6][3], W2[4][3];
    ora_whitney1(m, T, lam, W1);
    ora_whitney2(m, T, lam, W2);
    E[0] = E[1] = E[2] = 0.0;
    B[0] = B[1] = B[2] = 0.0;
    for (int e = 0; e < 6; ++e) {
        int64_t id = m->tet_edge[6 * T + e];
        double re = F->e_env[2 * id], im = F->e_env[2 * id + 1];
        double coef = re * c - im * s;           /* Re{(re + j im)(c + j s)} */
        if (F->e_dc) coef += F->e_dc[id];
        for (int k = 0; k < 3; ++k) E[k] += coef * W1[e][k];
    }
    for (int f = 0; f < 4; ++f) {
        int64_t id = m->tet_face[4 * T + f];
        double re = F->b_env[2 * id], im = F->b_env[2 * id + 1];
        double coef = re * c - im * s;
        if (F->b_dc) coef += F->b_dc[id];
        for (int k = 0; k < 3; ++k) B[k] += coef * W2[f][k];
    }
}

void ora_fields(const ora_mesh *m, int64_t T, const double lam[4], double omega, double t,
                const double *e_env, const double *e_dc, const double *b_env, const double *b_dc,
                double E[3], double B[3]) {
    ora_fields_t F = {e_env, e_dc, b_env, b_dc};
    fields_at(m, T, lam, cos(omega * t), sin(omega * t), &F, E, B);
}

/* Textbook Boris rotation (non-relativistic): half electric kick, magnetic
 * rotation by the implicit-midpoint rule, half electric kick. */
static void boris(double v[3], const double E[3], const double B[3], double qm, double dt) {
    double h = 0.5 * qm * dt;
    double vm[3], tau[3], sig[3], vp[3], cr[3];
    for (int k = 0; k < 3; ++k) { vm[k] = v[k] + h * E[k]; tau[k] = h * B[k]; }
    double t2 = dot3(tau, tau);
    for (int k = 0; k < 3; ++k) sig[k] = 2.0 * tau[k] / (1.0 + t2);
    cross3(vm, tau, cr);
    double vpr[3] = {vm[0] + cr[0], vm[1] + cr[1], vm[2] + cr[2]};
    cross3(vpr, sig, cr);
    for (int k = 0; k < 3; ++k) vp[k] = vm[k] + cr[k];
    for (int k = 0; k < 3; ++k) v[k] = vp[k] + h * E[k];
}

void ora_boris(double *v, const double *E, const double *B, double qm, double dt) { boris(v, E, B, qm, dt); }

/* Path integral of the six Whitney edge functions of tet T along the straight
 * piece that starts at barycentric point la and has Cartesian displacement d.
 * The integrand W1(r).dr is affine along a straight piece, so the midpoint rule
 * is exact: g_e = W1_e(midpoint) . d. */
static void piece_integral(const ora_mesh *m, int64_t T, const double la[4], const double dl[4],
                           const double d[3], double g[6]) {
    double mid[4], W1[6][3];
    for (int k = 0; k < 4; ++k) mid[k] = la[k] + 0.5 * dl[k];
    ora_whitney1(m, T, mid, W1);
    for (int e = 0; e < 6; ++e) g[e] = dot3(W1[e], d);
}

typedef struct {
    int64_t tet;
    double lam[4];
    double v[3];
    int hops;
    int status; /* 0 ok, -6 hop cap */
} ora_particle;

/* The walk's geometry is taken in extended precision (x87 long double, a
 * 64-bit significand).  The crossing parameter of a piece is the distance to a
 * face plane divided by the rate of approach, so it is as uncertain as the
 * start point's distance from the plane divided by the step's barycentric
 * length, ~1e-5 or less here: in float64 a Cartesian reconstruction of the
 * start point would leave the crossing point uncertain at the 1e-11 level.  The
 * extra digits keep the oracle's path exact to float64 rounding of its inputs. */
typedef long double xreal;

static void sub3x(const xreal *a, const xreal *b, xreal *c) { c[0] = a[0] - b[0]; c[1] = a[1] - b[1]; c[2] = a[2] - b[2]; }
static xreal dot3x(const xreal *a, const xreal *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Face k of a tet as a plane in Cartesian space: n = (r_b - r_a) x (r_c - r_a)
 * from the face's vertices a < b < c, turned to point into the tet; a point of
 * the plane (r_a, stored as an offset from the tet's vertex 0); and the height
 * h = n . (r_k - r_a) > 0 of the opposite vertex over the plane.  The signed
 * distance of a point y (offset from vertex 0) from the plane, scaled by |n|,
 * is n . (y - a): positive inside the tet. */
typedef struct {
    xreal n[3];
    xreal a[3];
    xreal h;
} ora_plane;

static void tet_planes(const ora_mesh *m, int64_t T, ora_plane pl[4]) {
    const int32_t *v = m->tv + 4 * T;
    xreal r[4][3];
    for (int k = 0; k < 4; ++k)
        for (int c = 0; c < 3; ++c) r[k][c] = (xreal)m->xyz[3 * v[k] + c] - (xreal)m->xyz[3 * v[0] + c];
    for (int k = 0; k < 4; ++k) {
        const xreal *ra = r[LF[k][0]], *rb = r[LF[k][1]], *rc = r[LF[k][2]];
        xreal ab[3], ac[3], ak[3];
        sub3x(rb, ra, ab); sub3x(rc, ra, ac); sub3x(r[k], ra, ak);
        pl[k].n[0] = ab[1] * ac[2] - ab[2] * ac[1];
        pl[k].n[1] = ab[2] * ac[0] - ab[0] * ac[2];
        pl[k].n[2] = ab[0] * ac[1] - ab[1] * ac[0];
        pl[k].h = dot3x(pl[k].n, ak);
        if (pl[k].h < 0.0L) {
            for (int c = 0; c < 3; ++c) pl[k].n[c] = -pl[k].n[c];
            pl[k].h = -pl[k].h;
        }
        for (int c = 0; c < 3; ++c) pl[k].a[c] = ra[c];
    }
}

/* Barycentric coordinates of the point y (offset from the tet's vertex 0) by
 * Cramer's rule: lambda_k = (volume of the tet the point spans with face k) /
 * (volume of the tet) = n_k . (y - a_k) / h_k. */
static void plane_bary(const ora_plane pl[4], const xreal y[3], xreal lam[4]) {
    for (int k = 0; k < 4; ++k) {
        xreal ya[3];
        sub3x(y, pl[k].a, ya);
        lam[k] = dot3x(pl[k].n, ya) / pl[k].h;
    }
}

/* Walk of the straight path with Cartesian displacement d from the particle's
 * (tet, lam), depositing q*w*(path integral) of every piece into dG (the sum
 * over pieces that eq. G_integral and the sum after it take).  The walk is
 * Cartesian: the point is carried as an offset y from vertex 0 of its tet; the
 * segment y -> y + d is intersected with the four face planes, and the piece
 * ends at the smallest parameter s in [0, 1] where it passes behind one of them
 * (ties: the lowest local face; a point already behind a plane it moves away
 * from leaves at s = 0).  The barycentric change of a piece is Cramer's rule
 * applied to its displacement; at a crossing the point is re-expressed from the
 * neighbour's vertex 0 and its barycentrics there are computed afresh by
 * Cramer's rule.  At a boundary face (the paper is silent on the particle
 * boundary condition; walls are conductors) the remaining displacement and
 * the velocity P->v are mirrored about the plane's unit normal, and so are the
 * nextra vectors extra[i] (velocity samples a multistep integrator keeps).
 * R (optional) accumulates the linear part of the reflections. */
static void walk_path(const ora_mesh *m, ora_particle *P, double d_io[3], double qw, double *dG, int64_t *piece_tets,
                      int *npieces_out, double *R, double (*extra)[3], int nextra) {
    int64_t T = P->tet;
    xreal l[4] = {1.0L - ((xreal)P->lam[1] + (xreal)P->lam[2] + (xreal)P->lam[3]), P->lam[1], P->lam[2], P->lam[3]};
    xreal d[3] = {d_io[0], d_io[1], d_io[2]};
    ora_plane pl[4];
    tet_planes(m, T, pl);
    xreal y[3] = {0.0L, 0.0L, 0.0L};
    {
        const int32_t *v = m->tv + 4 * T;
        for (int j = 1; j < 4; ++j)
            for (int c = 0; c < 3; ++c) y[c] += l[j] * ((xreal)m->xyz[3 * v[j] + c] - (xreal)m->xyz[3 * v[0] + c]);
    }
    int hops = 0, np = 0;
    P->status = 0;
    for (;;) {
        xreal s = 1.0L;
        int kmin = -1;
        for (int k = 0; k < 4; ++k) {
            xreal ya[3];
            sub3x(y, pl[k].a, ya);
            xreal dist = dot3x(pl[k].n, ya), rate = dot3x(pl[k].n, d);
            if (rate < 0.0L && dist + rate < 0.0L) {
                xreal sk = dist > 0.0L ? dist / (-rate) : 0.0L;
                if (kmin < 0 || sk < s) { s = sk; kmin = k; }
            }
        }
        xreal dp[3] = {s * d[0], s * d[1], s * d[2]};
        xreal dl[4];
        for (int k = 0; k < 4; ++k) dl[k] = dot3x(pl[k].n, dp) / pl[k].h;
        {
            double la[4], dla[4], dpa[3], gp[6];
            for (int k = 0; k < 4; ++k) { la[k] = (double)l[k]; dla[k] = (double)dl[k]; }
            for (int c = 0; c < 3; ++c) dpa[c] = (double)dp[c];
            piece_integral(m, T, la, dla, dpa, gp);
            for (int e = 0; e < 6; ++e) dG[m->tet_edge[6 * T + e]] += qw * gp[e];
        }
        if (piece_tets && np < ORA_HOP_CAP + 1) piece_tets[np] = T;
        ++np;
        for (int k = 0; k < 4; ++k) l[k] += dl[k];
        if (kmin < 0) break;
        for (int c = 0; c < 3; ++c) { y[c] += dp[c]; d[c] -= dp[c]; }
        int64_t nb = m->nbr[4 * T + kmin];
        if (nb < 0) {
            xreal nn = sqrtl(dot3x(pl[kmin].n, pl[kmin].n));
            xreal nh[3] = {pl[kmin].n[0] / nn, pl[kmin].n[1] / nn, pl[kmin].n[2] / nn};
            xreal dd = dot3x(d, nh);
            double nd[3] = {(double)nh[0], (double)nh[1], (double)nh[2]};
            double vv = dot3(P->v, nd);
            for (int k = 0; k < 3; ++k) { d[k] -= 2.0L * dd * nh[k]; P->v[k] -= 2.0 * vv * nd[k]; }
            for (int i = 0; i < nextra; ++i) {
                double xv = dot3(extra[i], nd);
                for (int k = 0; k < 3; ++k) extra[i][k] -= 2.0 * xv * nd[k];
            }
            if (R) {   /* R <- (I - 2 n n^T) R : the linear part of the reflected end point */
                double Rn[9];
                for (int i = 0; i < 3; ++i)
                    for (int j = 0; j < 3; ++j) {
                        double acc = 0.0;
                        for (int k = 0; k < 3; ++k) acc += ((i == k ? 1.0 : 0.0) - 2.0 * nd[i] * nd[k]) * R[3 * k + j];
                        Rn[3 * i + j] = acc;
                    }
                memcpy(R, Rn, sizeof Rn);
            }
        } else {
            const int32_t v0 = m->tv[4 * T], w0 = m->tv[4 * nb];
            for (int c = 0; c < 3; ++c) y[c] += (xreal)m->xyz[3 * v0 + c] - (xreal)m->xyz[3 * w0 + c];
            T = nb;
            tet_planes(m, T, pl);
            plane_bary(pl, y, l);
        }
        if (++hops > ORA_HOP_CAP) { P->status = -6; break; }
    }
    P->tet = T;
    for (int k = 0; k < 4; ++k) P->lam[k] = (double)l[k];
    for (int c = 0; c < 3; ++c) d_io[c] = (double)d[c];
    P->hops = hops;
    if (npieces_out) *npieces_out = np;
}

/* One fine step of one particle: gather at (x^n, t_n), Boris, walk, deposit.
 * qw_dG receives q*w*(path integrals) for every piece (6 edges per piece). */
static void step_one(const ora_mesh *m, ora_particle *P, double c, double s, const ora_fields_t *F,
                     double qm, double dt, double qw, double *dG, int64_t *piece_tets, int *npieces_out,
                     double *R) {
    double E[3], B[3];
    fields_at(m, P->tet, P->lam, c, s, F, E, B);
    boris(P->v, E, B, qm, dt);
    double d[3] = {dt * P->v[0], dt * P->v[1], dt * P->v[2]};
    walk_path(m, P, d, qw, dG, piece_tets, npieces_out, R, NULL, 0);
}

/*
 * One step for n particles.  State in and out: tet[n], lam[n*3] (lambda1..3 of
 * the ascending local order, lambda0 = 1 - sum), vel[n*3] (v^{n-1/2} in,
 * v^{n+1/2} out).  t_n = step*dt; the carrier phase is evaluated here.
 * dG[ne] accumulates q*w*path integrals; rho[nv] (optional) accumulates
 * q*w*lambda_k at the end point.  hops[n] optional.  nthreads <= 1: serial.
 * Returns 0, or -6 if any particle exceeded the hop cap.
 */
int ora_step_t(const ora_mesh *m, int64_t n, int32_t *tet, double *lam, double *vel,
               double q, double mass, double w, double t, double dt, double omega,
               const double *e_env, const double *e_dc, const double *b_env, const double *b_dc,
               double *dG, double *rho, int32_t *hops, int nthreads);

int ora_step(const ora_mesh *m, int64_t n, int32_t *tet, double *lam, double *vel,
             double q, double mass, double w, int64_t step, double dt, double omega,
             const double *e_env, const double *e_dc, const double *b_env, const double *b_dc,
             double *dG, double *rho, int32_t *hops, int nthreads) {
    return ora_step_t(m, n, tet, lam, vel, q, mass, w, (double)step * dt, dt, omega, e_env, e_dc, b_env, b_dc,
                      dG, rho, hops, nthreads);
}

/* The same step with the gather time t given directly (the fine steps of a
 * coarse field step). */
int ora_step_t(const ora_mesh *m, int64_t n, int32_t *tet, double *lam, double *vel,
               double q, double mass, double w, double t, double dt, double omega,
               const double *e_env, const double *e_dc, const double *b_env, const double *b_dc,
               double *dG, double *rho, int32_t *hops, int nthreads) {
    ora_fields_t F = {e_env, e_dc, b_env, b_dc};
    double c = cos(omega * t), s = sin(omega * t);
    double qm = q / mass, qw = q * w;
    int status = 0;
    int nth = nthreads > 1 ? nthreads : 1;
#ifndef _OPENMP
    nth = 1;
#endif
    if (nth == 1) {
        for (int64_t p = 0; p < n; ++p) {
            ora_particle P;
            P.tet = tet[p];
            P.lam[1] = lam[3 * p]; P.lam[2] = lam[3 * p + 1]; P.lam[3] = lam[3 * p + 2];
            P.lam[0] = 1.0 - P.lam[1] - P.lam[2] - P.lam[3];
            P.v[0] = vel[3 * p]; P.v[1] = vel[3 * p + 1]; P.v[2] = vel[3 * p + 2];
            step_one(m, &P, c, s, &F, qm, dt, qw, dG, NULL, NULL, NULL);
            tet[p] = (int32_t)P.tet;
            lam[3 * p] = P.lam[1]; lam[3 * p + 1] = P.lam[2]; lam[3 * p + 2] = P.lam[3];
            vel[3 * p] = P.v[0]; vel[3 * p + 1] = P.v[1]; vel[3 * p + 2] = P.v[2];
            if (hops) hops[p] = P.hops;
            if (P.status) status = P.status;
            if (rho) {
                const int32_t *v = m->tv + 4 * P.tet;
                for (int k = 0; k < 4; ++k) rho[v[k]] += qw * P.lam[k];
            }
        }
        return status;
    }
#ifdef _OPENMP
    double *priv = (double *)calloc((size_t)nth * (m->ne + (rho ? m->nv : 0)), sizeof(double));
    #pragma omp parallel num_threads(nth) reduction(min:status)
    {
        int tid = omp_get_thread_num();
        double *mydG = priv + (size_t)tid * (m->ne + (rho ? m->nv : 0));
        double *myrho = rho ? mydG + m->ne : NULL;
        #pragma omp for schedule(static)
        for (int64_t p = 0; p < n; ++p) {
            ora_particle P;
            P.tet = tet[p];
            P.lam[1] = lam[3 * p]; P.lam[2] = lam[3 * p + 1]; P.lam[3] = lam[3 * p + 2];
            P.lam[0] = 1.0 - P.lam[1] - P.lam[2] - P.lam[3];
            P.v[0] = vel[3 * p]; P.v[1] = vel[3 * p + 1]; P.v[2] = vel[3 * p + 2];
            step_one(m, &P, c, s, &F, qm, dt, qw, mydG, NULL, NULL, NULL);
            tet[p] = (int32_t)P.tet;
            lam[3 * p] = P.lam[1]; lam[3 * p + 1] = P.lam[2]; lam[3 * p + 2] = P.lam[3];
            vel[3 * p] = P.v[0]; vel[3 * p + 1] = P.v[1]; vel[3 * p + 2] = P.v[2];
            if (hops) hops[p] = P.hops;
            if (P.status) status = P.status;
            if (myrho) {
                const int32_t *v = m->tv + 4 * P.tet;
                for (int k = 0; k < 4; ++k) myrho[v[k]] += qw * P.lam[k];
            }
        }
    }
    for (int th = 0; th < nth; ++th) {
        double *mydG = priv + (size_t)th * (m->ne + (rho ? m->nv : 0));
        for (int64_t e = 0; e < m->ne; ++e) dG[e] += mydG[e];
        if (rho) for (int64_t k = 0; k < m->nv; ++k) rho[k] += mydG[m->ne + k];
    }
    free(priv);
#endif
    return status;
}

/* Vertex charge of the particles (rho = q sum_p S(r - r_p) with the W0 shape):
 * rho_k += q*w*lambda_k(x_p) for the four vertices of the particle's tet. */
void ora_charge(const ora_mesh *m, int64_t n, const int32_t *tet, const double *lam, double q, double w, double *rho) {
    for (int64_t p = 0; p < n; ++p) {
        const int32_t *v = m->tv + 4 * (int64_t)tet[p];
        double l1 = lam[3 * p], l2 = lam[3 * p + 1], l3 = lam[3 * p + 2];
        double l[4] = {1.0 - l1 - l2 - l3, l1, l2, l3};
        for (int k = 0; k < 4; ++k) rho[v[k]] += q * w * l[k];
    }
}

/* Discrete continuity residual (section on charge conservation: the discrete
 * divergence of G is tied to rho).  D is the edge-vertex incidence with -1 at
 * the tail and +1 at the head; r = D^T dG - (rho_new - rho_old).
 * out[0] = max|r|, out[1] = max|rho_old|. */
void ora_gauss(const ora_mesh *m, const double *dG, const double *rho_new, const double *rho_old, double *out) {
    double *r = (double *)calloc(m->nv, sizeof(double));
    for (int64_t e = 0; e < m->ne; ++e) {
        r[m->edges[2 * e + 1]] += dG[e];
        r[m->edges[2 * e]] -= dG[e];
    }
    double rmax = 0.0, pmax = 0.0;
    for (int64_t k = 0; k < m->nv; ++k) {
        double v = fabs(r[k] - (rho_new[k] - rho_old[k]));
        if (v > rmax) rmax = v;
        if (fabs(rho_old[k]) > pmax) pmax = fabs(rho_old[k]);
    }
    out[0] = rmax; out[1] = pmax;
    free(r);
}

/* Brute-force point location over all tets: the tet whose barycentrics of x
 * have the largest minimum (>= -tol means inside).  Returns the tet, writes
 * the min barycentric to *minlam. */
int64_t ora_locate(const ora_mesh *m, const double *x, double *minlam) {
    int64_t best = -1;
    double bmin = -1e300;
    for (int64_t t = 0; t < m->nt; ++t) {
        double l[4];
        ora_bary(m, t, x, l);
        double mn = l[0];
        for (int k = 1; k < 4; ++k) if (l[k] < mn) mn = l[k];
        if (mn > bmin) { bmin = mn; best = t; }
    }
    if (minlam) *minlam = bmin;
    return best;
}

/* Single particle, single step, with per-piece tets reported (walk tests). */
int ora_step_one(const ora_mesh *m, int32_t *tet, double *lam3, double *v, double q, double mass, double w,
                 int64_t step, double dt, double omega, const double *e_env, const double *e_dc,
                 const double *b_env, const double *b_dc, double *dG, int64_t *piece_tets, int32_t *npieces) {
    ora_fields_t F = {e_env, e_dc, b_env, b_dc};
    double t = (double)step * dt;
    ora_particle P;
    P.tet = *tet;
    P.lam[1] = lam3[0]; P.lam[2] = lam3[1]; P.lam[3] = lam3[2];
    P.lam[0] = 1.0 - lam3[0] - lam3[1] - lam3[2];
    P.v[0] = v[0]; P.v[1] = v[1]; P.v[2] = v[2];
    int np = 0;
    step_one(m, &P, cos(omega * t), sin(omega * t), &F, q / mass, dt, q * w, dG, piece_tets, &np, NULL);
    *tet = (int32_t)P.tet;
    lam3[0] = P.lam[1]; lam3[1] = P.lam[2]; lam3[2] = P.lam[3];
    v[0] = P.v[0]; v[1] = P.v[1]; v[2] = P.v[2];
    *npieces = np;
    return P.status;
}

/* ------------------------------------------------------------------------
 * Reverse-mode derivative of nsteps particle steps (the gradient path of the
 * differentiation workload).  For each particle independently (the fields are
 * given, so trajectories do not interact): run the steps forward keeping the
 * state before every step and the linear part R of that step's wall
 * reflections, then go backwards through position update, Boris and gather.
 * Given vbar / xbar, the adjoints of the final velocity and (Cartesian)
 * position, accumulate into grad_e[2*ne] the gradient with respect to the
 * complex edge envelope in the convention d/dRe + j d/dIm, and return the
 * adjoints of the initial velocity and position if asked.  Tet sequences and
 * reflections are those of the forward run (the map is piecewise smooth).
 * The face envelope and the dc DoFs are held fixed.
 */
static void boris_fwd(const double v[3], const double E[3], const double B[3], double h, double vm[3], double tau[3],
                      double sig[3], double vpr[3], double out[3]) {
    double cr[3];
    for (int k = 0; k < 3; ++k) { vm[k] = v[k] + h * E[k]; tau[k] = h * B[k]; }
    double t2 = dot3(tau, tau);
    for (int k = 0; k < 3; ++k) sig[k] = 2.0 * tau[k] / (1.0 + t2);
    cross3(vm, tau, cr);
    for (int k = 0; k < 3; ++k) vpr[k] = vm[k] + cr[k];
    cross3(vpr, sig, cr);
    for (int k = 0; k < 3; ++k) out[k] = vm[k] + cr[k] + h * E[k];
}

/* adjoint of boris_fwd: given obar (adjoint of out) produce vbar, Ebar, Bbar */
static void boris_vjp(const double vm[3], const double tau[3], const double sig[3], const double vpr[3], double h,
                      const double obar[3], double vbar[3], double Ebar[3], double Bbar[3]) {
    double vmbar[3], vprbar[3], sigbar[3], taubar[3], cr[3];
    /* out = vm + vpr x sig + h E */
    for (int k = 0; k < 3; ++k) { vmbar[k] = obar[k]; Ebar[k] = h * obar[k]; }
    cross3(sig, obar, vprbar);              /* d(vpr x sig)/dvpr ^T obar = sig x obar */
    cross3(obar, vpr, sigbar);              /* d(vpr x sig)/dsig ^T obar = obar x vpr */
    /* vpr = vm + vm x tau */
    cross3(tau, vprbar, cr);
    for (int k = 0; k < 3; ++k) vmbar[k] += vprbar[k] + cr[k];
    cross3(vprbar, vm, taubar);
    /* sig = 2 tau / (1 + |tau|^2) */
    double t2 = dot3(tau, tau), den = 1.0 + t2, st = dot3(sigbar, tau);
    for (int k = 0; k < 3; ++k) taubar[k] += 2.0 * sigbar[k] / den - 4.0 * st * tau[k] / (den * den);
    /* tau = h B ; vm = v + h E */
    for (int k = 0; k < 3; ++k) { Bbar[k] = h * taubar[k]; vbar[k] = vmbar[k]; Ebar[k] += h * vmbar[k]; }
}

int ora_vjp(const ora_mesh *m, int64_t n, const int32_t *tet0, const double *lam0, const double *vel0, double q,
            double mass, double w, int64_t step0, int nsteps, double dt, double omega, const double *e_env,
            const double *e_dc, const double *b_env, const double *b_dc, const double *vbar_in,
            const double *xbar_in, double *grad_e, double *vbar_out, double *xbar_out, int nthreads) {
    ora_fields_t F = {e_env, e_dc, b_env, b_dc};
    double qm = q / mass, h = 0.5 * qm * dt;
    int status = 0;
    int nth = nthreads > 1 ? nthreads : 1;
#ifndef _OPENMP
    nth = 1;
#endif
    double *priv = (double *)calloc((size_t)nth * 2 * m->ne, sizeof(double));
    #pragma omp parallel num_threads(nth) reduction(min:status)
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *g = priv + (size_t)tid * 2 * m->ne;
        ora_particle *st = (ora_particle *)malloc(sizeof(ora_particle) * (nsteps + 1));
        double *Rs = (double *)malloc(sizeof(double) * 9 * (nsteps + 1));
        double *dummy = (double *)calloc(m->ne, sizeof(double));
        #pragma omp for schedule(static)
        for (int64_t p = 0; p < n; ++p) {
            ora_particle P;
            P.tet = tet0[p];
            P.lam[1] = lam0[3 * p]; P.lam[2] = lam0[3 * p + 1]; P.lam[3] = lam0[3 * p + 2];
            P.lam[0] = 1.0 - P.lam[1] - P.lam[2] - P.lam[3];
            for (int k = 0; k < 3; ++k) P.v[k] = vel0[3 * p + k];
            for (int k = 0; k < nsteps; ++k) {
                st[k] = P;
                double *R = Rs + 9 * k;
                for (int i = 0; i < 9; ++i) R[i] = (i % 4 == 0) ? 1.0 : 0.0;
                double t = (double)(step0 + k) * dt;
                step_one(m, &P, cos(omega * t), sin(omega * t), &F, qm, dt, 0.0, dummy, NULL, NULL, R);
                if (P.status) status = P.status;
            }
            double vb[3], xb[3];
            for (int k = 0; k < 3; ++k) { vb[k] = vbar_in[3 * p + k]; xb[k] = xbar_in ? xbar_in[3 * p + k] : 0.0; }
            for (int k = nsteps - 1; k >= 0; --k) {
                const ora_particle *S = &st[k];
                const double *R = Rs + 9 * k;
                double t = (double)(step0 + k) * dt, c = cos(omega * t), sn = sin(omega * t);
                double E[3], B[3];
                fields_at(m, S->tet, S->lam, c, sn, &F, E, B);
                double vm[3], tau[3], sig[3], vpr[3], out[3];
                boris_fwd(S->v, E, B, h, vm, tau, sig, vpr, out);
                /* x_{k+1} = R (x_k + dt out) + const ; v_{k+1} = R out */
                double ob[3], xk[3];
                for (int i = 0; i < 3; ++i) {
                    ob[i] = 0.0; xk[i] = 0.0;
                    for (int j = 0; j < 3; ++j) { ob[i] += R[3 * j + i] * (vb[j] + dt * xb[j]); xk[i] += R[3 * j + i] * xb[j]; }
                }
                double vin[3], Eb[3], Bb[3];
                boris_vjp(vm, tau, sig, vpr, h, ob, vin, Eb, Bb);
                /* gather: E = sum_e eps_e W1_e(x), B = sum_f beta_f W2_f(x), W affine in x */
                double gr[4][3];
                ora_grad(m, S->tet, gr);
                for (int e = 0; e < 6; ++e) {
                    int i = LE[e][0], j = LE[e][1];
                    int64_t id = m->tet_edge[6 * S->tet + e];
                    double eps = F.e_env[2 * id] * c - F.e_env[2 * id + 1] * sn + (F.e_dc ? F.e_dc[id] : 0.0);
                    double Ei = dot3(Eb, gr[i]), Ej = dot3(Eb, gr[j]);
                    for (int b = 0; b < 3; ++b) xk[b] += eps * (Ej * gr[i][b] - Ei * gr[j][b]);
                    double wdot = S->lam[i] * Ej - S->lam[j] * Ei;          /* Ebar . W1_e(x_k) */
                    g[2 * id] += wdot * c;
                    g[2 * id + 1] -= wdot * sn;
                }
                for (int f = 0; f < 4; ++f) {
                    int i = LF[f][0], j = LF[f][1], kk = LF[f][2];
                    int64_t id = m->tet_face[4 * S->tet + f];
                    double beta = F.b_env[2 * id] * c - F.b_env[2 * id + 1] * sn + (F.b_dc ? F.b_dc[id] : 0.0);
                    double jk[3], ki[3], ij[3];
                    cross3(gr[j], gr[kk], jk); cross3(gr[kk], gr[i], ki); cross3(gr[i], gr[j], ij);
                    double a1 = dot3(Bb, jk), a2 = dot3(Bb, ki), a3 = dot3(Bb, ij);
                    for (int b = 0; b < 3; ++b) xk[b] += 2.0 * beta * (a1 * gr[i][b] + a2 * gr[j][b] + a3 * gr[kk][b]);
                }
                for (int i = 0; i < 3; ++i) { vb[i] = vin[i]; xb[i] = xk[i]; }
            }
            if (vbar_out) for (int k = 0; k < 3; ++k) vbar_out[3 * p + k] = vb[k];
            if (xbar_out) for (int k = 0; k < 3; ++k) xbar_out[3 * p + k] = xb[k];
        }
        free(st); free(Rs); free(dummy);
    }
    for (int th = 0; th < nth; ++th)
        for (int64_t i = 0; i < 2 * m->ne; ++i) grad_e[i] += priv[(size_t)th * 2 * m->ne + i];
    free(priv);
    return status;
}

/* ------------------------------------------------------------------------
 * Tangent-linear (forward-mode) derivative of nsteps particle steps along one
 * direction de of the complex edge envelope: the same steps as step_one, in
 * dual numbers (value, derivative).  It is a second, independent derivative
 * of the differentiation workload's map, against which the reverse mode
 * (ora_vjp) and the GPU adjoint are checked: dL = sum_p m w v_p . dv_p must
 * equal Re(grad) . Re(de) + Im(grad) . Im(de).  Decisions (exit face, wall)
 * are taken on the values, so the tet sequence and the reflections are those
 * of the forward run, as in the reverse mode.  Mesh geometry, the face
 * envelope and the dc DoFs are constants.
 */
typedef struct { double v, d; } dual;

static dual dmk(double v, double d) { dual r = {v, d}; return r; }
static dual dadd(dual a, dual b) { return dmk(a.v + b.v, a.d + b.d); }
static dual dsub(dual a, dual b) { return dmk(a.v - b.v, a.d - b.d); }
static dual dmul(dual a, dual b) { return dmk(a.v * b.v, a.d * b.v + a.v * b.d); }
static dual dscale(dual a, double s) { return dmk(a.v * s, a.d * s); }
static dual ddiv(dual a, dual b) { return dmk(a.v / b.v, (a.d * b.v - a.v * b.d) / (b.v * b.v)); }
static dual ddot3(const dual *a, const double *b) {
    return dmk(a[0].v * b[0] + a[1].v * b[1] + a[2].v * b[2], a[0].d * b[0] + a[1].d * b[1] + a[2].d * b[2]);
}
static void dcross3(const dual *a, const dual *b, dual *c) {
    c[0] = dsub(dmul(a[1], b[2]), dmul(a[2], b[1]));
    c[1] = dsub(dmul(a[2], b[0]), dmul(a[0], b[2]));
    c[2] = dsub(dmul(a[0], b[1]), dmul(a[1], b[0]));
}

/* fields at a dual barycentric point; the edge DoFs' derivative is the
 * direction de through the same carrier factor */
static void fields_at_dual(const ora_mesh *m, int64_t T, const dual lam[4], double c, double s,
                           const ora_fields_t *F, const double *de, dual E[3], dual B[3]) {
    double g[4][3];
    ora_grad(m, T, g);
    for (int k = 0; k < 3; ++k) { E[k] = dmk(0.0, 0.0); B[k] = dmk(0.0, 0.0); }
    for (int e = 0; e < 6; ++e) {
        int i = LE[e][0], j = LE[e][1];
        int64_t id = m->tet_edge[6 * T + e];
        double coef = F->e_env[2 * id] * c - F->e_env[2 * id + 1] * s + (F->e_dc ? F->e_dc[id] : 0.0);
        double dcoef = de[2 * id] * c - de[2 * id + 1] * s;
        dual cf = dmk(coef, dcoef);
        for (int k = 0; k < 3; ++k) {
            dual w = dsub(dscale(lam[i], g[j][k]), dscale(lam[j], g[i][k]));   /* W1_ij = l_i gl_j - l_j gl_i */
            E[k] = dadd(E[k], dmul(cf, w));
        }
    }
    for (int f = 0; f < 4; ++f) {
        int i = LF[f][0], j = LF[f][1], kk = LF[f][2];
        int64_t id = m->tet_face[4 * T + f];
        double beta = F->b_env[2 * id] * c - F->b_env[2 * id + 1] * s + (F->b_dc ? F->b_dc[id] : 0.0);
        double jk[3], ki[3], ij[3];
        cross3(g[j], g[kk], jk); cross3(g[kk], g[i], ki); cross3(g[i], g[j], ij);
        for (int k = 0; k < 3; ++k) {
            dual w = dadd(dadd(dscale(lam[i], jk[k]), dscale(lam[j], ki[k])), dscale(lam[kk], ij[k]));
            B[k] = dadd(B[k], dscale(w, 2.0 * beta));
        }
    }
}

static void boris_dual(dual v[3], const dual E[3], const dual B[3], double h) {
    dual vm[3], tau[3], sig[3], cr[3], vpr[3];
    for (int k = 0; k < 3; ++k) { vm[k] = dadd(v[k], dscale(E[k], h)); tau[k] = dscale(B[k], h); }
    dual t2 = dadd(dadd(dmul(tau[0], tau[0]), dmul(tau[1], tau[1])), dmul(tau[2], tau[2]));
    dual den = dadd(dmk(1.0, 0.0), t2);
    for (int k = 0; k < 3; ++k) sig[k] = ddiv(dscale(tau[k], 2.0), den);
    dcross3(vm, tau, cr);
    for (int k = 0; k < 3; ++k) vpr[k] = dadd(vm[k], cr[k]);
    dcross3(vpr, sig, cr);
    for (int k = 0; k < 3; ++k) v[k] = dadd(dadd(vm[k], cr[k]), dscale(E[k], h));
}

/* one step of one particle in dual numbers (no deposit); returns the new tet
 * or -1 at the hop cap.  The same Cartesian walk as walk_path, with the point,
 * the displacement and the crossing parameter carried as duals. */
static int64_t step_one_dual(const ora_mesh *m, int64_t T, dual l[4], dual v[3], double c, double s,
                             const ora_fields_t *F, const double *de, double h, double dt) {
    dual E[3], B[3];
    fields_at_dual(m, T, l, c, s, F, de, E, B);
    boris_dual(v, E, B, h);
    dual d[3] = {dscale(v[0], dt), dscale(v[1], dt), dscale(v[2], dt)};
    double pn[4][3], pa[4][3], ph[4];   /* the face planes in float64 (value and derivative parts alike) */
    ora_plane pl[4];
#define LOAD_PLANES()                                                       \
    do {                                                                    \
        tet_planes(m, T, pl);                                               \
        for (int k_ = 0; k_ < 4; ++k_) {                                    \
            for (int c_ = 0; c_ < 3; ++c_) {                                \
                pn[k_][c_] = (double)pl[k_].n[c_];                          \
                pa[k_][c_] = (double)pl[k_].a[c_];                          \
            }                                                               \
            ph[k_] = (double)pl[k_].h;                                      \
        }                                                                   \
    } while (0)
    LOAD_PLANES();
    dual y[3] = {dmk(0.0, 0.0), dmk(0.0, 0.0), dmk(0.0, 0.0)};
    {
        const int32_t *vt = m->tv + 4 * T;
        const double *o = m->xyz + 3 * vt[0];
        for (int j = 1; j < 4; ++j)
            for (int k = 0; k < 3; ++k) y[k] = dadd(y[k], dscale(l[j], m->xyz[3 * vt[j] + k] - o[k]));
    }
    for (int hops = 0; hops <= ORA_HOP_CAP; ++hops) {
        dual sd = dmk(1.0, 0.0);
        int kmin = -1;
        for (int k = 0; k < 4; ++k) {
            dual ya[3] = {dsub(y[0], dmk(pa[k][0], 0.0)), dsub(y[1], dmk(pa[k][1], 0.0)), dsub(y[2], dmk(pa[k][2], 0.0))};
            dual dist = ddot3(ya, pn[k]), rate = ddot3(d, pn[k]);
            if (rate.v < 0.0 && dist.v + rate.v < 0.0) {
                dual sk = dist.v > 0.0 ? ddiv(dist, dscale(rate, -1.0)) : dmk(0.0, 0.0);
                if (kmin < 0 || sk.v < sd.v) { sd = sk; kmin = k; }
            }
        }
        dual dp[3] = {dmul(sd, d[0]), dmul(sd, d[1]), dmul(sd, d[2])};
        for (int k = 0; k < 4; ++k) l[k] = dadd(l[k], dscale(ddot3(dp, pn[k]), 1.0 / ph[k]));
        if (kmin < 0) return T;
        for (int k = 0; k < 3; ++k) { y[k] = dadd(y[k], dp[k]); d[k] = dsub(d[k], dp[k]); }
        int64_t nb = m->nbr[4 * T + kmin];
        if (nb < 0) {
            double nn = sqrt(dot3(pn[kmin], pn[kmin]));
            double nh[3] = {pn[kmin][0] / nn, pn[kmin][1] / nn, pn[kmin][2] / nn};
            dual dd = ddot3(d, nh), vv = ddot3(v, nh);
            for (int k = 0; k < 3; ++k) {
                d[k] = dsub(d[k], dscale(dd, 2.0 * nh[k]));
                v[k] = dsub(v[k], dscale(vv, 2.0 * nh[k]));
            }
        } else {
            const double *o = m->xyz + 3 * m->tv[4 * T], *on = m->xyz + 3 * m->tv[4 * nb];
            for (int k = 0; k < 3; ++k) y[k] = dadd(y[k], dmk(o[k] - on[k], 0.0));
            T = nb;
            LOAD_PLANES();
            for (int k = 0; k < 4; ++k) {
                dual ya[3] = {dsub(y[0], dmk(pa[k][0], 0.0)), dsub(y[1], dmk(pa[k][1], 0.0)),
                              dsub(y[2], dmk(pa[k][2], 0.0))};
                l[k] = dscale(ddot3(ya, pn[k]), 1.0 / ph[k]);
            }
        }
    }
#undef LOAD_PLANES
    return -1;
}

/* dv_out[3n] (and dx_out[3n] if not NULL): derivatives of the final velocity
 * and Cartesian position along de[2*ne] (re, im per edge).  Returns 0, or -6
 * if a particle reached the hop cap. */
int ora_jvp(const ora_mesh *m, int64_t n, const int32_t *tet0, const double *lam0, const double *vel0, double q,
            double mass, int64_t step0, int nsteps, double dt, double omega, const double *e_env,
            const double *e_dc, const double *b_env, const double *b_dc, const double *de, double *dv_out,
            double *dx_out, int nthreads) {
    ora_fields_t F = {e_env, e_dc, b_env, b_dc};
    double h = 0.5 * (q / mass) * dt;
    int status = 0;
    int nth = nthreads > 1 ? nthreads : 1;
#ifndef _OPENMP
    nth = 1;
#endif
    #pragma omp parallel for num_threads(nth) schedule(static) reduction(min:status)
    for (int64_t p = 0; p < n; ++p) {
        int64_t T = tet0[p];
        dual l[4], v[3];
        l[1] = dmk(lam0[3 * p], 0.0); l[2] = dmk(lam0[3 * p + 1], 0.0); l[3] = dmk(lam0[3 * p + 2], 0.0);
        l[0] = dmk(1.0 - l[1].v - l[2].v - l[3].v, 0.0);
        for (int k = 0; k < 3; ++k) v[k] = dmk(vel0[3 * p + k], 0.0);
        for (int k = 0; k < nsteps && T >= 0; ++k) {
            double t = (double)(step0 + k) * dt;
            T = step_one_dual(m, T, l, v, cos(omega * t), sin(omega * t), &F, de, h, dt);
        }
        if (T < 0) { status = -6; T = tet0[p]; }
        for (int k = 0; k < 3; ++k) dv_out[3 * p + k] = v[k].d;
        if (dx_out) {
            const int32_t *vt = m->tv + 4 * T;
            for (int c = 0; c < 3; ++c) {
                double acc = 0.0;
                for (int k = 0; k < 4; ++k) acc += l[k].d * m->xyz[3 * vt[k] + c];
                dx_out[3 * p + c] = acc;
            }
        }
    }
    return status;
}

/* ------------------------------------------------------------------------
 * Downshifted velocity integrator with Adams-Bashforth positions (Particle
 * Push section, the first of its two schemes: the fast carrier is treated
 * analytically inside the velocity update).  Over one particle step
 * [t_n, t_n + h] the slowly varying quantities along the trajectory -- the
 * envelope fields at the particle and the velocity -- are replaced by their
 * Lagrange interpolants N_k through the samples at t_n, t_{n-1}, t_{n-2}, and
 * the carrier is integrated exactly against them:
 *   v^{n+1} = v^n + q/m sum_k (Re E_k M^r_k + Im E_k M^i_k + Edc_k P_k)
 *           + q/m sum_{j,k} v^{n-j} x (Re B_k L^r_jk + Im B_k L^i_jk + Bdc_k Q_jk)
 * with M^r_k = int N_k cos(wt), M^i_k = -int N_k sin(wt), L^r_jk = int N_j N_k
 * cos(wt), L^i_jk = -int N_j N_k sin(wt) (the operators the section defines),
 * and P_k = int N_k, Q_jk = int N_j N_k for the unmodulated (dc) DoFs.
 * Positions advance with the fourth-order Adams-Bashforth stencil in the
 * velocities (eq. newtons); the path r^n -> r^{n+1} is walked and deposited as
 * in the fine-step scheme.  With hist < 3 previous steps the orders ramp up:
 * K = min(hist, 2) + 1 interpolation nodes, Adams-Bashforth order
 * min(hist, 3) + 1.
 * The weights are computed here by composite Gauss-Legendre quadrature.
 */

/* n-point Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_n). */
static void gauss_legendre(int n, double *x, double *w) {
    for (int i = 0; i < n; ++i) {
        double z = cos(acos(-1.0) * (i + 0.75) / (n + 0.5)), dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = 0.0;
            for (int k = 1; k <= n; ++k) {
                double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p2) / k;
            }
            dp = n * (z * p0 - p1) / (z * z - 1.0);
            double dz = p0 / dp;
            z -= dz;
            if (fabs(dz) < 1e-16) break;
        }
        x[i] = z;
        w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
    }
}

/* Lagrange polynomial of the nodes tau_i = -i h (i < K) that is 1 at tau_k. */
static double lagrange_node(int K, int k, double tau, double h) {
    double r = 1.0;
    for (int i = 0; i < K; ++i)
        if (i != k) r *= (tau + i * h) / ((double)(i - k) * h);
    return r;
}

/* Weights of one step [t0, t0 + h] with K nodes: Mr[K], Mi[K], P[K],
 * Lr[K*K], Li[K*K], Q[K*K] (row j, column k). */
void ora_ds_weights(int K, double t0, double h, double omega, double *Mr, double *Mi, double *P, double *Lr,
                    double *Li, double *Q) {
    enum { NG = 16, PANELS = 8 };
    double gx[NG], gw[NG];
    gauss_legendre(NG, gx, gw);
    for (int k = 0; k < K; ++k) Mr[k] = Mi[k] = P[k] = 0.0;
    for (int k = 0; k < K * K; ++k) Lr[k] = Li[k] = Q[k] = 0.0;
    const double ph = h / PANELS;
    for (int pn = 0; pn < PANELS; ++pn)
        for (int g = 0; g < NG; ++g) {
            double tau = ph * (pn + 0.5 * (gx[g] + 1.0)), wq = 0.5 * ph * gw[g];
            double c = cos(omega * (t0 + tau)), sn = sin(omega * (t0 + tau));
            double N[3];
            for (int k = 0; k < K; ++k) N[k] = lagrange_node(K, k, tau, h);
            for (int k = 0; k < K; ++k) {
                Mr[k] += wq * N[k] * c;
                Mi[k] -= wq * N[k] * sn;
                P[k] += wq * N[k];
                for (int j = 0; j < K; ++j) {
                    Lr[j * K + k] += wq * N[j] * N[k] * c;
                    Li[j * K + k] -= wq * N[j] * N[k] * sn;
                    Q[j * K + k] += wq * N[j] * N[k];
                }
            }
        }
}

/* Envelope samples at (T, lam): complex E~ = sum_e e~_e W1_e and B~ = sum_f
 * b~_f W2_f (edge by edge, face by face), and the dc parts. */
static void envelope_at(const ora_mesh *m, int64_t T, const double lam[4], const ora_fields_t *F, double Er[3],
                        double Ei[3], double Ed[3], double Br[3], double Bi[3], double Bd[3]) {
    double W1[6][3], W2[4][3];
    ora_whitney1(m, T, lam, W1);
    ora_whitney2(m, T, lam, W2);
    for (int k = 0; k < 3; ++k) Er[k] = Ei[k] = Ed[k] = Br[k] = Bi[k] = Bd[k] = 0.0;
    for (int e = 0; e < 6; ++e) {
        int64_t id = m->tet_edge[6 * T + e];
        for (int k = 0; k < 3; ++k) {
            Er[k] += F->e_env[2 * id] * W1[e][k];
            Ei[k] += F->e_env[2 * id + 1] * W1[e][k];
            if (F->e_dc) Ed[k] += F->e_dc[id] * W1[e][k];
        }
    }
    for (int f = 0; f < 4; ++f) {
        int64_t id = m->tet_face[4 * T + f];
        for (int k = 0; k < 3; ++k) {
            Br[k] += F->b_env[2 * id] * W2[f][k];
            Bi[k] += F->b_env[2 * id + 1] * W2[f][k];
            if (F->b_dc) Bd[k] += F->b_dc[id] * W2[f][k];
        }
    }
}

typedef struct {
    int K, A;
    double Mr[3], Mi[3], P[3], Lr[9], Li[9], Q[9];
    double ab[4];
} ds_weights_t;

/* One downshifted step of one particle.  vh[3][3] = v^{n-1}, v^{n-2}, v^{n-3};
 * es / bs [2][9] = the samples at t_{n-1}, t_{n-2}, each (Re[3], Im[3], dc[3]).
 * On return P->v = v^{n+1}, vh = v^n, v^{n-1}, v^{n-2} and es / bs = the
 * samples at t_n, t_{n-1} (the history of the next step). */
static void ds_step_one(const ora_mesh *m, ora_particle *P, double vh[3][3], double es[2][9], double bs[2][9],
                        const ds_weights_t *W, const ora_fields_t *F, double qm, double h, double qw, double *dG) {
    double Es[3][9], Bs[3][9], V[4][3];
    envelope_at(m, P->tet, P->lam, F, Es[0], Es[0] + 3, Es[0] + 6, Bs[0], Bs[0] + 3, Bs[0] + 6);
    for (int k = 1; k < 3; ++k)
        for (int i = 0; i < 9; ++i) { Es[k][i] = es[k - 1][i]; Bs[k][i] = bs[k - 1][i]; }
    for (int c = 0; c < 3; ++c) V[0][c] = P->v[c];
    for (int j = 1; j < 4; ++j)
        for (int c = 0; c < 3; ++c) V[j][c] = vh[j - 1][c];
    const int K = W->K;
    double acc[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < K; ++k)
        for (int c = 0; c < 3; ++c) acc[c] += Es[k][c] * W->Mr[k] + Es[k][3 + c] * W->Mi[k] + Es[k][6 + c] * W->P[k];
    for (int j = 0; j < K; ++j)
        for (int k = 0; k < K; ++k) {
            double Bw[3], cr[3];
            for (int c = 0; c < 3; ++c)
                Bw[c] = Bs[k][c] * W->Lr[j * K + k] + Bs[k][3 + c] * W->Li[j * K + k] + Bs[k][6 + c] * W->Q[j * K + k];
            cross3(V[j], Bw, cr);
            for (int c = 0; c < 3; ++c) acc[c] += cr[c];
        }
    double vnew[3];
    for (int c = 0; c < 3; ++c) vnew[c] = V[0][c] + qm * acc[c];
    /* Adams-Bashforth displacement in the velocities v^n, v^{n-1}, ... */
    double d[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < W->A; ++i)
        for (int c = 0; c < 3; ++c) d[c] += h * W->ab[i] * V[i][c];
    /* the velocities the next steps use are mirrored with v^{n+1} at a wall */
    double keep[3][3];
    for (int j = 0; j < 3; ++j)
        for (int c = 0; c < 3; ++c) keep[j][c] = V[j][c];
    for (int c = 0; c < 3; ++c) P->v[c] = vnew[c];
    walk_path(m, P, d, qw, dG, NULL, NULL, NULL, keep, 3);
    for (int j = 0; j < 3; ++j)
        for (int c = 0; c < 3; ++c) vh[j][c] = keep[j][c];
    for (int i = 0; i < 9; ++i) {
        es[1][i] = Es[1][i];
        bs[1][i] = Bs[1][i];
        es[0][i] = Es[0][i];
        bs[0][i] = Bs[0][i];
    }
}

static const double AB_COEF[4][4] = {{1.0, 0.0, 0.0, 0.0},
                                     {1.5, -0.5, 0.0, 0.0},
                                     {23.0 / 12.0, -16.0 / 12.0, 5.0 / 12.0, 0.0},
                                     {55.0 / 24.0, -59.0 / 24.0, 37.0 / 24.0, -9.0 / 24.0}};

/* One downshifted step for n particles at t = t_n with step h.  State in and
 * out: tet[n], lam[n*3], vel[n*3] (v^n in, v^{n+1} out), vhist[n*9]
 * (v^{n-1}, v^{n-2}, v^{n-3} in; v^n, v^{n-1}, v^{n-2} out), esamp / bsamp
 * [n*18] (samples at t_{n-1}, t_{n-2} in; at t_n, t_{n-1} out; each sample
 * Re[3], Im[3], dc[3]).  hist = number of downshifted steps taken before this
 * one (entries beyond it are not read).  dG / rho accumulate as in ora_step. */
int ora_ds_step(const ora_mesh *m, int64_t n, int32_t *tet, double *lam, double *vel, double *vhist, double *esamp,
                double *bsamp, int hist, double q, double mass, double w, double t, double h, double omega,
                const double *e_env, const double *e_dc, const double *b_env, const double *b_dc, double *dG,
                double *rho, int nthreads) {
    ora_fields_t F = {e_env, e_dc, b_env, b_dc};
    ds_weights_t W;
    W.K = (hist < 2 ? hist : 2) + 1;
    W.A = (hist < 3 ? hist : 3) + 1;
    ora_ds_weights(W.K, t, h, omega, W.Mr, W.Mi, W.P, W.Lr, W.Li, W.Q);
    for (int i = 0; i < 4; ++i) W.ab[i] = AB_COEF[W.A - 1][i];
    double qm = q / mass, qw = q * w;
    int status = 0;
    int nth = nthreads > 1 ? nthreads : 1;
#ifndef _OPENMP
    nth = 1;
#endif
    size_t stride = (size_t)m->ne + (rho ? m->nv : 0);
    double *priv = (double *)calloc((size_t)nth * stride, sizeof(double));
#ifdef _OPENMP
    #pragma omp parallel num_threads(nth) reduction(min:status)
#endif
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *mydG = priv + (size_t)tid * stride;
        double *myrho = rho ? mydG + m->ne : NULL;
#ifdef _OPENMP
        #pragma omp for schedule(static)
#endif
        for (int64_t p = 0; p < n; ++p) {
            ora_particle P;
            double vh[3][3], es[2][9], bs[2][9];
            P.tet = tet[p];
            P.lam[1] = lam[3 * p]; P.lam[2] = lam[3 * p + 1]; P.lam[3] = lam[3 * p + 2];
            P.lam[0] = 1.0 - P.lam[1] - P.lam[2] - P.lam[3];
            for (int c = 0; c < 3; ++c) P.v[c] = vel[3 * p + c];
            for (int j = 0; j < 3; ++j)
                for (int c = 0; c < 3; ++c) vh[j][c] = vhist[9 * p + 3 * j + c];
            for (int k = 0; k < 2; ++k)
                for (int i = 0; i < 9; ++i) { es[k][i] = esamp[18 * p + 9 * k + i]; bs[k][i] = bsamp[18 * p + 9 * k + i]; }
            ds_step_one(m, &P, vh, es, bs, &W, &F, qm, h, qw, mydG);
            tet[p] = (int32_t)P.tet;
            lam[3 * p] = P.lam[1]; lam[3 * p + 1] = P.lam[2]; lam[3 * p + 2] = P.lam[3];
            for (int c = 0; c < 3; ++c) vel[3 * p + c] = P.v[c];
            for (int j = 0; j < 3; ++j)
                for (int c = 0; c < 3; ++c) vhist[9 * p + 3 * j + c] = vh[j][c];
            for (int k = 0; k < 2; ++k)
                for (int i = 0; i < 9; ++i) { esamp[18 * p + 9 * k + i] = es[k][i]; bsamp[18 * p + 9 * k + i] = bs[k][i]; }
            if (P.status) status = P.status;
            if (myrho) {
                const int32_t *v = m->tv + 4 * P.tet;
                for (int k = 0; k < 4; ++k) myrho[v[k]] += qw * P.lam[k];
            }
        }
    }
    for (int th = 0; th < nth; ++th) {
        double *mydG = priv + (size_t)th * stride;
        for (int64_t e = 0; e < m->ne; ++e) dG[e] += mydG[e];
        if (rho) for (int64_t k = 0; k < m->nv; ++k) rho[k] += mydG[m->ne + k];
    }
    free(priv);
    return status;
}
