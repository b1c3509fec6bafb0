/* Exercise of the CPU oracle (oracle/oracle.c) built with AddressSanitizer and
 * UndefinedBehaviorSanitizer: mesh build, gather, Boris, walk and deposit of
 * many steps (including crossing-heavy and wall-hitting steps), vertex charge
 * and continuity residual, point location, the reverse and tangent-linear
 * derivatives and the downshifted step, on a small jittered Kuhn box made
 * here.  Exit status 0 when every call succeeds and continuity holds. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct ora_mesh ora_mesh;
int ora_mesh_build(int64_t nv, const double *xyz, int64_t nt, const int32_t *tv, ora_mesh **out);
void ora_mesh_free(ora_mesh *m);
void ora_mesh_counts(const ora_mesh *m, int64_t *out4);
int ora_step(const ora_mesh *m, int64_t n, int32_t *tet, double *lam, double *vel, double q, double mass, double w,
             int64_t step, double dt, double omega, const double *e_env, const double *e_dc, const double *b_env,
             const double *b_dc, double *dG, double *rho, int32_t *hops, int nthreads);
void ora_charge(const ora_mesh *m, int64_t n, const int32_t *tet, const double *lam, double q, double w, double *rho);
void ora_gauss(const ora_mesh *m, const double *dG, const double *rho_new, const double *rho_old, double *out);
int64_t ora_locate(const ora_mesh *m, const double *x, double *minlam);
void ora_point(const ora_mesh *m, int64_t T, const double lam[4], double *x);
int ora_vjp(const ora_mesh *m, int64_t n, const int32_t *tet0, const double *lam0, const double *vel0, double q,
            double mass, double w, int64_t step0, int nsteps, double dt, double omega, const double *e_env,
            const double *e_dc, const double *b_env, const double *b_dc, const double *vbar_in,
            const double *xbar_in, double *grad_e, double *vbar_out, double *xbar_out, int nthreads);
int ora_jvp(const ora_mesh *m, int64_t n, const int32_t *tet0, const double *lam0, const double *vel0, double q,
            double mass, int64_t step0, int nsteps, double dt, double omega, const double *e_env,
            const double *e_dc, const double *b_env, const double *b_dc, const double *de, double *dv_out,
            double *dx_out, int nthreads);
int ora_ds_step(const ora_mesh *m, int64_t n, int32_t *tet, double *lam, double *vel, double *vhist, double *esamp,
                double *bsamp, int hist, double q, double mass, double w, double t, double h, double omega,
                const double *e_env, const double *e_dc, const double *b_env, const double *b_dc, double *dG,
                double *rho, int nthreads);

static uint64_t state = 88172645463325252ull;
static double uniform(void) {
    state ^= state << 13;
    state ^= state >> 7;
    state ^= state << 17;
    return (double)(state >> 11) * (1.0 / 9007199254740992.0);
}
static double normal(void) {
    double u = uniform() + 1e-300, v = uniform();
    return sqrt(-2.0 * log(u)) * cos(6.283185307179586 * v);
}

static void swap32(int32_t *a, int32_t *b) { int32_t t = *a; *a = *b; *b = t; }

int main(void) {
    const int n[3] = {4, 3, 5};
    const int nx = n[0] + 1, ny = n[1] + 1, nz = n[2] + 1;
    const int64_t nv = (int64_t)nx * ny * nz, nt = 6LL * n[0] * n[1] * n[2];
    double *xyz = malloc(sizeof(double) * 3 * nv);
    int32_t *tv = malloc(sizeof(int32_t) * 4 * nt);
    for (int k = 0; k < nz; ++k)
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const int c[3] = {i, j, k};
                for (int d = 0; d < 3; ++d) {
                    double x = (double)c[d] / n[d];
                    if (c[d] > 0 && c[d] < n[d]) x += (uniform() - 0.5) * 0.2 / n[d];
                    xyz[3 * ((k * ny + j) * nx + i) + d] = x;
                }
            }
    static const int perms[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int64_t t = 0;
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i)
                for (int p = 0; p < 6; ++p, ++t) {
                    int c[3] = {i, j, k};
                    int32_t *v = tv + 4 * t;
                    v[0] = (c[2] * ny + c[1]) * nx + c[0];
                    for (int s = 0; s < 3; ++s) {
                        c[perms[p][s]] += 1;
                        v[s + 1] = (c[2] * ny + c[1]) * nx + c[0];
                    }
                    for (int a = 0; a < 4; ++a)
                        for (int b = a + 1; b < 4; ++b)
                            if (v[b] < v[a]) swap32(&v[a], &v[b]);
                }
    ora_mesh *m = NULL;
    if (ora_mesh_build(nv, xyz, nt, tv, &m) != 0) { fprintf(stderr, "mesh build failed\n"); return 1; }
    int64_t cnt[4];
    ora_mesh_counts(m, cnt);
    const int64_t ne = cnt[1], nf = cnt[2];
    double *e_env = malloc(sizeof(double) * 2 * ne), *b_env = malloc(sizeof(double) * 2 * nf);
    double *b_dc = malloc(sizeof(double) * nf), *e_dc = malloc(sizeof(double) * ne);
    for (int64_t e = 0; e < ne; ++e) { e_env[2 * e] = 1e-3 * normal(); e_env[2 * e + 1] = 1e-3 * normal(); e_dc[e] = 1e-3 * normal(); }
    for (int64_t f = 0; f < nf; ++f) { b_env[2 * f] = 1e-7 * normal(); b_env[2 * f + 1] = 1e-7 * normal(); b_dc[f] = 1e-3 * normal(); }
    const int64_t np = 400;
    int32_t *tet = malloc(sizeof(int32_t) * np), *hops = malloc(sizeof(int32_t) * np);
    double *lam = malloc(sizeof(double) * 3 * np), *vel = malloc(sizeof(double) * 3 * np);
    for (int64_t p = 0; p < np; ++p) {
        tet[p] = (int32_t)(uniform() * nt);
        double g[4], s = 0.0;
        for (int k = 0; k < 4; ++k) { g[k] = -log(uniform() + 1e-300); s += g[k]; }
        for (int k = 0; k < 3; ++k) lam[3 * p + k] = g[k + 1] / s;
        for (int k = 0; k < 3; ++k) vel[3 * p + k] = 1e5 * normal();
    }
    const double q = -1.602176634e-19, mass = 9.1093837015e-31;
    double *dG = calloc(ne, sizeof(double)), *rho0 = calloc(nv, sizeof(double)), *rho1 = calloc(nv, sizeof(double));
    int bad = 0;
    /* ordinary steps, then long steps that cross several tets and hit walls */
    for (int s = 0; s < 40; ++s) {
        const double dt = s < 20 ? 1e-11 : 5e-6;   /* 0.5 m at 1e5 m/s: several cells, walls hit */
        memset(dG, 0, sizeof(double) * ne);
        memset(rho0, 0, sizeof(double) * nv);
        memset(rho1, 0, sizeof(double) * nv);
        ora_charge(m, np, tet, lam, q, 1.0, rho0);
        if (ora_step(m, np, tet, lam, vel, q, mass, 1.0, s, dt, 6.283e9, e_env, e_dc, b_env, b_dc, dG, NULL, hops,
                     s % 2 ? 2 : 1) != 0) {
            fprintf(stderr, "step %d hit the hop cap\n", s);
            bad = 1;
        }
        ora_charge(m, np, tet, lam, q, 1.0, rho1);
        double out[2];
        ora_gauss(m, dG, rho1, rho0, out);
        if (!(out[0] <= 1e-13 * out[1])) { fprintf(stderr, "step %d continuity %g\n", s, out[0] / out[1]); bad = 1; }
    }
    for (int64_t p = 0; p < 20; ++p) {
        double l4[4] = {1.0 - lam[3 * p] - lam[3 * p + 1] - lam[3 * p + 2], lam[3 * p], lam[3 * p + 1], lam[3 * p + 2]};
        double x[3], ml;
        ora_point(m, tet[p], l4, x);
        int64_t T = ora_locate(m, x, &ml);
        if (T < 0 || ml < -1e-12) { fprintf(stderr, "locate failed for particle %lld\n", (long long)p); bad = 1; }
    }
    double *grad = calloc(2 * ne, sizeof(double)), *vb = malloc(sizeof(double) * 3 * np);
    double *vbo = malloc(sizeof(double) * 3 * np), *xbo = malloc(sizeof(double) * 3 * np);
    double *de = malloc(sizeof(double) * 2 * ne), *dv = malloc(sizeof(double) * 3 * np), *dx = malloc(sizeof(double) * 3 * np);
    for (int64_t i = 0; i < 3 * np; ++i) vb[i] = normal();
    for (int64_t i = 0; i < 2 * ne; ++i) de[i] = normal();
    if (ora_vjp(m, np, tet, lam, vel, q, mass, 1.0, 0, 5, 1e-9, 6.283e9, e_env, e_dc, b_env, b_dc, vb, NULL, grad, vbo,
                xbo, 2) != 0) bad = 1;
    if (ora_jvp(m, np, tet, lam, vel, q, mass, 0, 5, 1e-9, 6.283e9, e_env, e_dc, b_env, b_dc, de, dv, dx, 2) != 0) bad = 1;
    double *vh = calloc(9 * np, sizeof(double)), *es = calloc(18 * np, sizeof(double)), *bs = calloc(18 * np, sizeof(double));
    for (int h = 0; h < 6; ++h) {
        memset(dG, 0, sizeof(double) * ne);
        if (ora_ds_step(m, np, tet, lam, vel, vh, es, bs, h, q, mass, 1.0, h * 1e-10, 1e-10, 6.283e9, e_env, e_dc, b_env,
                        b_dc, dG, rho1, 1) != 0) bad = 1;
    }
    ora_mesh_free(m);
    free(xyz); free(tv); free(e_env); free(b_env); free(b_dc); free(e_dc); free(tet); free(hops); free(lam); free(vel);
    free(dG); free(rho0); free(rho1); free(grad); free(vb); free(vbo); free(xbo); free(de); free(dv); free(dx);
    free(vh); free(es); free(bs);
    if (bad) return 1;
    printf("oracle driver: all calls succeeded\n");
    return 0;
}
