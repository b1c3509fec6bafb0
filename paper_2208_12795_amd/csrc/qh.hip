// Quasi-Helmholtz projectors for gfx950 (Quasi Helmholtz or Coulomb gauge
// section, eqs. proj_es, proj_el, bfld_projector, efld_projected; operators
// of App. A).
//
//   P^Lambda_b = I - div^T (div div^T)^-1 div      on face DoFs,
//   P^Sigma_e  = Sigma (Sigma^T Sigma)^+ Sigma^T   on edge DoFs, Sigma = [*eps] D,
//   P^Lambda_e = I - P^Sigma_e,
//
// div the signed tet-face incidence (+1 where the face's global normal points
// out of the tet), D the node-edge incidence, [*eps] the Whitney edge mass.
// Both inverses are applied by conjugate gradients on complex vectors (the
// operators are real): div div^T = 4 I - (tet adjacency) matrix-free, and
// Sigma^T Sigma = D^T [*eps] [*eps] D as four passes (gradient, two edge
// mass products, divergence), Jacobi-preconditioned; it is singular (the
// constants), the right-hand side is orthogonal to them, and the mean of the
// result is removed, which gives the pseudoinverse's minimum-norm solution.
//
// The tree-cotree split of the edges and faces (etpic_tree_cotree, host
// only) selects the unknowns of the divergence-free fields.
//
// Every CG kernel runs on at most kQBlocks blocks (grid-stride loops) so that
// each block sums the previous kernel's block partials itself, in one fixed
// order: no scalar kernels, deterministic results.  The host launches 10
// iterations at a time; the device raises a done flag after which the rest of
// the batch returns at once.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <complex>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "etpic.h"
#include "field_host.hpp"
#include "mesh_host.hpp"

namespace {

thread_local std::string g_qh_error;

int qfail(int code, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_qh_error = buf;
    return code;
}

#define QH_TRY(expr)                                                                           \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return qfail(ETPIC_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr int kQThreads = 1024;
constexpr int kQBlocks = 512;
constexpr int kQRowLanes = 8;

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 cfma(double s, double2 a, double2 b) {   // s a + b
    return make_double2(fma(s, a.x, b.x), fma(s, a.y, b.y));
}
__device__ __forceinline__ double cdotr(double2 a, double2 b) { return a.x * b.x + a.y * b.y; }   // Re(conj(a) b)

// Block sum of 4 doubles into partial[blockIdx.x * 4 + k].
__device__ __forceinline__ void q_block_sum4(double v[4], double *partial) {
    __shared__ double sh[kQThreads / 64][4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < 4; ++k) sh[threadIdx.x >> 6][k] = v[k];
    __syncthreads();
    if (threadIdx.x < 4) {
        double t = 0.0;
        for (int w = 0; w < kQThreads / 64; ++w) t += sh[w][threadIdx.x];
        partial[blockIdx.x * 4 + threadIdx.x] = t;
    }
}

// Every thread gets the sums of the nb partials (fixed order).
__device__ __forceinline__ void q_all_sum4(int64_t nb, const double *__restrict__ partial, double tot[4]) {
    __shared__ double sh[kQThreads / 64][4];
    __shared__ double res[4];
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t b = threadIdx.x; b < nb; b += blockDim.x)
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] += partial[4 * b + k];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < 4; ++k) sh[threadIdx.x >> 6][k] = v[k];
    __syncthreads();
    if (threadIdx.x < 4) {
        double t = 0.0;
        for (int w = 0; w < kQThreads / 64; ++w) t += sh[w][threadIdx.x];
        res[threadIdx.x] = t;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) tot[k] = res[k];
}

// Scalars sc (written by thread 0 of block 0 only, read by later kernels):
// sc[0], sc[1] rho of even / odd iterations, sc[8] |r|^2, sc[9] |b|^2,
// sc[10] done flag, sc[11] iterations taken.
//
// Convergence test and scalar bookkeeping at the head of iteration k, from
// the partials [rho, -, |r|^2, |b|^2 (k = 0 only)] of the previous kernel.
// Returns beta (0 at k = 0); *stop is set when the iteration is over.
__device__ __forceinline__ double cg_head(double *__restrict__ sc, const double *__restrict__ pin, int64_t nb_in,
                                          int k, double tol2, bool &stop) {
    double tot[4];
    q_all_sum4(nb_in, pin, tot);
    const double b2 = k == 0 ? tot[3] : sc[9];
    const double r2 = tot[2], rn = tot[0];
    const bool done = b2 == 0.0 || !(r2 > tol2 * b2);
    const double ro = sc[(k + 1) & 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc[8] = r2;
        if (k == 0) sc[9] = b2;
        sc[k & 1] = rn;
        sc[10] = done ? 1.0 : 0.0;
        sc[11] = (double)k;
    }
    stop = done;
    return (k == 0 || ro == 0.0) ? 0.0 : rn / ro;
}

// beta of iteration k again (for a later kernel of the same iteration)
__device__ __forceinline__ double cg_beta(const double *__restrict__ sc, const double *__restrict__ pin, int64_t nb_in,
                                          int k) {
    double tot[4];
    q_all_sum4(nb_in, pin, tot);
    const double ro = sc[(k + 1) & 1];
    return (k == 0 || ro == 0.0) ? 0.0 : tot[0] / ro;
}

// ---------------------------------------------------------------- P^Lambda_b
// Per tet: the 4 face ids, the 4 neighbours (-1 at the wall) and the signs
// (bit k set: the global normal of face k points into the tet).
struct TetFaces {
    const int4 *f;
    const int4 *n;
    const uint8_t *neg;
};

// s = div b; x = 0, r = s, p = q = 0; partials |r|^2, 0, |r|^2, |s|^2 (no
// preconditioner: the diagonal of div div^T is 4 everywhere).
__global__ void __launch_bounds__(kQThreads) k_qb_start(int64_t nt, TetFaces T, const double2 *__restrict__ b,
                                                        double2 *__restrict__ x, double2 *__restrict__ r,
                                                        double2 *__restrict__ p, double2 *__restrict__ q,
                                                        double *__restrict__ partial, double *__restrict__ sc) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += (int64_t)gridDim.x * blockDim.x) {
        const int4 f = T.f[t];
        const unsigned ng = T.neg[t];
        const int fk[4] = {f.x, f.y, f.z, f.w};
        double2 s = make_double2(0.0, 0.0);
#pragma unroll
        for (int k = 0; k < 4; ++k) s = ((ng >> k) & 1u) ? csub(s, b[fk[k]]) : cadd(s, b[fk[k]]);
        x[t] = make_double2(0.0, 0.0);
        r[t] = s;
        p[t] = make_double2(0.0, 0.0);
        q[t] = make_double2(0.0, 0.0);
        const double s2 = cdotr(s, s);
        v[0] += s2;
        v[2] += s2;
        v[3] += s2;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc[10] = 0.0;
        sc[11] = 0.0;
    }
    q_block_sum4(v, partial);
}

// Iteration k, first half: p = r + beta p, q = A p = A r + beta q with
// A = div div^T = 4 I - adjacency; partials of p . q.
__global__ void __launch_bounds__(kQThreads) k_qb_apply(int64_t nt, TetFaces T, double *__restrict__ sc,
                                                        const double2 *__restrict__ r, double2 *__restrict__ p,
                                                        double2 *__restrict__ q, const double *__restrict__ pin,
                                                        int64_t nb_in, double *__restrict__ pout, int k, double tol2,
                                                        int check_only) {
    if (sc[10] != 0.0) return;
    bool stop;
    const double be = cg_head(sc, pin, nb_in, k, tol2, stop);
    if (stop || check_only) return;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += (int64_t)gridDim.x * blockDim.x) {
        const int4 n = T.n[t];
        const int nk[4] = {n.x, n.y, n.z, n.w};
        const double2 rt = r[t];
        double2 ar = cscale(rt, 4.0);
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (nk[j] >= 0) ar = csub(ar, r[nk[j]]);
        const double2 pn = k == 0 ? rt : cfma(be, p[t], rt);
        const double2 qn = k == 0 ? ar : cfma(be, q[t], ar);
        p[t] = pn;
        q[t] = qn;
        v[0] += cdotr(pn, qn);
    }
    q_block_sum4(v, pout);
}

// Iteration k, second half: alpha = rho / (p . q); x += alpha p, r -= alpha q;
// partials |r|^2, 0, |r|^2, 0.
__global__ void __launch_bounds__(kQThreads) k_qb_update(int64_t nt, const double *__restrict__ sc,
                                                         const double2 *__restrict__ p, const double2 *__restrict__ q,
                                                         double2 *__restrict__ x, double2 *__restrict__ r,
                                                         const double *__restrict__ pin, int64_t nb_in,
                                                         double *__restrict__ pout, int k) {
    if (sc[10] != 0.0) return;
    double tot[4];
    q_all_sum4(nb_in, pin, tot);
    const double al = tot[0] != 0.0 ? sc[k & 1] / tot[0] : 0.0;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += (int64_t)gridDim.x * blockDim.x) {
        x[t] = cfma(al, p[t], x[t]);
        const double2 rt = cfma(-al, q[t], r[t]);
        r[t] = rt;
        const double r2 = cdotr(rt, rt);
        v[0] += r2;
        v[2] += r2;
    }
    q_block_sum4(v, pout);
}

// out_f = b_f - (div^T x)_f: the face's one or two tets with their signs
// (ft[2f + i] = tet or -1; bit i of fneg[f] set: the face's normal points
// into tet i).
__global__ void __launch_bounds__(kQThreads) k_qb_out(int64_t nf, const int2 *__restrict__ ft,
                                                      const uint8_t *__restrict__ fneg, const double2 *__restrict__ x,
                                                      const double2 *__restrict__ b, double2 *__restrict__ out) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    const int2 t = ft[f];
    const unsigned ng = fneg[f];
    double2 o = b[f];
    if (t.x >= 0) o = (ng & 1u) ? cadd(o, x[t.x]) : csub(o, x[t.x]);
    if (t.y >= 0) o = (ng & 2u) ? cadd(o, x[t.y]) : csub(o, x[t.y]);
    out[f] = o;
}

// ---------------------------------------------------------------- P^Sigma_e
struct EdgeCsr {
    int64_t ne;
    const int32_t *rowptr, *col;
    const double *M;
};

// y = [*eps] x (complex x, y), kQRowLanes lanes per row; skipped once the
// iteration is done (sc NULL: always runs).
__global__ void __launch_bounds__(kQThreads) k_qe_mass(EdgeCsr S, const double *__restrict__ sc,
                                                       const double2 *__restrict__ x, double2 *__restrict__ y) {
    if (sc && sc[10] != 0.0) return;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t / kQRowLanes < S.ne; t += stride) {
        const int64_t row = t / kQRowLanes;
        const int sub = (int)(t % kQRowLanes);
        double2 acc = make_double2(0.0, 0.0);
        for (int32_t j = S.rowptr[row] + sub; j < S.rowptr[row + 1]; j += kQRowLanes) {
            const double m = S.M[j];
            const double2 a = x[S.col[j]];
            acc.x = fma(m, a.x, acc.x);
            acc.y = fma(m, a.y, acc.y);
        }
#pragma unroll
        for (int off = kQRowLanes / 2; off > 0; off >>= 1) {
            acc.x += __shfl_xor(acc.x, off);
            acc.y += __shfl_xor(acc.y, off);
        }
        if (sub == 0) y[row] = acc;
    }
}

// (D^T w)_i: sum of +-w over the edges at node i (+ where i is the head)
__device__ __forceinline__ double2 node_div(int64_t i, const int32_t *__restrict__ ptr, const int32_t *__restrict__ code,
                                            const double2 *__restrict__ w) {
    double2 s = make_double2(0.0, 0.0);
    for (int32_t k = ptr[i]; k < ptr[i + 1]; ++k) {
        const int32_t c = code[k];
        s = (c & 1) ? cadd(s, w[c >> 1]) : csub(s, w[c >> 1]);
    }
    return s;
}

// rhs = Sigma^T d = D^T ([*eps] d) from w = [*eps] d; x = 0, r = rhs,
// z = Dinv r, p = q = 0; partials r.z, 0, |r|^2, |rhs|^2.
__global__ void __launch_bounds__(kQThreads) k_qe_start(int64_t nv, const int32_t *__restrict__ ptr,
                                                        const int32_t *__restrict__ code, const double2 *__restrict__ w,
                                                        const double *__restrict__ dinv, double2 *__restrict__ x,
                                                        double2 *__restrict__ r, double2 *__restrict__ z,
                                                        double2 *__restrict__ p, double2 *__restrict__ q,
                                                        double *__restrict__ partial, double *__restrict__ sc) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x) {
        const double2 b = node_div(i, ptr, code, w);
        const double2 zi = cscale(b, dinv[i]);
        x[i] = make_double2(0.0, 0.0);
        r[i] = b;
        z[i] = zi;
        p[i] = make_double2(0.0, 0.0);
        q[i] = make_double2(0.0, 0.0);
        v[0] += cdotr(b, zi);
        v[2] += cdotr(b, b);
        v[3] += cdotr(b, b);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc[10] = 0.0;
        sc[11] = 0.0;
    }
    q_block_sum4(v, partial);
}

// Iteration k, pass 1: convergence test; t1 = D p = D z + beta t1 (edge e
// from ev[2e] to ev[2e+1]).
__global__ void __launch_bounds__(kQThreads) k_qe_grad(int64_t ne, const int32_t *__restrict__ ev,
                                                       double *__restrict__ sc, const double2 *__restrict__ z,
                                                       double2 *__restrict__ t1, const double *__restrict__ pin,
                                                       int64_t nb_in, int k, double tol2, int check_only) {
    if (sc[10] != 0.0) return;
    bool stop;
    const double be = cg_head(sc, pin, nb_in, k, tol2, stop);
    if (stop || check_only) return;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
        const double2 dz = csub(z[ev[2 * e + 1]], z[ev[2 * e]]);
        t1[e] = k == 0 ? dz : cfma(be, t1[e], dz);
    }
}

// Iteration k, pass 4 (after t3 = [*eps] [*eps] t1): p = z + beta p,
// q = D^T t3; partials of p . q.
__global__ void __launch_bounds__(kQThreads) k_qe_divq(int64_t nv, const int32_t *__restrict__ ptr,
                                                       const int32_t *__restrict__ code, const double *__restrict__ sc,
                                                       const double2 *__restrict__ z, double2 *__restrict__ p,
                                                       double2 *__restrict__ q, const double2 *__restrict__ t3,
                                                       const double *__restrict__ pin, int64_t nb_in,
                                                       double *__restrict__ pout, int k) {
    if (sc[10] != 0.0) return;
    const double be = cg_beta(sc, pin, nb_in, k);
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x) {
        const double2 pn = k == 0 ? z[i] : cfma(be, p[i], z[i]);
        const double2 qn = node_div(i, ptr, code, t3);
        p[i] = pn;
        q[i] = qn;
        v[0] += cdotr(pn, qn);
    }
    q_block_sum4(v, pout);
}

// Iteration k, pass 5: alpha = rho / (p . q); x += alpha p, r -= alpha q,
// z = Dinv r; partials r.z, 0, |r|^2, 0.
__global__ void __launch_bounds__(kQThreads) k_qe_update(int64_t nv, const double *__restrict__ sc,
                                                         const double *__restrict__ dinv, const double2 *__restrict__ p,
                                                         const double2 *__restrict__ q, double2 *__restrict__ x,
                                                         double2 *__restrict__ r, double2 *__restrict__ z,
                                                         const double *__restrict__ pin, int64_t nb_in,
                                                         double *__restrict__ pout, int k) {
    if (sc[10] != 0.0) return;
    double tot[4];
    q_all_sum4(nb_in, pin, tot);
    const double al = tot[0] != 0.0 ? sc[k & 1] / tot[0] : 0.0;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] = cfma(al, p[i], x[i]);
        const double2 ri = cfma(-al, q[i], r[i]);
        r[i] = ri;
        const double2 zi = cscale(ri, dinv[i]);
        z[i] = zi;
        v[0] += cdotr(ri, zi);
        v[2] += cdotr(ri, ri);
    }
    q_block_sum4(v, pout);
}

// partials of the sum of x (re, im)
__global__ void __launch_bounds__(kQThreads) k_qe_sum(int64_t nv, const double2 *__restrict__ x,
                                                      double *__restrict__ partial) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x) {
        const double2 a = x[i];
        v[0] += a.x;
        v[1] += a.y;
    }
    q_block_sum4(v, partial);
}

// x -= mean(x) (the minimum-norm solution), copied to x_out if not NULL
__global__ void __launch_bounds__(kQThreads) k_qe_center(int64_t nv, double2 *__restrict__ x,
                                                         const double *__restrict__ pin, int64_t nb_in,
                                                         double2 *__restrict__ x_out) {
    double tot[4];
    q_all_sum4(nb_in, pin, tot);
    const double2 mean = make_double2(tot[0] / (double)nv, tot[1] / (double)nv);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x) {
        const double2 a = csub(x[i], mean);
        x[i] = a;
        if (x_out) x_out[i] = a;
    }
}

// t1 = D x
__global__ void __launch_bounds__(kQThreads) k_qe_dx(int64_t ne, const int32_t *__restrict__ ev,
                                                     const double2 *__restrict__ x, double2 *__restrict__ t1) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e < ne) t1[e] = csub(x[ev[2 * e + 1]], x[ev[2 * e]]);
}

// d_sigma = s, d_lambda = d - s (either output may be NULL)
__global__ void __launch_bounds__(kQThreads) k_qe_split(int64_t ne, const double2 *__restrict__ d,
                                                        const double2 *__restrict__ s, double2 *__restrict__ d_sigma,
                                                        double2 *__restrict__ d_lambda) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    const double2 se = s[e];
    if (d_sigma) d_sigma[e] = se;
    if (d_lambda) d_lambda[e] = csub(d[e], se);
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kQThreads - 1) / kQThreads); }
inline unsigned cg_blocks(int64_t n) { return (unsigned)std::min<int64_t>(blocks_for(n), kQBlocks); }

}  // namespace

struct etpic_qh {
    int device = 0;
    int64_t nv = 0, ne = 0, nf = 0, nt = 0, nnz = 0;
    // P^Lambda_b
    int4 *tf = nullptr, *tn = nullptr;
    uint8_t *tneg = nullptr;
    int2 *ft = nullptr;
    uint8_t *fneg = nullptr;
    double2 *tv = nullptr;     // 4 complex tet vectors: x, r, p, q
    // P^Sigma_e
    int32_t *rowptr = nullptr, *col = nullptr, *ev = nullptr, *v2e_ptr = nullptr, *v2e_code = nullptr;
    double *M = nullptr, *dinv = nullptr;
    double2 *nvec = nullptr;   // 5 complex node vectors: x, r, z, p, q
    double2 *evec = nullptr;   // 3 complex edge vectors: t1, t2, t3
    double *partial = nullptr; // two sets of 4 per block
    double *sc = nullptr;      // 12 scalars
    bool bound = false;        // device part in the caller's buffer (etpic_qh_bind)
    // the host tables the device part is filled from
    std::vector<int4> h_tf, h_tn;
    std::vector<uint8_t> h_tneg, h_fneg;
    std::vector<int2> h_ft;
    std::vector<int32_t> h_rowptr, h_col, h_ev, h_v2e_ptr, h_v2e_code;
    std::vector<double> h_M, h_dinv;

    TetFaces tet_faces() const { return TetFaces{tf, tn, tneg}; }
    EdgeCsr csr() const { return EdgeCsr{ne, rowptr, col, M}; }
};

namespace {

// Arrays carved from the caller's buffer in a fixed order, each on a 256-byte
// boundary (a null base only counts the bytes).
struct QhCarve {
    char *base = nullptr;
    size_t used = 0;
    template <typename T>
    T *take(size_t count) {
        const size_t off = (used + 255) & ~(size_t)255;
        used = off + sizeof(T) * std::max<size_t>(count, 1);
        return base ? reinterpret_cast<T *>(base + off) : nullptr;
    }
};

// The device part of the object: the host tables' copies, then the work
// vectors, partials and scalars.
struct QhPtrs {
    int4 *tf, *tn;
    uint8_t *tneg, *fneg;
    int2 *ft;
    int32_t *rowptr, *col, *ev, *v2e_ptr, *v2e_code;
    double *M, *dinv, *partial, *sc;
    double2 *tv, *nvec, *evec;
};
QhPtrs qh_layout(const etpic_qh *Q, QhCarve &cv) {
    QhPtrs d;
    d.tf = cv.take<int4>(Q->h_tf.size());
    d.tn = cv.take<int4>(Q->h_tn.size());
    d.tneg = cv.take<uint8_t>(Q->h_tneg.size());
    d.ft = cv.take<int2>(Q->h_ft.size());
    d.fneg = cv.take<uint8_t>(Q->h_fneg.size());
    d.rowptr = cv.take<int32_t>(Q->h_rowptr.size());
    d.col = cv.take<int32_t>(Q->h_col.size());
    d.M = cv.take<double>(Q->h_M.size());
    d.ev = cv.take<int32_t>(Q->h_ev.size());
    d.v2e_ptr = cv.take<int32_t>(Q->h_v2e_ptr.size());
    d.v2e_code = cv.take<int32_t>(Q->h_v2e_code.size());
    d.dinv = cv.take<double>(Q->h_dinv.size());
    d.tv = cv.take<double2>(4 * Q->nt);
    d.nvec = cv.take<double2>(5 * Q->nv);
    d.evec = cv.take<double2>(3 * Q->ne);
    d.partial = cv.take<double>(8 * kQBlocks);
    d.sc = cv.take<double>(12);
    return d;
}

template <typename T>
int upload(T *dst, const std::vector<T> &src) {
    if (!src.empty()) QH_TRY(hipMemcpy(dst, src.data(), sizeof(T) * src.size(), hipMemcpyHostToDevice));
    return ETPIC_OK;
}

int qh_build(etpic_qh *Q, int64_t nv, const double *xyz, int64_t nt, const int32_t *tet_vert, double eps) {
    std::string err;
    etpic::HostMesh H;
    if (int r = etpic::build_host_mesh(nv, xyz, nt, tet_vert, H, err)) return qfail(r == -4 ? ETPIC_EMESH : ETPIC_EINVAL,
                                                                                    "qh mesh: %s", err.c_str());
    {   // connected vertex graph: the constants are then the only null space of Sigma^T Sigma
        std::vector<uint8_t> seen((size_t)H.nv, 0);
        std::vector<int32_t> queue(1, 0);
        seen[0] = 1;
        for (size_t h = 0; h < queue.size(); ++h)
            for (int32_t k = H.v2e_ptr[queue[h]]; k < H.v2e_ptr[queue[h] + 1]; ++k) {
                const int32_t e = H.v2e_code[k] >> 1;
                for (int32_t w : {H.edges[2 * e], H.edges[2 * e + 1]})
                    if (!seen[w]) {
                        seen[w] = 1;
                        queue.push_back(w);
                    }
            }
        if ((int64_t)queue.size() != H.nv)
            return qfail(ETPIC_EMESH, "qh mesh: not connected (%zu of %lld vertices reachable)", queue.size(),
                         (long long)H.nv);
    }
    Q->nv = H.nv;
    Q->ne = H.ne;
    Q->nf = H.nf;
    Q->nt = H.nt;
    // tet faces, neighbours and face signs; face -> tets
    std::vector<int4> tf((size_t)nt), tn((size_t)nt);
    std::vector<uint8_t> tneg((size_t)nt, 0);
    std::vector<int2> ft((size_t)H.nf, make_int2(-1, -1));
    std::vector<uint8_t> fneg((size_t)H.nf, 0);
    for (int64_t t = 0; t < nt; ++t) {
        const etpic::TetTopo &tp = H.topo[t];
        tf[t] = make_int4(tp.f[0], tp.f[1], tp.f[2], tp.f[3]);
        tn[t] = make_int4(tp.n[0], tp.n[1], tp.n[2], tp.n[3]);
        for (int k = 0; k < 4; ++k) {
            const int32_t f = tp.f[k];
            const double *a = xyz + 3 * H.faces[3 * f], *b = xyz + 3 * H.faces[3 * f + 1],
                         *c = xyz + 3 * H.faces[3 * f + 2], *o = xyz + 3 * tp.v[k];
            const double u[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
            const double w[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
            const double n[3] = {u[1] * w[2] - u[2] * w[1], u[2] * w[0] - u[0] * w[2], u[0] * w[1] - u[1] * w[0]};
            const double out = n[0] * (a[0] - o[0]) + n[1] * (a[1] - o[1]) + n[2] * (a[2] - o[2]);
            const bool neg = !(out > 0.0);
            if (neg) tneg[t] |= (uint8_t)(1u << k);
            int2 &slot = ft[f];
            if (slot.x < 0) {
                slot.x = (int32_t)t;
                if (neg) fneg[f] |= 1u;
            } else if (slot.y < 0) {
                slot.y = (int32_t)t;
                if (neg) fneg[f] |= 2u;
            } else {
                return qfail(ETPIC_EMESH, "qh mesh: face %d in more than two tets", f);
            }
        }
    }
    // full edge mass (no boundary rows replaced)
    etpic::FieldSystem S;
    if (etpic::build_field_system(H, eps, 1.0, S, err, false)) return qfail(ETPIC_EINVAL, "qh: %s", err.c_str());
    Q->nnz = S.nnz;
    // Jacobi: diag(Sigma^T Sigma)_i = |[*eps] D e_i|^2, column i of D = +-1 at the edges of node i
    std::vector<double> dinv((size_t)H.nv, 0.0), acc((size_t)H.ne, 0.0);
    std::vector<int32_t> touched;
    std::vector<uint8_t> mark((size_t)H.ne, 0);
    for (int64_t i = 0; i < H.nv; ++i) {
        touched.clear();
        for (int32_t k = H.v2e_ptr[i]; k < H.v2e_ptr[i + 1]; ++k) {
            const int32_t code = H.v2e_code[k], e = code >> 1;
            const double sgn = (code & 1) ? 1.0 : -1.0;
            for (int32_t j = S.rowptr[e]; j < S.rowptr[e + 1]; ++j) {   // [*eps] is symmetric: row e = column e
                const int32_t c = S.col[j];
                if (!mark[c]) {
                    mark[c] = 1;
                    touched.push_back(c);
                }
                acc[c] += sgn * S.M[j];
            }
        }
        double d = 0.0;
        for (int32_t c : touched) {
            d += acc[c] * acc[c];
            acc[c] = 0.0;
            mark[c] = 0;
        }
        if (!(d > 0.0)) return qfail(ETPIC_EMESH, "qh: node %lld has no edge", (long long)i);
        dinv[i] = 1.0 / d;
    }
    int count = 0;
    QH_TRY(hipGetDeviceCount(&count));
    if (Q->device < 0 || Q->device >= count)
        return qfail(ETPIC_EINVAL, "device %d not present (%d devices)", Q->device, count);
    Q->h_tf = std::move(tf);
    Q->h_tn = std::move(tn);
    Q->h_tneg = std::move(tneg);
    Q->h_ft = std::move(ft);
    Q->h_fneg = std::move(fneg);
    Q->h_rowptr = std::move(S.rowptr);
    Q->h_col = std::move(S.col);
    Q->h_M = std::move(S.M);
    Q->h_ev = std::move(H.edges);
    Q->h_v2e_ptr = std::move(H.v2e_ptr);
    Q->h_v2e_code = std::move(H.v2e_code);
    Q->h_dinv = std::move(dinv);
    return ETPIC_OK;
}

// Reads the scalars after a batch; true when the loop is over.
int read_scalars(const etpic_qh *Q, hipStream_t st, double hs[12]) {
    QH_TRY(hipMemcpyAsync(hs, Q->sc, sizeof(double) * 12, hipMemcpyDeviceToHost, st));
    QH_TRY(hipStreamSynchronize(st));
    return ETPIC_OK;
}

int finish(const double hs[12], double tol, int *iters_out, double *resid_out) {
    const double b2 = hs[9];
    const double rel = b2 > 0.0 ? std::sqrt(hs[8] / b2) : 0.0;
    const int it = (int)hs[11];
    if (iters_out) *iters_out = it;
    if (resid_out) *resid_out = rel;
    if (hs[10] == 0.0 || !std::isfinite(rel))
        return qfail(ETPIC_ENOCONV, "qh CG: relative residual %.3e after %d iterations (tol %.1e)", rel, it, tol);
    return ETPIC_OK;
}

}  // namespace

extern "C" {

const char *etpic_qh_last_error(void) { return g_qh_error.c_str(); }

int etpic_qh_create(etpic_qh **out, int device, int64_t nv, const double *xyz, int64_t nt, const int32_t *tet_vert,
                    double eps) {
    if (!out) return qfail(ETPIC_EINVAL, "null output handle");
    *out = nullptr;
    if (!(eps > 0.0) || !std::isfinite(eps)) return qfail(ETPIC_EINVAL, "eps must be positive");
    etpic_qh *Q = new etpic_qh();
    Q->device = device;
    if (int r = qh_build(Q, nv, xyz, nt, tet_vert, eps)) {
        delete Q;
        return r;
    }
    *out = Q;
    return ETPIC_OK;
}

int etpic_qh_bytes(const etpic_qh *qh, size_t *bytes) {
    if (!qh || !bytes) return qfail(ETPIC_EINVAL, "null argument");
    QhCarve cv;
    (void)qh_layout(qh, cv);
    *bytes = cv.used;
    return ETPIC_OK;
}

int etpic_qh_bind(etpic_qh *qh, void *dev_buf, size_t bytes) {
    if (!qh || !dev_buf) return qfail(ETPIC_EINVAL, "null argument");
    if (reinterpret_cast<uintptr_t>(dev_buf) & 255u) return qfail(ETPIC_EINVAL, "buffer not 256-byte aligned");
    size_t need = 0;
    if (int r = etpic_qh_bytes(qh, &need)) return r;
    if (bytes < need) return qfail(ETPIC_EINVAL, "buffer of %zu bytes, %zu needed", bytes, need);
    QH_TRY(hipSetDevice(qh->device));
    QH_TRY(hipDeviceSynchronize());
    QhCarve cv;
    cv.base = static_cast<char *>(dev_buf);
    const QhPtrs d = qh_layout(qh, cv);
    qh->tf = d.tf;
    qh->tn = d.tn;
    qh->tneg = d.tneg;
    qh->fneg = d.fneg;
    qh->ft = d.ft;
    qh->rowptr = d.rowptr;
    qh->col = d.col;
    qh->ev = d.ev;
    qh->v2e_ptr = d.v2e_ptr;
    qh->v2e_code = d.v2e_code;
    qh->M = d.M;
    qh->dinv = d.dinv;
    qh->partial = d.partial;
    qh->sc = d.sc;
    qh->tv = d.tv;
    qh->nvec = d.nvec;
    qh->evec = d.evec;
    if (int r = upload(qh->tf, qh->h_tf)) return r;
    if (int r = upload(qh->tn, qh->h_tn)) return r;
    if (int r = upload(qh->tneg, qh->h_tneg)) return r;
    if (int r = upload(qh->ft, qh->h_ft)) return r;
    if (int r = upload(qh->fneg, qh->h_fneg)) return r;
    if (int r = upload(qh->rowptr, qh->h_rowptr)) return r;
    if (int r = upload(qh->col, qh->h_col)) return r;
    if (int r = upload(qh->M, qh->h_M)) return r;
    if (int r = upload(qh->ev, qh->h_ev)) return r;
    if (int r = upload(qh->v2e_ptr, qh->h_v2e_ptr)) return r;
    if (int r = upload(qh->v2e_code, qh->h_v2e_code)) return r;
    if (int r = upload(qh->dinv, qh->h_dinv)) return r;
    QH_TRY(hipMemset(qh->sc, 0, sizeof(double) * 12));
    QH_TRY(hipDeviceSynchronize());
    qh->bound = true;
    return ETPIC_OK;
}

void etpic_qh_destroy(etpic_qh *qh) {
    if (!qh) return;
    (void)hipSetDevice(qh->device);
    (void)hipDeviceSynchronize();
    delete qh;
}

int etpic_qh_counts(const etpic_qh *qh, int64_t counts_out[5]) {
    if (!qh || !counts_out) return qfail(ETPIC_EINVAL, "null argument");
    counts_out[0] = qh->nv;
    counts_out[1] = qh->ne;
    counts_out[2] = qh->nf;
    counts_out[3] = qh->nt;
    counts_out[4] = qh->nnz;
    return ETPIC_OK;
}

int etpic_qh_project_b(etpic_qh *qh, const double *b, double *b_out, double tol, int max_iter, int *iters_out,
                       double *resid_out, void *stream) {
    if (!qh || !b || !b_out) return qfail(ETPIC_EINVAL, "null argument");
    if (!qh->bound) return qfail(ETPIC_ESTATE, "no device buffer bound (etpic_qh_bytes, etpic_qh_bind)");
    if (!(tol > 0.0) || max_iter < 1) return qfail(ETPIC_EINVAL, "bad tol / max_iter");
    QH_TRY(hipSetDevice(qh->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t nt = qh->nt;
    const unsigned g = cg_blocks(nt);
    double2 *x = qh->tv, *r = qh->tv + nt, *p = qh->tv + 2 * nt, *q = qh->tv + 3 * nt;
    double *pa = qh->partial, *pb = qh->partial + 4 * kQBlocks;
    const double2 *B = reinterpret_cast<const double2 *>(b);
    k_qb_start<<<g, kQThreads, 0, st>>>(nt, qh->tet_faces(), B, x, r, p, q, pb, qh->sc);
    QH_TRY(hipGetLastError());
    const double tol2 = tol * tol;
    double hs[12];
    int k = 0;
    for (;;) {
        const int n = std::min(10, max_iter - k);
        for (int j = 0; j < n; ++j, ++k) {
            k_qb_apply<<<g, kQThreads, 0, st>>>(nt, qh->tet_faces(), qh->sc, r, p, q, pb, g, pa, k, tol2, 0);
            k_qb_update<<<g, kQThreads, 0, st>>>(nt, qh->sc, p, q, x, r, pa, g, pb, k);
        }
        if (k >= max_iter) k_qb_apply<<<g, kQThreads, 0, st>>>(nt, qh->tet_faces(), qh->sc, r, p, q, pb, g, pa, k, tol2, 1);
        QH_TRY(hipGetLastError());
        if (int rr = read_scalars(qh, st, hs)) return rr;
        if (hs[10] != 0.0 || k >= max_iter) break;
    }
    if (int rr = finish(hs, tol, iters_out, resid_out)) return rr;
    k_qb_out<<<blocks_for(qh->nf), kQThreads, 0, st>>>(qh->nf, qh->ft, qh->fneg, x, B, reinterpret_cast<double2 *>(b_out));
    QH_TRY(hipGetLastError());
    return ETPIC_OK;
}

int etpic_qh_project_e(etpic_qh *qh, const double *d, double *d_sigma, double *d_lambda, double *e_ns, double tol,
                       int max_iter, int *iters_out, double *resid_out, void *stream) {
    if (!qh || !d) return qfail(ETPIC_EINVAL, "null argument");
    if (!qh->bound) return qfail(ETPIC_ESTATE, "no device buffer bound (etpic_qh_bytes, etpic_qh_bind)");
    if (!d_sigma && !d_lambda && !e_ns) return qfail(ETPIC_EINVAL, "no output requested");
    if (d_sigma == d || d_lambda == d || (d_sigma && d_sigma == d_lambda))
        return qfail(ETPIC_EINVAL, "outputs alias the input or each other");
    if (!(tol > 0.0) || max_iter < 1) return qfail(ETPIC_EINVAL, "bad tol / max_iter");
    QH_TRY(hipSetDevice(qh->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t nv = qh->nv, ne = qh->ne;
    const unsigned gv = cg_blocks(nv), ge = cg_blocks(ne), gm = cg_blocks(ne * kQRowLanes);
    double2 *x = qh->nvec, *r = x + nv, *z = x + 2 * nv, *p = x + 3 * nv, *q = x + 4 * nv;
    double2 *t1 = qh->evec, *t2 = t1 + ne, *t3 = t1 + 2 * ne;
    double *pa = qh->partial, *pb = qh->partial + 4 * kQBlocks;
    const double2 *Dd = reinterpret_cast<const double2 *>(d);
    // right-hand side Sigma^T d = D^T [*eps] d
    k_qe_mass<<<gm, kQThreads, 0, st>>>(qh->csr(), nullptr, Dd, t2);
    k_qe_start<<<gv, kQThreads, 0, st>>>(nv, qh->v2e_ptr, qh->v2e_code, t2, qh->dinv, x, r, z, p, q, pb, qh->sc);
    QH_TRY(hipGetLastError());
    const double tol2 = tol * tol;
    double hs[12];
    int k = 0;
    for (;;) {
        const int n = std::min(10, max_iter - k);
        for (int j = 0; j < n; ++j, ++k) {
            k_qe_grad<<<ge, kQThreads, 0, st>>>(ne, qh->ev, qh->sc, z, t1, pb, gv, k, tol2, 0);
            k_qe_mass<<<gm, kQThreads, 0, st>>>(qh->csr(), qh->sc, t1, t2);
            k_qe_mass<<<gm, kQThreads, 0, st>>>(qh->csr(), qh->sc, t2, t3);
            k_qe_divq<<<gv, kQThreads, 0, st>>>(nv, qh->v2e_ptr, qh->v2e_code, qh->sc, z, p, q, t3, pb, gv, pa, k);
            k_qe_update<<<gv, kQThreads, 0, st>>>(nv, qh->sc, qh->dinv, p, q, x, r, z, pa, gv, pb, k);
        }
        if (k >= max_iter) k_qe_grad<<<ge, kQThreads, 0, st>>>(ne, qh->ev, qh->sc, z, t1, pb, gv, k, tol2, 1);
        QH_TRY(hipGetLastError());
        if (int rr = read_scalars(qh, st, hs)) return rr;
        if (hs[10] != 0.0 || k >= max_iter) break;
    }
    if (int rr = finish(hs, tol, iters_out, resid_out)) return rr;
    // minimum-norm E_ns, then Sigma E_ns = [*eps] D E_ns and the split of d
    k_qe_sum<<<gv, kQThreads, 0, st>>>(nv, x, pa);
    k_qe_center<<<gv, kQThreads, 0, st>>>(nv, x, pa, gv, reinterpret_cast<double2 *>(e_ns));
    if (d_sigma || d_lambda) {
        k_qe_dx<<<blocks_for(ne), kQThreads, 0, st>>>(ne, qh->ev, x, t1);
        k_qe_mass<<<gm, kQThreads, 0, st>>>(qh->csr(), nullptr, t1, t2);
        k_qe_split<<<blocks_for(ne), kQThreads, 0, st>>>(ne, Dd, t2, reinterpret_cast<double2 *>(d_sigma),
                                                         reinterpret_cast<double2 *>(d_lambda));
    }
    QH_TRY(hipGetLastError());
    return ETPIC_OK;
}

int etpic_tree_cotree(int64_t n_vert, const double *xyz_host, int64_t n_tet, const int32_t *tet_vert_host,
                      uint8_t *edge_tree_host, uint8_t *face_tree_host, int64_t counts_out[4]) {
    if (!edge_tree_host || !face_tree_host || !counts_out) return qfail(ETPIC_EINVAL, "null argument");
    std::string err;
    etpic::HostMesh H;
    if (int r = etpic::build_host_mesh(n_vert, xyz_host, n_tet, tet_vert_host, H, err))
        return qfail(r == -4 ? ETPIC_EMESH : ETPIC_EINVAL, "mesh: %s", err.c_str());
    etpic::tree_cotree(H, edge_tree_host, face_tree_host);
    int64_t te = 0, tf = 0;
    for (int64_t e = 0; e < H.ne; ++e) te += edge_tree_host[e];
    for (int64_t f = 0; f < H.nf; ++f) tf += face_tree_host[f];
    counts_out[0] = te;
    counts_out[1] = H.ne - te;
    counts_out[2] = tf;
    counts_out[3] = H.nf - tf;
    return ETPIC_OK;
}

}  // extern "C"

// ================================================================ eq. sol_disc
// The solenoidal system on the cotree unknowns (Quasi Helmholtz section,
// Discrete System; blocks of App. A as printed, Euclidean projectors):
//   Z11 = C_b^T P^Lambda_b C_b,            Z12 = C_b^T [curl] [*eps]^-1 P^Lambda_e [*eps] C_e,
//   Z13 = C_b^T [curl] [*eps]^-1 Sigma C_z, Z21 = C_e^T P^Lambda_e [*eps] C_e,
//   Z22 = C_e^T [curl]^T [*mu^-1] P^Lambda_b C_b,  Z23 = C_e^T Sigma C_z,
// with [curl] = C, the signed face-edge incidence ((C e)_f = e_ab + e_bc - e_ac
// for the face a < b < c: the curl of a Whitney edge function is that sum of
// face functions), Sigma = [*eps] D, so [*eps]^-1 P^Lambda_e [*eps] u =
// u - D E_ns(u) with E_ns the minimum-norm solution of
// Sigma^T Sigma E_ns = Sigma^T [*eps] u, and [*eps]^-1 Sigma = D.  C_e and C_b
// select the cotree edges and faces of the tree-cotree split, C_z the nodes
// off the wall.  Every block is applied matrix-free; the projectors by the CG
// solves above.
//
// The step (trapezoidal rule over [t_n, t_n + dt], a = 1/dt + j w/2):
//   Z11 (a B1 - conj(a) B0) + Z12 (E1 + E0)/2 = 0       (Z13 = 0: C D = 0)
//   Z21 (a E1 - conj(a) E0) - Z22 (B1 + B0)/2 = src.
// With b = P^Lambda_b C_b B_s (the divergence-free face field the blocks act
// on), the first row holds on every face, not only on the cotree ones: b and
// C C_e E are divergence-free, and a divergence-free face field that vanishes
// on the cotree faces vanishes.  So b1 = (conj(a) b0 - C C_e (E0 + E1)/2) / a
// explicitly, and the second row becomes one system on the cotree edges,
//   S E1 = [a Z21 + C_e^T K C_e / (4a)] E1 = conj(a) Z21 E0
//          + C_e^T C^T [*mu^-1] (b0 + conj(a) b0 / a) / 2 - C_e^T K C_e E0 / (4a) + src,
// K = C^T [*mu^-1] C the curl-curl stiffness, solved by restarted GMRES with
// right Jacobi preconditioning (diagonal a [*eps]_ee + K_ee / (4a)).  The
// state carried from step to step is (b, E_s).

namespace {

constexpr int kZThreads = 256;
constexpr int kZDotBlocks = 64;
constexpr int kZRestart = 100;   // GMRES restart length

inline unsigned zgrid(int64_t n) { return (unsigned)std::max<int64_t>(1, (n + kZThreads - 1) / kZThreads); }

__global__ void __launch_bounds__(kZThreads) k_z_fill(int64_t n, double2 *__restrict__ x) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = make_double2(0.0, 0.0);
}

// full[ids[i]] = x[i] (the other entries left as they are)
__global__ void __launch_bounds__(kZThreads) k_z_scatter(int64_t n, const int32_t *__restrict__ ids,
                                                         const double2 *__restrict__ x, double2 *__restrict__ full) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) full[ids[i]] = x[i];
}

// y[i] = alpha * u[ids[i]] + beta * v[ids[i]] (v may be NULL)
__global__ void __launch_bounds__(kZThreads) k_z_gather(int64_t n, const int32_t *__restrict__ ids, double2 alpha,
                                                        const double2 *__restrict__ u, double2 beta,
                                                        const double2 *__restrict__ v, double2 *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double2 a = u[ids[i]];
    double2 r = make_double2(alpha.x * a.x - alpha.y * a.y, alpha.x * a.y + alpha.y * a.x);
    if (v) {
        const double2 b = v[ids[i]];
        r.x += beta.x * b.x - beta.y * b.y;
        r.y += beta.x * b.y + beta.y * b.x;
    }
    y[i] = r;
}

// c = C e: (C e)_f = e_ab + e_bc - e_ac
__global__ void __launch_bounds__(kZThreads) k_z_curl(int64_t nf, const int4 *__restrict__ fe,
                                                      const double2 *__restrict__ e, double2 *__restrict__ c) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    const int4 t = fe[f];
    c[f] = csub(cadd(e[t.x], e[t.y]), e[t.z]);
}

// y = C^T c: per edge the signed sum over its faces (code = 2 f + (sign > 0))
__global__ void __launch_bounds__(kZThreads) k_z_curlt(int64_t ne, const int32_t *__restrict__ ptr,
                                                       const int32_t *__restrict__ code, const double2 *__restrict__ c,
                                                       double2 *__restrict__ y) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ne) return;
    double2 s = make_double2(0.0, 0.0);
    for (int32_t k = ptr[e]; k < ptr[e + 1]; ++k) {
        const int32_t q = code[k];
        s = (q & 1) ? cadd(s, c[q >> 1]) : csub(s, c[q >> 1]);
    }
    y[e] = s;
}

// z = u - v
__global__ void __launch_bounds__(kZThreads) k_z_sub(int64_t n, const double2 *__restrict__ u,
                                                     const double2 *__restrict__ v, double2 *__restrict__ z) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) z[i] = csub(u[i], v[i]);
}

// b = (ab b - c / 2) / a (complex a, ab)
__global__ void __launch_bounds__(kZThreads) k_z_faraday(int64_t nf, double2 a, double2 ab,
                                                         const double2 *__restrict__ c, double2 *__restrict__ b) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    const double2 x = b[f], h = cscale(c[f], 0.5);
    const double2 t = make_double2(ab.x * x.x - ab.y * x.y - h.x, ab.x * x.y + ab.y * x.x - h.y);
    const double den = a.x * a.x + a.y * a.y;   // t / a = t conj(a) / |a|^2
    b[f] = make_double2((t.x * a.x + t.y * a.y) / den, (t.y * a.x - t.x * a.y) / den);
}

// z_i = v_i / (a m_i + k_i / (4a)): right Jacobi preconditioner of S
__global__ void __launch_bounds__(kZThreads) k_z_precond(int64_t n, double2 a, const double *__restrict__ m,
                                                         const double *__restrict__ kd, const double2 *__restrict__ v,
                                                         double2 *__restrict__ z) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double den = a.x * a.x + a.y * a.y;
    const double2 ia = make_double2(a.x / den, -a.y / den);   // 1 / a
    const double2 d = make_double2(a.x * m[i] + 0.25 * kd[i] * ia.x, a.y * m[i] + 0.25 * kd[i] * ia.y);
    const double dd = d.x * d.x + d.y * d.y;
    const double2 x = v[i];
    z[i] = make_double2((x.x * d.x + x.y * d.y) / dd, (x.y * d.x - x.x * d.y) / dd);
}

// partial[(i * nb + b)] = block b's share of <V_i, w> = sum conj(V_i) w, i < nvec
__global__ void __launch_bounds__(kZThreads) k_z_dots(int64_t n, const double2 *__restrict__ V, int64_t ld,
                                                      const double2 *__restrict__ w, double2 *__restrict__ partial) {
    const int i = blockIdx.y;
    const double2 *v = V + (int64_t)i * ld;
    double re = 0.0, im = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < n; k += (int64_t)gridDim.x * blockDim.x) {
        const double2 a = v[k], b = w[k];
        re += a.x * b.x + a.y * b.y;
        im += a.x * b.y - a.y * b.x;
    }
    __shared__ double sr[kZThreads / 64], si[kZThreads / 64];
    for (int off = 32; off > 0; off >>= 1) {
        re += __shfl_xor(re, off);
        im += __shfl_xor(im, off);
    }
    if ((threadIdx.x & 63) == 0) {
        sr[threadIdx.x >> 6] = re;
        si[threadIdx.x >> 6] = im;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double tr = 0.0, ti = 0.0;
        for (int k = 0; k < kZThreads / 64; ++k) {
            tr += sr[k];
            ti += si[k];
        }
        partial[(int64_t)i * gridDim.x + blockIdx.x] = make_double2(tr, ti);
    }
}

// h[i] = sum over the nb partials of vector i (one block per i, fixed order)
__global__ void __launch_bounds__(kZThreads) k_z_dsum(int nb, const double2 *__restrict__ partial,
                                                      double2 *__restrict__ h) {
    if (threadIdx.x != 0) return;
    double re = 0.0, im = 0.0;
    for (int b = 0; b < nb; ++b) {
        const double2 p = partial[(int64_t)blockIdx.x * nb + b];
        re += p.x;
        im += p.y;
    }
    h[blockIdx.x] = make_double2(re, im);
}

// w -= sum_{i < m} h[i] V_i
__global__ void __launch_bounds__(kZThreads) k_z_orth(int64_t n, const double2 *__restrict__ V, int64_t ld, int m,
                                                      const double2 *__restrict__ h, double2 *__restrict__ w) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double2 s = w[k];
    for (int i = 0; i < m; ++i) {
        const double2 c = h[i], v = V[(int64_t)i * ld + k];
        s.x -= c.x * v.x - c.y * v.y;
        s.y -= c.x * v.y + c.y * v.x;
    }
    w[k] = s;
}

// v = w * s (real s)
__global__ void __launch_bounds__(kZThreads) k_z_scale(int64_t n, const double2 *__restrict__ w, double s,
                                                       double2 *__restrict__ v) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) v[k] = cscale(w[k], s);
}

// u = sum_{i < m} y[i] V_i
__global__ void __launch_bounds__(kZThreads) k_z_comb(int64_t n, const double2 *__restrict__ V, int64_t ld, int m,
                                                      const double2 *__restrict__ y, double2 *__restrict__ u) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    double2 s = make_double2(0.0, 0.0);
    for (int i = 0; i < m; ++i) {
        const double2 c = y[i], v = V[(int64_t)i * ld + k];
        s.x += c.x * v.x - c.y * v.y;
        s.y += c.x * v.y + c.y * v.x;
    }
    u[k] = s;
}

// x += u; r = rhs - s (either may be NULL)
__global__ void __launch_bounds__(kZThreads) k_z_axpy(int64_t n, double2 *__restrict__ x, const double2 *__restrict__ u,
                                                      double2 *__restrict__ r, const double2 *__restrict__ rhs,
                                                      const double2 *__restrict__ s) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    if (x) x[k] = cadd(x[k], u[k]);
    if (r) r[k] = csub(rhs[k], s[k]);
}

}  // namespace

struct etpic_cotree {
    int device = 0;
    int64_t nv = 0, ne = 0, nf = 0, nt = 0, nec = 0, nfc = 0, nz = 0, fnnz = 0;
    // device part (caller's buffer)
    int32_t *ce = nullptr, *cb = nullptr, *cz = nullptr;   // cotree edges, cotree faces, nodes off the wall
    int4 *fe = nullptr;                                   // per face: edges ab, bc, ac
    int32_t *e2f_ptr = nullptr, *e2f_code = nullptr;      // edge -> faces, 2 f + (sign > 0)
    int32_t *frow = nullptr, *fcol = nullptr;             // [*mu^-1] CSR
    double *fval = nullptr;
    double *mdiag = nullptr, *kdiag = nullptr;            // per cotree edge: [*eps]_ee, K_ee
    double2 *ue = nullptr, *te = nullptr, *le = nullptr, *ke = nullptr, *ke2 = nullptr;   // edge vectors
    double2 *cf = nullptr, *ff = nullptr, *gf = nullptr;  // face vectors
    double2 *nn = nullptr;                                // node vector
    double2 *V = nullptr;                                 // (kZRestart + 1) x nec Krylov basis
    double2 *w = nullptr, *z = nullptr, *r = nullptr, *rhs = nullptr, *sx = nullptr, *e0 = nullptr;   // nec each
    double2 *h = nullptr, *part = nullptr;                // dots and their block partials
    bool bound = false;
    // host tables
    std::vector<int32_t> h_ce, h_cb, h_cz, h_e2f_ptr, h_e2f_code, h_frow, h_fcol;
    std::vector<int4> h_fe;
    std::vector<double> h_fval, h_mdiag, h_kdiag;

    EdgeCsr face_csr() const { return EdgeCsr{nf, frow, fcol, fval}; }
};

namespace {

struct ZPtrs {
    int32_t *ce, *cb, *cz, *e2f_ptr, *e2f_code, *frow, *fcol;
    int4 *fe;
    double *fval, *mdiag, *kdiag;
    double2 *ue, *te, *le, *ke, *ke2, *cf, *ff, *gf, *nn, *V, *w, *z, *r, *rhs, *sx, *e0, *h, *part;
};
ZPtrs z_layout(const etpic_cotree *Z, QhCarve &cv) {
    ZPtrs d;
    d.ce = cv.take<int32_t>(Z->h_ce.size());
    d.cb = cv.take<int32_t>(Z->h_cb.size());
    d.cz = cv.take<int32_t>(Z->h_cz.size());
    d.fe = cv.take<int4>(Z->h_fe.size());
    d.e2f_ptr = cv.take<int32_t>(Z->h_e2f_ptr.size());
    d.e2f_code = cv.take<int32_t>(Z->h_e2f_code.size());
    d.frow = cv.take<int32_t>(Z->h_frow.size());
    d.fcol = cv.take<int32_t>(Z->h_fcol.size());
    d.fval = cv.take<double>(Z->h_fval.size());
    d.mdiag = cv.take<double>(Z->h_mdiag.size());
    d.kdiag = cv.take<double>(Z->h_kdiag.size());
    d.ue = cv.take<double2>(Z->ne);
    d.te = cv.take<double2>(Z->ne);
    d.le = cv.take<double2>(Z->ne);
    d.ke = cv.take<double2>(Z->ne);
    d.ke2 = cv.take<double2>(Z->ne);
    d.cf = cv.take<double2>(Z->nf);
    d.ff = cv.take<double2>(Z->nf);
    d.gf = cv.take<double2>(Z->nf);
    d.nn = cv.take<double2>(Z->nv);
    d.V = cv.take<double2>((size_t)(kZRestart + 1) * Z->nec);
    d.w = cv.take<double2>(Z->nec);
    d.z = cv.take<double2>(Z->nec);
    d.r = cv.take<double2>(Z->nec);
    d.rhs = cv.take<double2>(Z->nec);
    d.sx = cv.take<double2>(Z->nec);
    d.e0 = cv.take<double2>(Z->nec);
    d.h = cv.take<double2>(kZRestart + 1);
    d.part = cv.take<double2>((size_t)(kZRestart + 1) * kZDotBlocks);
    return d;
}

// Host tables of the cotree object: the split, the incidences, the face mass.
int z_build(etpic_cotree *Z, const etpic_qh *Q, int64_t nv, const double *xyz, int64_t nt, const int32_t *tet_vert,
            double mu) {
    std::string err;
    etpic::HostMesh H;
    if (int r = etpic::build_host_mesh(nv, xyz, nt, tet_vert, H, err))
        return qfail(r == -4 ? ETPIC_EMESH : ETPIC_EINVAL, "cotree mesh: %s", err.c_str());
    if (H.nv != Q->nv || H.ne != Q->ne || H.nf != Q->nf || H.nt != Q->nt)
        return qfail(ETPIC_EINVAL, "cotree: the mesh is not the projector object's");
    Z->nv = H.nv;
    Z->ne = H.ne;
    Z->nf = H.nf;
    Z->nt = H.nt;
    std::vector<uint8_t> et((size_t)H.ne), ft((size_t)H.nf), wall((size_t)H.nv, 0);
    etpic::tree_cotree(H, et.data(), ft.data());
    for (int64_t e = 0; e < H.ne; ++e)
        if (!et[e]) Z->h_ce.push_back((int32_t)e);
    for (int64_t f = 0; f < H.nf; ++f)
        if (!ft[f]) Z->h_cb.push_back((int32_t)f);
    Z->nec = (int64_t)Z->h_ce.size();
    Z->nfc = (int64_t)Z->h_cb.size();
    // face -> edges (ab, bc, ac), the wall nodes, the face mass (per tet, 4 x 4)
    Z->h_fe.assign((size_t)H.nf, make_int4(-1, -1, -1, 0));
    auto le = [](int i, int j) { return i == 0 ? j - 1 : (i == 1 ? j + 1 : 5); };   // local edge of i < j
    std::vector<int64_t> key;
    std::vector<double> val;
    key.reserve((size_t)16 * H.nt);
    val.reserve((size_t)16 * H.nt);
    for (int64_t t = 0; t < H.nt; ++t) {
        const etpic::TetTopo &tp = H.topo[t];
        const double *g = &H.grad[12 * t];
        double X[4][3][3];   // face k: the three vectors g_j x g_l, g_l x g_i, g_i x g_j
        int idx[4][3];
        for (int k = 0; k < 4; ++k) {
            const int i = etpic::kLocalFace[k][0], j = etpic::kLocalFace[k][1], l = etpic::kLocalFace[k][2];
            const int pr[3][3] = {{i, j, l}, {j, l, i}, {l, i, j}};   // (lambda, cross of the other two in order)
            for (int p = 0; p < 3; ++p) {
                const double *u = g + 3 * pr[p][1], *v = g + 3 * pr[p][2];
                X[k][p][0] = u[1] * v[2] - u[2] * v[1];
                X[k][p][1] = u[2] * v[0] - u[0] * v[2];
                X[k][p][2] = u[0] * v[1] - u[1] * v[0];
                idx[k][p] = pr[p][0];
            }
            int4 &fe = Z->h_fe[tp.f[k]];
            if (fe.x < 0) fe = make_int4(tp.e[le(i, j)], tp.e[le(j, l)], tp.e[le(i, l)], 0);
            if (tp.n[k] < 0)
                for (int q = 0; q < 3; ++q) wall[tp.v[etpic::kLocalFace[k][q]]] = 1;
        }
        // (1/mu) int W2_k . W2_m, W2 = 2 sum lambda_p X_p, int lambda_p lambda_q = V (1 + delta_pq) / 20
        const double V = H.vol[t];
        for (int k = 0; k < 4; ++k)
            for (int m = 0; m < 4; ++m) {
                double s = 0.0;
                for (int p = 0; p < 3; ++p)
                    for (int q = 0; q < 3; ++q) {
                        const double dot = X[k][p][0] * X[m][q][0] + X[k][p][1] * X[m][q][1] + X[k][p][2] * X[m][q][2];
                        s += dot * (idx[k][p] == idx[m][q] ? 2.0 : 1.0);
                    }
                key.push_back((int64_t)tp.f[k] * H.nf + tp.f[m]);
                val.push_back(4.0 * s * V / (20.0 * mu));
            }
    }
    for (int64_t v = 0; v < H.nv; ++v)
        if (!wall[v]) Z->h_cz.push_back((int32_t)v);
    Z->nz = (int64_t)Z->h_cz.size();
    {   // COO -> CSR, duplicates summed
        std::vector<int64_t> order(key.size());
        for (size_t i = 0; i < order.size(); ++i) order[i] = (int64_t)i;
        std::sort(order.begin(), order.end(), [&](int64_t a, int64_t b) { return key[a] < key[b]; });
        Z->h_frow.assign((size_t)H.nf + 1, 0);
        for (size_t i = 0; i < order.size();) {
            const int64_t k = key[order[i]];
            double s = 0.0;
            for (; i < order.size() && key[order[i]] == k; ++i) s += val[order[i]];
            Z->h_fcol.push_back((int32_t)(k % H.nf));
            Z->h_fval.push_back(s);
            ++Z->h_frow[k / H.nf + 1];
        }
        for (int64_t f = 0; f < H.nf; ++f) Z->h_frow[f + 1] += Z->h_frow[f];
        Z->fnnz = (int64_t)Z->h_fval.size();
    }
    {   // edge -> faces with signs (+ for ab, bc; - for ac)
        Z->h_e2f_ptr.assign((size_t)H.ne + 1, 0);
        for (const int4 &fe : Z->h_fe) {
            if (fe.x < 0) return qfail(ETPIC_EMESH, "cotree: a face in no tet");
            ++Z->h_e2f_ptr[fe.x + 1];
            ++Z->h_e2f_ptr[fe.y + 1];
            ++Z->h_e2f_ptr[fe.z + 1];
        }
        for (int64_t e = 0; e < H.ne; ++e) Z->h_e2f_ptr[e + 1] += Z->h_e2f_ptr[e];
        Z->h_e2f_code.assign((size_t)Z->h_e2f_ptr[H.ne], 0);
        std::vector<int32_t> fill(Z->h_e2f_ptr.begin(), Z->h_e2f_ptr.end() - 1);
        for (int64_t f = 0; f < H.nf; ++f) {
            const int4 fe = Z->h_fe[f];
            Z->h_e2f_code[fill[fe.x]++] = (int32_t)(2 * f + 1);
            Z->h_e2f_code[fill[fe.y]++] = (int32_t)(2 * f + 1);
            Z->h_e2f_code[fill[fe.z]++] = (int32_t)(2 * f);
        }
    }
    // preconditioner diagonals on the cotree edges: [*eps]_ee and K_ee = sum s_f s_g F_fg
    auto fentry = [&](int32_t f, int32_t g) {
        const auto b = Z->h_fcol.begin() + Z->h_frow[f], e = Z->h_fcol.begin() + Z->h_frow[f + 1];
        const auto it = std::lower_bound(b, e, g);
        return (it != e && *it == g) ? Z->h_fval[it - Z->h_fcol.begin()] : 0.0;
    };
    for (int32_t e : Z->h_ce) {
        double m = 0.0;
        for (int32_t j = Q->h_rowptr[e]; j < Q->h_rowptr[e + 1]; ++j)
            if (Q->h_col[j] == e) m = Q->h_M[j];
        double k = 0.0;
        for (int32_t a = Z->h_e2f_ptr[e]; a < Z->h_e2f_ptr[e + 1]; ++a)
            for (int32_t b = Z->h_e2f_ptr[e]; b < Z->h_e2f_ptr[e + 1]; ++b) {
                const int32_t ca = Z->h_e2f_code[a], cbb = Z->h_e2f_code[b];
                const double s = ((ca & 1) ? 1.0 : -1.0) * ((cbb & 1) ? 1.0 : -1.0);
                k += s * fentry(ca >> 1, cbb >> 1);
            }
        if (!(m > 0.0)) return qfail(ETPIC_EMESH, "cotree: edge %d has no mass", e);
        Z->h_mdiag.push_back(m);
        Z->h_kdiag.push_back(k);
    }
    return ETPIC_OK;
}

int z_check(const etpic_cotree *Z, const etpic_qh *Q) {
    if (!Z || !Q) return qfail(ETPIC_EINVAL, "null argument");
    if (!Z->bound) return qfail(ETPIC_ESTATE, "no device buffer bound (etpic_cotree_bytes, etpic_cotree_bind)");
    if (!Q->bound) return qfail(ETPIC_ESTATE, "projector object not bound");
    if (Z->nv != Q->nv || Z->ne != Q->ne || Z->nf != Q->nf || Z->nt != Q->nt || Z->device != Q->device)
        return qfail(ETPIC_EINVAL, "cotree and projector objects of different meshes or devices");
    return ETPIC_OK;
}

}  // namespace

namespace {

using cplx = std::complex<double>;

inline double2 d2(cplx c) { return make_double2(c.real(), c.imag()); }

// y = x (device copy)
int zcopy(const double2 *x, double2 *y, int64_t n, hipStream_t st) {
    QH_TRY(hipMemcpyAsync(y, x, sizeof(double2) * n, hipMemcpyDeviceToDevice, st));
    return ETPIC_OK;
}

// out[i] = <V_i, w>, i < m (synchronises)
int zdots(etpic_cotree *Z, int64_t n, const double2 *V, int64_t ld, int m, const double2 *w, cplx *out,
          hipStream_t st) {
    k_z_dots<<<dim3(kZDotBlocks, m), kZThreads, 0, st>>>(n, V, ld, w, Z->part);
    k_z_dsum<<<m, kZThreads, 0, st>>>(kZDotBlocks, Z->part, Z->h);
    QH_TRY(hipGetLastError());
    std::vector<double2> hv((size_t)m);
    QH_TRY(hipMemcpyAsync(hv.data(), Z->h, sizeof(double2) * m, hipMemcpyDeviceToHost, st));
    QH_TRY(hipStreamSynchronize(st));
    for (int i = 0; i < m; ++i) out[i] = cplx(hv[i].x, hv[i].y);
    return ETPIC_OK;
}

int znorm(etpic_cotree *Z, int64_t n, const double2 *w, double *nrm, hipStream_t st) {
    cplx d;
    if (int r = zdots(Z, n, w, n, 1, w, &d, st)) return r;
    *nrm = std::sqrt(std::max(d.real(), 0.0));
    return ETPIC_OK;
}

int zproj_e(etpic_qh *Q, const double2 *d, double2 *d_lambda, double2 *e_ns, double tol, int max_iter, hipStream_t st) {
    return etpic_qh_project_e(Q, reinterpret_cast<const double *>(d), nullptr, reinterpret_cast<double *>(d_lambda),
                              reinterpret_cast<double *>(e_ns), tol, max_iter, nullptr, nullptr, st);
}

int zproj_b(etpic_qh *Q, const double2 *b, double2 *b_out, double tol, int max_iter, hipStream_t st) {
    return etpic_qh_project_b(Q, reinterpret_cast<const double *>(b), reinterpret_cast<double *>(b_out), tol,
                              max_iter, nullptr, nullptr, st);
}

void zmass_e(const etpic_qh *Q, const double2 *x, double2 *y, hipStream_t st) {
    k_qe_mass<<<cg_blocks(Q->ne * kQRowLanes), kQThreads, 0, st>>>(Q->csr(), nullptr, x, y);
}

void zmass_f(const etpic_cotree *Z, const double2 *x, double2 *y, hipStream_t st) {
    k_qe_mass<<<cg_blocks(Z->nf * kQRowLanes), kQThreads, 0, st>>>(Z->face_csr(), nullptr, x, y);
}

// ue = C_e x (tree edges zero)
void zscatter_e(etpic_cotree *Z, const double2 *x, hipStream_t st) {
    k_z_fill<<<zgrid(Z->ne), kZThreads, 0, st>>>(Z->ne, Z->ue);
    k_z_scatter<<<zgrid(Z->nec), kZThreads, 0, st>>>(Z->nec, Z->ce, x, Z->ue);
}

// S x = a C_e^T P^Lambda_e [*eps] C_e x + C_e^T K C_e x / (4a) into y
int zS(etpic_cotree *Z, etpic_qh *Q, cplx a, const double2 *x, double2 *y, double itol, int imax, hipStream_t st) {
    zscatter_e(Z, x, st);
    zmass_e(Q, Z->ue, Z->te, st);
    if (int r = zproj_e(Q, Z->te, Z->le, nullptr, itol, imax, st)) return r;
    k_z_curl<<<zgrid(Z->nf), kZThreads, 0, st>>>(Z->nf, Z->fe, Z->ue, Z->cf);
    zmass_f(Z, Z->cf, Z->gf, st);
    k_z_curlt<<<zgrid(Z->ne), kZThreads, 0, st>>>(Z->ne, Z->e2f_ptr, Z->e2f_code, Z->gf, Z->ke);
    k_z_gather<<<zgrid(Z->nec), kZThreads, 0, st>>>(Z->nec, Z->ce, d2(a), Z->le, d2(0.25 / a), Z->ke, y);
    QH_TRY(hipGetLastError());
    return ETPIC_OK;
}

// Restarted GMRES(kZRestart) on S x = rhs, right Jacobi preconditioning, x
// holding the initial guess; classical Gram-Schmidt applied twice.
int zgmres(etpic_cotree *Z, etpic_qh *Q, cplx a, double2 *x, double tol, int max_iter, double itol, int imax,
           int *iters_out, double *resid_out, hipStream_t st) {
    const int64_t n = Z->nec;
    const int M = kZRestart;
    double bn = 0.0, beta = 0.0;
    if (int r = znorm(Z, n, Z->rhs, &bn, st)) return r;
    if (bn == 0.0) {
        k_z_fill<<<zgrid(n), kZThreads, 0, st>>>(n, x);
        if (iters_out) *iters_out = 0;
        if (resid_out) *resid_out = 0.0;
        QH_TRY(hipGetLastError());
        return ETPIC_OK;
    }
    auto residual = [&]() -> int {
        if (int r = zS(Z, Q, a, x, Z->sx, itol, imax, st)) return r;
        k_z_axpy<<<zgrid(n), kZThreads, 0, st>>>(n, nullptr, nullptr, Z->r, Z->rhs, Z->sx);
        return znorm(Z, n, Z->r, &beta, st);
    };
    if (int r = residual()) return r;
    int total = 0;
    std::vector<cplx> H((size_t)(M + 1) * M), g((size_t)M + 1), cs((size_t)M), sn((size_t)M), hc((size_t)M + 1),
        h2((size_t)M + 1), y((size_t)M);
    auto Hij = [&](int i, int j) -> cplx & { return H[(size_t)i * M + j]; };
    while (beta > tol * bn) {
        if (total >= max_iter || !std::isfinite(beta)) break;
        std::fill(H.begin(), H.end(), cplx(0.0, 0.0));
        std::fill(g.begin(), g.end(), cplx(0.0, 0.0));
        g[0] = beta;
        k_z_scale<<<zgrid(n), kZThreads, 0, st>>>(n, Z->r, 1.0 / beta, Z->V);
        int j = 0;
        while (j < M && total < max_iter) {
            double2 *vj = Z->V + (int64_t)j * n, *vn = Z->V + (int64_t)(j + 1) * n;
            k_z_precond<<<zgrid(n), kZThreads, 0, st>>>(n, d2(a), Z->mdiag, Z->kdiag, vj, Z->z);
            if (int r = zS(Z, Q, a, Z->z, Z->w, itol, imax, st)) return r;
            for (int pass = 0; pass < 2; ++pass) {
                if (int r = zdots(Z, n, Z->V, n, j + 1, Z->w, (pass ? h2 : hc).data(), st)) return r;
                std::vector<double2> hv((size_t)j + 1);
                for (int i = 0; i <= j; ++i) hv[i] = d2(pass ? h2[i] : hc[i]);
                QH_TRY(hipMemcpyAsync(Z->h, hv.data(), sizeof(double2) * (j + 1), hipMemcpyHostToDevice, st));
                k_z_orth<<<zgrid(n), kZThreads, 0, st>>>(n, Z->V, n, j + 1, Z->h, Z->w);
                QH_TRY(hipStreamSynchronize(st));
            }
            double hn = 0.0;
            if (int r = znorm(Z, n, Z->w, &hn, st)) return r;
            for (int i = 0; i <= j; ++i) Hij(i, j) = hc[i] + h2[i];
            Hij(j + 1, j) = hn;
            for (int i = 0; i < j; ++i) {   // earlier rotations on column j
                const cplx t = cs[i] * Hij(i, j) + sn[i] * Hij(i + 1, j);
                Hij(i + 1, j) = -std::conj(sn[i]) * Hij(i, j) + cs[i] * Hij(i + 1, j);
                Hij(i, j) = t;
            }
            {   // the rotation that zeroes H(j+1, j)
                const cplx p = Hij(j, j), q = Hij(j + 1, j);
                const double ap = std::abs(p), t = std::sqrt(std::norm(p) + std::norm(q));
                if (t == 0.0) {
                    cs[j] = 1.0;
                    sn[j] = 0.0;
                } else if (ap == 0.0) {
                    cs[j] = 0.0;
                    sn[j] = std::conj(q) / std::abs(q);
                } else {
                    cs[j] = ap / t;
                    sn[j] = (p / ap) * std::conj(q) / t;
                }
                Hij(j, j) = cs[j] * p + sn[j] * q;
                Hij(j + 1, j) = 0.0;
                g[j + 1] = -std::conj(sn[j]) * g[j];
                g[j] = cs[j] * g[j];
            }
            ++j;
            ++total;
            if (hn > 0.0) k_z_scale<<<zgrid(n), kZThreads, 0, st>>>(n, Z->w, 1.0 / hn, vn);
            if (std::abs(g[j]) <= tol * bn || hn == 0.0) break;
        }
        for (int i = j - 1; i >= 0; --i) {   // H y = g, upper triangular
            cplx s = g[i];
            for (int k = i + 1; k < j; ++k) s -= Hij(i, k) * y[k];
            y[i] = s / Hij(i, i);
        }
        std::vector<double2> yv((size_t)j);
        for (int i = 0; i < j; ++i) yv[i] = d2(y[i]);
        QH_TRY(hipMemcpyAsync(Z->h, yv.data(), sizeof(double2) * j, hipMemcpyHostToDevice, st));
        k_z_comb<<<zgrid(n), kZThreads, 0, st>>>(n, Z->V, n, j, Z->h, Z->w);
        k_z_precond<<<zgrid(n), kZThreads, 0, st>>>(n, d2(a), Z->mdiag, Z->kdiag, Z->w, Z->z);
        k_z_axpy<<<zgrid(n), kZThreads, 0, st>>>(n, x, Z->z, nullptr, nullptr, nullptr);
        QH_TRY(hipStreamSynchronize(st));
        if (int r = residual()) return r;
    }
    if (iters_out) *iters_out = total;
    if (resid_out) *resid_out = beta / bn;
    if (!(beta <= tol * bn))
        return qfail(ETPIC_ENOCONV, "cotree GMRES: relative residual %.3e after %d iterations (tol %.1e)", beta / bn,
                     total, tol);
    return ETPIC_OK;
}

}  // namespace

extern "C" {

int etpic_cotree_create(etpic_cotree **out, const etpic_qh *qh, int64_t nv, const double *xyz, int64_t nt,
                        const int32_t *tet_vert, double mu) {
    if (!out || !qh) return qfail(ETPIC_EINVAL, "null argument");
    *out = nullptr;
    if (!(mu > 0.0) || !std::isfinite(mu)) return qfail(ETPIC_EINVAL, "mu must be positive");
    etpic_cotree *Z = new etpic_cotree();
    Z->device = qh->device;
    if (int r = z_build(Z, qh, nv, xyz, nt, tet_vert, mu)) {
        delete Z;
        return r;
    }
    *out = Z;
    return ETPIC_OK;
}

int etpic_cotree_bytes(const etpic_cotree *z, size_t *bytes) {
    if (!z || !bytes) return qfail(ETPIC_EINVAL, "null argument");
    QhCarve cv;
    (void)z_layout(z, cv);
    *bytes = cv.used;
    return ETPIC_OK;
}

int etpic_cotree_bind(etpic_cotree *z, void *dev_buf, size_t bytes) {
    if (!z || !dev_buf) return qfail(ETPIC_EINVAL, "null argument");
    if (reinterpret_cast<uintptr_t>(dev_buf) & 255u) return qfail(ETPIC_EINVAL, "buffer not 256-byte aligned");
    size_t need = 0;
    if (int r = etpic_cotree_bytes(z, &need)) return r;
    if (bytes < need) return qfail(ETPIC_EINVAL, "buffer of %zu bytes, %zu needed", bytes, need);
    QH_TRY(hipSetDevice(z->device));
    QH_TRY(hipDeviceSynchronize());
    QhCarve cv;
    cv.base = static_cast<char *>(dev_buf);
    const ZPtrs d = z_layout(z, cv);
    z->ce = d.ce;
    z->cb = d.cb;
    z->cz = d.cz;
    z->fe = d.fe;
    z->e2f_ptr = d.e2f_ptr;
    z->e2f_code = d.e2f_code;
    z->frow = d.frow;
    z->fcol = d.fcol;
    z->fval = d.fval;
    z->mdiag = d.mdiag;
    z->kdiag = d.kdiag;
    z->ue = d.ue;
    z->te = d.te;
    z->le = d.le;
    z->ke = d.ke;
    z->ke2 = d.ke2;
    z->cf = d.cf;
    z->ff = d.ff;
    z->gf = d.gf;
    z->nn = d.nn;
    z->V = d.V;
    z->w = d.w;
    z->z = d.z;
    z->r = d.r;
    z->rhs = d.rhs;
    z->sx = d.sx;
    z->e0 = d.e0;
    z->h = d.h;
    z->part = d.part;
    if (int r = upload(z->ce, z->h_ce)) return r;
    if (int r = upload(z->cb, z->h_cb)) return r;
    if (int r = upload(z->cz, z->h_cz)) return r;
    if (int r = upload(z->fe, z->h_fe)) return r;
    if (int r = upload(z->e2f_ptr, z->h_e2f_ptr)) return r;
    if (int r = upload(z->e2f_code, z->h_e2f_code)) return r;
    if (int r = upload(z->frow, z->h_frow)) return r;
    if (int r = upload(z->fcol, z->h_fcol)) return r;
    if (int r = upload(z->fval, z->h_fval)) return r;
    if (int r = upload(z->mdiag, z->h_mdiag)) return r;
    if (int r = upload(z->kdiag, z->h_kdiag)) return r;
    QH_TRY(hipDeviceSynchronize());
    z->bound = true;
    return ETPIC_OK;
}

void etpic_cotree_destroy(etpic_cotree *z) {
    if (!z) return;
    (void)hipSetDevice(z->device);
    (void)hipDeviceSynchronize();
    delete z;
}

int etpic_cotree_counts(const etpic_cotree *z, int64_t counts_out[4]) {
    if (!z || !counts_out) return qfail(ETPIC_EINVAL, "null argument");
    counts_out[0] = z->nec;
    counts_out[1] = z->nfc;
    counts_out[2] = z->nz;
    counts_out[3] = z->fnnz;
    return ETPIC_OK;
}

int etpic_cotree_apply(etpic_cotree *z, etpic_qh *qh, int block, const double *x, double *y, double tol,
                       int max_iter, void *stream) {
    if (int r = z_check(z, qh)) return r;
    if (!(tol > 0.0) || max_iter < 1) return qfail(ETPIC_EINVAL, "bad tol / max_iter");
    if (block != 11 && block != 12 && block != 13 && block != 21 && block != 22 && block != 23)
        return qfail(ETPIC_EINVAL, "block %d is not one of 11, 12, 13, 21, 22, 23", block);
    const int64_t nin = (block == 11 || block == 22) ? z->nfc : (block == 12 || block == 21) ? z->nec : z->nz;
    const int64_t nout = (block / 10 == 1) ? z->nfc : z->nec;
    if ((!x && nin > 0) || (!y && nout > 0)) return qfail(ETPIC_EINVAL, "null vector");
    QH_TRY(hipSetDevice(z->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (nout == 0) return ETPIC_OK;
    const double2 *X = reinterpret_cast<const double2 *>(x);
    double2 *Y = reinterpret_cast<double2 *>(y);
    const double2 one = make_double2(1.0, 0.0), zero = make_double2(0.0, 0.0);
    switch (block) {
    case 11:
    case 22:
        k_z_fill<<<zgrid(z->nf), kZThreads, 0, st>>>(z->nf, z->cf);
        k_z_scatter<<<zgrid(z->nfc), kZThreads, 0, st>>>(z->nfc, z->cb, X, z->cf);
        if (int r = zproj_b(qh, z->cf, z->ff, tol, max_iter, st)) return r;
        if (block == 11) {
            k_z_gather<<<zgrid(z->nfc), kZThreads, 0, st>>>(z->nfc, z->cb, one, z->ff, zero, nullptr, Y);
        } else {
            zmass_f(z, z->ff, z->gf, st);
            k_z_curlt<<<zgrid(z->ne), kZThreads, 0, st>>>(z->ne, z->e2f_ptr, z->e2f_code, z->gf, z->ke);
            k_z_gather<<<zgrid(z->nec), kZThreads, 0, st>>>(z->nec, z->ce, one, z->ke, zero, nullptr, Y);
        }
        break;
    case 12:
    case 21:
        zscatter_e(z, X, st);
        zmass_e(qh, z->ue, z->te, st);
        if (int r = zproj_e(qh, z->te, z->le, z->nn, tol, max_iter, st)) return r;
        if (block == 21) {
            k_z_gather<<<zgrid(z->nec), kZThreads, 0, st>>>(z->nec, z->ce, one, z->le, zero, nullptr, Y);
        } else {   // C (u - D E_ns)
            k_qe_dx<<<blocks_for(z->ne), kQThreads, 0, st>>>(z->ne, qh->ev, z->nn, z->ke);
            k_z_sub<<<zgrid(z->ne), kZThreads, 0, st>>>(z->ne, z->ue, z->ke, z->ke2);
            k_z_curl<<<zgrid(z->nf), kZThreads, 0, st>>>(z->nf, z->fe, z->ke2, z->cf);
            k_z_gather<<<zgrid(z->nfc), kZThreads, 0, st>>>(z->nfc, z->cb, one, z->cf, zero, nullptr, Y);
        }
        break;
    case 13:
    case 23:
        k_z_fill<<<zgrid(z->nv), kZThreads, 0, st>>>(z->nv, z->nn);
        k_z_scatter<<<zgrid(z->nz), kZThreads, 0, st>>>(z->nz, z->cz, X, z->nn);
        k_qe_dx<<<blocks_for(z->ne), kQThreads, 0, st>>>(z->ne, qh->ev, z->nn, z->ke);
        if (block == 13) {
            k_z_curl<<<zgrid(z->nf), kZThreads, 0, st>>>(z->nf, z->fe, z->ke, z->cf);
            k_z_gather<<<zgrid(z->nfc), kZThreads, 0, st>>>(z->nfc, z->cb, one, z->cf, zero, nullptr, Y);
        } else {
            zmass_e(qh, z->ke, z->te, st);
            k_z_gather<<<zgrid(z->nec), kZThreads, 0, st>>>(z->nec, z->ce, one, z->te, zero, nullptr, Y);
        }
        break;
    default:
        return qfail(ETPIC_EINVAL, "block %d is not one of 11, 12, 13, 21, 22, 23", block);
    }
    QH_TRY(hipGetLastError());
    return ETPIC_OK;
}

int etpic_cotree_b_field(etpic_cotree *z, etpic_qh *qh, const double *bs, double *b_out, double tol, int max_iter,
                         void *stream) {
    if (int r = z_check(z, qh)) return r;
    if (!bs || !b_out) return qfail(ETPIC_EINVAL, "null vector");
    if (!(tol > 0.0) || max_iter < 1) return qfail(ETPIC_EINVAL, "bad tol / max_iter");
    QH_TRY(hipSetDevice(z->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    k_z_fill<<<zgrid(z->nf), kZThreads, 0, st>>>(z->nf, z->cf);
    k_z_scatter<<<zgrid(z->nfc), kZThreads, 0, st>>>(z->nfc, z->cb, reinterpret_cast<const double2 *>(bs), z->cf);
    QH_TRY(hipGetLastError());
    return zproj_b(qh, z->cf, reinterpret_cast<double2 *>(b_out), tol, max_iter, st);
}

int etpic_cotree_step(etpic_cotree *z, etpic_qh *qh, double dt, double omega, double *b, double *es,
                      const double *src, double tol, int max_iter, double inner_tol, int inner_max, int *iters_out,
                      double *resid_out, void *stream) {
    if (int r = z_check(z, qh)) return r;
    if (!b || !es) return qfail(ETPIC_EINVAL, "null vector");
    if (!(dt > 0.0) || !std::isfinite(dt) || !std::isfinite(omega)) return qfail(ETPIC_EINVAL, "bad dt / omega");
    if (!(tol > 0.0) || max_iter < 1 || !(inner_tol > 0.0) || inner_max < 1)
        return qfail(ETPIC_EINVAL, "bad tolerances / iteration limits");
    QH_TRY(hipSetDevice(z->device));
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t nec = z->nec;
    const cplx a(1.0 / dt, 0.5 * omega), ab(1.0 / dt, -0.5 * omega);
    double2 *B = reinterpret_cast<double2 *>(b), *E = reinterpret_cast<double2 *>(es);
    if (int r = zcopy(E, z->e0, nec, st)) return r;
    // right-hand side: conj(a) Z21 E0 - C_e^T K C_e E0 / (4a) + (1 + conj(a)/a)/2 C_e^T C^T [*mu^-1] b0 + src
    zscatter_e(z, E, st);
    zmass_e(qh, z->ue, z->te, st);
    if (int r = zproj_e(qh, z->te, z->le, nullptr, inner_tol, inner_max, st)) return r;
    k_z_curl<<<zgrid(z->nf), kZThreads, 0, st>>>(z->nf, z->fe, z->ue, z->cf);
    zmass_f(z, z->cf, z->gf, st);
    k_z_curlt<<<zgrid(z->ne), kZThreads, 0, st>>>(z->ne, z->e2f_ptr, z->e2f_code, z->gf, z->ke);
    k_z_gather<<<zgrid(nec), kZThreads, 0, st>>>(nec, z->ce, d2(ab), z->le, d2(-0.25 / a), z->ke, z->rhs);
    zmass_f(z, B, z->ff, st);
    k_z_curlt<<<zgrid(z->ne), kZThreads, 0, st>>>(z->ne, z->e2f_ptr, z->e2f_code, z->ff, z->ke2);
    k_z_gather<<<zgrid(nec), kZThreads, 0, st>>>(nec, z->ce, d2(0.5 * (1.0 + ab / a)), z->ke2, make_double2(0.0, 0.0),
                                                 nullptr, z->w);
    k_z_axpy<<<zgrid(nec), kZThreads, 0, st>>>(nec, z->rhs, z->w, nullptr, nullptr, nullptr);
    if (src) k_z_axpy<<<zgrid(nec), kZThreads, 0, st>>>(nec, z->rhs, reinterpret_cast<const double2 *>(src), nullptr,
                                                      nullptr, nullptr);
    QH_TRY(hipGetLastError());
    // Ampere rows on the cotree edges (E1 from the guess E0)
    if (int r = zgmres(z, qh, a, E, tol, max_iter, inner_tol, inner_max, iters_out, resid_out, st)) return r;
    // Faraday on every face: b1 = (conj(a) b0 - C C_e (E0 + E1) / 2) / a
    if (int r = zcopy(E, z->sx, nec, st)) return r;
    k_z_axpy<<<zgrid(nec), kZThreads, 0, st>>>(nec, z->sx, z->e0, nullptr, nullptr, nullptr);
    zscatter_e(z, z->sx, st);
    k_z_curl<<<zgrid(z->nf), kZThreads, 0, st>>>(z->nf, z->fe, z->ue, z->cf);
    k_z_faraday<<<zgrid(z->nf), kZThreads, 0, st>>>(z->nf, d2(a), d2(ab), z->cf, B);
    QH_TRY(hipGetLastError());
    return ETPIC_OK;
}

}  // extern "C"
