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
