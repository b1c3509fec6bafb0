// etpic: envelope-tracking particle-mesh step for gfx950 (MI355X).
//
// Kernels (all launched on the caller's stream):
//   k_tet_coef    per tet and step: carrier-rotated Whitney coefficients.  With
//                 lam the barycentrics, E(x) = sum_i lam_i A_i and
//                 B(x) = sum_i lam_i C_i inside a tet (both expansions are affine
//                 in lam), where A_i, C_i fold the real parts Re{dof e^{jwt}} + dc
//                 of the 6 edge and 4 face DoFs into the gradients.
//   k_step        per particle, tet-sorted: per-tet coefficients staged in LDS,
//                 gather, Boris push, in-tet path-integral deposit reduced
//                 over runs of equal tet (wave) and slots (LDS), float64
//                 atomics; particles leaving their tet are queued.
//   k_walk        the queued particles: barycentric walk, reflection, deposit.
//   k_hist/k_scan*/k_scatter   counting sort by tet.
//   k_charge      vertex charge of the particles.
//   k_gauss       continuity residual D^T dG - (rho_new - rho_old).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "etpic.h"
#include "mesh_host.hpp"

using etpic::TetTopo;

namespace {

thread_local std::string g_last_error;

int fail(int code, const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return code;
}

#define HIP_TRY(expr)                                                                         \
    do {                                                                                      \
        hipError_t e_ = (expr);                                                               \
        if (e_ != hipSuccess) return fail(ETPIC_EHIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

constexpr int kBlock = 256;
constexpr unsigned kWalkQueueCap = 1u << 22;  // blocks; bounds N_p by 2^30
constexpr unsigned kWalkBlocks = 1024;        // grid of the walk kernel

// Runs of equal key among the 64 lanes of a wavefront (particles are kept
// sorted by tet, so neighbouring lanes mostly share a key).  head: first lane
// of a run; head_lane / run_end: first and last lane of this lane's run.
struct WaveRuns {
    int lane, head_lane, run_end;
    bool head;
};

__device__ __forceinline__ WaveRuns wave_runs(int key) {
    WaveRuns r;
    r.lane = threadIdx.x & 63;
    const int prev = __shfl_up(key, 1);
    r.head = r.lane == 0 || key != prev;
    const unsigned long long hm = __ballot(r.head);
    const unsigned long long upto = r.lane == 63 ? ~0ull : ((2ull << r.lane) - 1ull);  // lanes 0..lane
    const unsigned long long after = hm & ~upto;
    r.head_lane = 63 - __clzll((long long)(hm & upto));
    r.run_end = after ? (__ffsll((unsigned long long)after) - 2) : 63;
    return r;
}

// Segmented suffix sum: after the call the head lane of each run holds the
// run's total (other lanes hold partial sums).
template <typename T>
__device__ __forceinline__ T run_total(T x, const WaveRuns &r) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const T y = __shfl_down(x, off);
        if (r.lane + off <= r.run_end) x += y;
    }
    return x;
}

// ------------------------------------------------------------------ per-tet coefficients
// W1_ij = l_i grad l_j - l_j grad l_i  =>  eps_ij W1_ij adds eps_ij grad l_j to A_i and
// -eps_ij grad l_i to A_j.  W2 of face (a<b<c) = 2(l_a gb x gc + l_b gc x ga + l_c ga x gb).
template <typename Real>
__global__ void __launch_bounds__(kBlock) k_tet_coef(int64_t nt, const TetTopo *__restrict__ topo,
                                                     const double *__restrict__ grad,
                                                     const double2 *__restrict__ e_env,
                                                     const double *__restrict__ e_dc,
                                                     const double2 *__restrict__ b_env,
                                                     const double *__restrict__ b_dc, double c, double s,
                                                     Real *__restrict__ coef) {
    int64_t T = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (T >= nt) return;
    const TetTopo tp = topo[T];
    double g[4][3];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int d = 0; d < 3; ++d) g[k][d] = grad[T * 12 + 3 * k + d];
    double A[4][3] = {}, C[4][3] = {};
    const int le[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    const int lf[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        const int i = le[e][0], j = le[e][1];
        const double2 z = e_env[tp.e[e]];
        double eps = z.x * c - z.y * s;
        if (e_dc) eps += e_dc[tp.e[e]];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            A[i][d] += eps * g[j][d];
            A[j][d] -= eps * g[i][d];
        }
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const int a = lf[f][0], b = lf[f][1], cc = lf[f][2];
        const double2 z = b_env[tp.f[f]];
        double beta = z.x * c - z.y * s;
        if (b_dc) beta += b_dc[tp.f[f]];
        beta *= 2.0;
        double x_bc[3], x_ca[3], x_ab[3];
        x_bc[0] = g[b][1] * g[cc][2] - g[b][2] * g[cc][1];
        x_bc[1] = g[b][2] * g[cc][0] - g[b][0] * g[cc][2];
        x_bc[2] = g[b][0] * g[cc][1] - g[b][1] * g[cc][0];
        x_ca[0] = g[cc][1] * g[a][2] - g[cc][2] * g[a][1];
        x_ca[1] = g[cc][2] * g[a][0] - g[cc][0] * g[a][2];
        x_ca[2] = g[cc][0] * g[a][1] - g[cc][1] * g[a][0];
        x_ab[0] = g[a][1] * g[b][2] - g[a][2] * g[b][1];
        x_ab[1] = g[a][2] * g[b][0] - g[a][0] * g[b][2];
        x_ab[2] = g[a][0] * g[b][1] - g[a][1] * g[b][0];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            C[a][d] += beta * x_bc[d];
            C[b][d] += beta * x_ca[d];
            C[cc][d] += beta * x_ab[d];
        }
    }
    Real *o = coef + T * 24;
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            o[3 * k + d] = (Real)A[k][d];
            o[12 + 3 * k + d] = (Real)C[k][d];
        }
}

// ------------------------------------------------------------------ particle step
template <typename Real>
struct StepArgs {
    int64_t n, nt;
    double *lam1, *lam2, *lam3;
    Real *v0, *v1, *v2;
    int32_t *tet;
    const double *grad;        // nt*12 float64 barycentric gradients
    const TetTopo *topo;
    double *dG;
    double *rho;
    unsigned *status;
    unsigned *walk_queue;      // blocks holding particles that left their tet
    unsigned *walk_ctr;        // [0] queue length, [1] walk blocks done
    double qw;
    Real h;                    // q dt / (2 m)
    Real dt_r;
};

// A particle that leaves its tet is marked in place (tet = -(T + 2)) by the
// step kernel, which keeps its start barycentrics and stores its new velocity;
// the block's index goes to the walk queue.  k_walk then walks it.
__device__ __forceinline__ int walker_mark(int T) { return -(T + 2); }
__device__ __forceinline__ int walker_tet(int marked) { return -marked - 2; }

// q w * path integral of the six edge functions along one straight piece inside
// a tet: with lam linear along the piece, int W1_ij . dr = m_i dl_j - m_j dl_i,
// m = lam at the midpoint, dl the barycentric increment of the piece.
__device__ __forceinline__ void deposit_piece(double *__restrict__ dG, const TetTopo &tp, const double l[4],
                                              const double dl[4], double qw) {
    double m[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) m[k] = l[k] + 0.5 * dl[k];
    const int le[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        const int i = le[e][0], j = le[e][1];
        unsafeAtomicAdd(&dG[tp.e[e]], qw * (m[i] * dl[j] - m[j] * dl[i]));
    }
}

// Walk of the straight path with Cartesian remaining displacement d, starting in
// tet T at barycentrics l.  Each piece is deposited.  At a face crossing the exit
// coordinate is set to exactly 0, the other three are rescaled to sum to one and
// handed to the neighbour's shared vertices; at a boundary face the remaining
// displacement and the velocity are reflected about the face normal.
template <typename Real>
__device__ __forceinline__ int walk(const StepArgs<Real> &a, int T, double l[4], double d[3], Real v[3]) {
    int hops = 0;
    for (;;) {
        const double *gp = a.grad + (int64_t)T * 12;
        double g[4][3];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int c = 0; c < 3; ++c) g[k][c] = gp[3 * k + c];
        double dl[4];
#pragma unroll
        for (int k = 1; k < 4; ++k) dl[k] = g[k][0] * d[0] + g[k][1] * d[1] + g[k][2] * d[2];
        dl[0] = -(dl[1] + dl[2] + dl[3]);
        double smin = 1.0;
        int kmin = -1;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (dl[k] < 0.0 && l[k] + dl[k] < 0.0) {
                const double sk = l[k] > 0.0 ? l[k] / (-dl[k]) : 0.0;
                if (kmin < 0 || sk < smin) {
                    smin = sk;
                    kmin = k;
                }
            }
        }
        const TetTopo tp = a.topo[T];
        // values at the exit face, selected without dynamic register indexing
        double gx = 0.0, gy = 0.0, gz = 0.0;
        int nb = -1;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (k == kmin) {
                gx = g[k][0];
                gy = g[k][1];
                gz = g[k][2];
                nb = tp.n[k];
            }
        if (kmin < 0) {
            deposit_piece(a.dG, tp, l, dl, a.qw);
#pragma unroll
            for (int k = 0; k < 4; ++k) l[k] += dl[k];
            break;
        }
        double dlp[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) dlp[k] = smin * dl[k];
        deposit_piece(a.dG, tp, l, dlp, a.qw);
        double lc[4], sum = 0.0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            lc[k] = (k == kmin) ? 0.0 : fmax(l[k] + dlp[k], 0.0);
            sum += lc[k];
        }
#pragma unroll
        for (int k = 0; k < 4; ++k) lc[k] /= sum;
#pragma unroll
        for (int c = 0; c < 3; ++c) d[c] -= smin * d[c];
        if (nb < 0) {
            const double nn = sqrt(gx * gx + gy * gy + gz * gz);
            const double nh[3] = {gx / nn, gy / nn, gz / nn};
            double dd = d[0] * nh[0] + d[1] * nh[1] + d[2] * nh[2];
            Real vv = v[0] * (Real)nh[0] + v[1] * (Real)nh[1] + v[2] * (Real)nh[2];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                d[c] -= 2.0 * dd * nh[c];
                v[c] -= (Real)2 * vv * (Real)nh[c];
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) l[k] = lc[k];
        } else {
            const TetTopo tn = a.topo[nb];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                double x = 0.0;
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (tp.v[i] == tn.v[j]) x = lc[i];
                l[j] = x;
            }
            T = nb;
        }
        if (++hops > ETPIC_HOP_CAP) {
            atomicOr(a.status, (unsigned)ETPIC_DEV_HOPCAP);
            break;
        }
    }
    return T;
}

// ------------------------------------------------------------------ fused staged step
// One block of kBlock threads takes kBlock consecutive particles.  Runs of equal
// tet in thread order (particles are kept sorted by tet) become "slots".  For up
// to kSlots slots at a time, 8 threads per slot build the carrier-rotated
// Whitney coefficients of that tet straight from the edge/face DoFs into LDS
// (A_k and C_k, one thread per vertex k each).  Every particle then gathers from
// LDS, pushes, and -- if it stays in its tet, which is the common case --
// deposits its six path integrals into the slot's LDS accumulators (float64
// LDS atomics).  The accumulators are flushed with one float64 global atomic
// per (slot, edge).  Particles that leave their tet walk and deposit every
// piece with global atomics.
constexpr int kSlots = 32;

template <typename Real>
struct StageLds {
    Real coef[kSlots][24];
    Real grad[kSlots][9];
    double acc[kSlots][6];
    double racc[kSlots][4];
    int32_t edge[kSlots][6];
    int32_t vert[kSlots][4];
    int32_t tet[kSlots];
    int32_t wave_last[kBlock / 64];
    int32_t wave_heads[kBlock / 64];
};

struct FieldPtrs {
    const double2 *e_env;
    const double *e_dc;
    const double2 *b_env;
    const double *b_dc;
    double c, s;   // cos(w t_n), sin(w t_n)
};

// local edge index of the vertex pair {i, j}, i < j
__device__ __forceinline__ int local_edge(int i, int j) { return i == 0 ? j - 1 : (i == 1 ? j + 1 : 5); }

template <int K, typename Real>
__device__ __forceinline__ void stage_A(StageLds<Real> &L, int s, const int32_t *tp, const double g[4][3],
                                        const FieldPtrs &F) {
    double A[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (j == K) continue;
        const int id = tp[local_edge(j < K ? j : K, j < K ? K : j)];
        const double2 z = F.e_env[id];
        double eps = z.x * F.c - z.y * F.s;
        if (F.e_dc) eps += F.e_dc[id];
        if (j < K) eps = -eps;
#pragma unroll
        for (int d = 0; d < 3; ++d) A[d] += eps * g[j][d];
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) L.coef[s][3 * K + d] = (Real)A[d];
    if (K < 3) {
#pragma unroll
        for (int d = 0; d < 3; ++d) L.grad[s][3 * K + d] = (Real)g[K + 1][d];
    } else {
#pragma unroll
        for (int e = 0; e < 6; ++e) L.edge[s][e] = tp[e];
#pragma unroll
        for (int v = 0; v < 4; ++v) L.vert[s][v] = tp[10 + v];
    }
    L.racc[s][K] = 0.0;
    L.acc[s][K] = 0.0;
}

template <int K, typename Real>
__device__ __forceinline__ void stage_C(StageLds<Real> &L, int s, const int32_t *tp, const double g[4][3],
                                        const FieldPtrs &F) {
    double Cv[3] = {0.0, 0.0, 0.0};
    constexpr int lf[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        if (f == K) continue;
        const int a = lf[f][0] == K ? lf[f][1] : (lf[f][1] == K ? lf[f][2] : lf[f][0]);
        const int b = lf[f][0] == K ? lf[f][2] : (lf[f][1] == K ? lf[f][0] : lf[f][1]);
        const int id = tp[6 + f];
        const double2 z = F.b_env[id];
        double beta = z.x * F.c - z.y * F.s;
        if (F.b_dc) beta += F.b_dc[id];
        beta *= 2.0;
        Cv[0] += beta * (g[a][1] * g[b][2] - g[a][2] * g[b][1]);
        Cv[1] += beta * (g[a][2] * g[b][0] - g[a][0] * g[b][2]);
        Cv[2] += beta * (g[a][0] * g[b][1] - g[a][1] * g[b][0]);
    }
#pragma unroll
    for (int d = 0; d < 3; ++d) L.coef[s][12 + 3 * K + d] = (Real)Cv[d];
    if (K < 2) L.acc[s][4 + K] = 0.0;
}

// Part `part` (0..7) of the coefficients of tet T into slot s:
//   part k < 4 : A_k = sum_{j != k} sign(j - k) eps_{kj} grad l_j   (E = sum_k l_k A_k)
//   part 4 + k : C_k = 2 sum_{faces f containing k} beta_f (grad l_a x grad l_b),
//                (k, a, b) the cyclic order of f's ascending triple starting at k.
// eps and beta are the real parts Re{dof e^{jwt}} + dc of the edge and face DoFs.
template <typename Real>
__device__ __forceinline__ void stage_part(StageLds<Real> &L, int s, int part, int T, const TetTopo *__restrict__ topo,
                                           const double *__restrict__ grad, const FieldPtrs &F) {
    const double *gp = grad + (int64_t)T * 12;
    double g[4][3];
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int d = 0; d < 3; ++d) g[k][d] = gp[3 * k + d];
    const int32_t *tp = reinterpret_cast<const int32_t *>(topo + T);
    switch (part) {
        case 0: stage_A<0>(L, s, tp, g, F); break;
        case 1: stage_A<1>(L, s, tp, g, F); break;
        case 2: stage_A<2>(L, s, tp, g, F); break;
        case 3: stage_A<3>(L, s, tp, g, F); break;
        case 4: stage_C<0>(L, s, tp, g, F); break;
        case 5: stage_C<1>(L, s, tp, g, F); break;
        case 6: stage_C<2>(L, s, tp, g, F); break;
        default: stage_C<3>(L, s, tp, g, F); break;
    }
}

template <typename Real>
__global__ void __launch_bounds__(kBlock) k_step(StepArgs<Real> a, FieldPtrs F, int remap) {
    __shared__ StageLds<Real> L;
    unsigned blk = blockIdx.x;
    if (remap) {
        // the dispatcher deals blocks round-robin over the 8 XCDs; give each XCD
        // one contiguous range of particles (hence of tets and edges in its L2)
        const unsigned G = gridDim.x, q = G / 8, r = G % 8, x = blk % 8, j = blk / 8;
        blk = x * q + min(x, r) + j;
    }
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int64_t p = (int64_t)blk * kBlock + tid;
    int T = -1;
    if (p < a.n) {
        T = a.tet[p];
        if ((unsigned)T >= (unsigned)a.nt) {
            atomicOr(a.status, (unsigned)ETPIC_DEV_BADTET);
            T = -1;
        }
    }
    const bool act = T >= 0;
    double l[4];
    Real v[3];
    if (act) {
        l[1] = a.lam1[p];
        l[2] = a.lam2[p];
        l[3] = a.lam3[p];
        v[0] = a.v0[p];
        v[1] = a.v1[p];
        v[2] = a.v2[p];
    }
    // runs of equal tet -> slots
    int prevT = __shfl_up(T, 1);
    if (lane == 63) L.wave_last[wid] = T;
    __syncthreads();
    if (lane == 0) prevT = wid == 0 ? -2 : L.wave_last[wid - 1];
    const bool head = act && T != prevT;
    const unsigned long long hm = __ballot(head);
    const unsigned long long upto = lane == 63 ? ~0ull : ((1ull << (lane + 1)) - 1ull);
    const int incl = __popcll(hm & upto);
    if (lane == 0) L.wave_heads[wid] = __popcll(hm);
    __syncthreads();
    int before = 0, nslot = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        const int c = L.wave_heads[w];
        before += w < wid ? c : 0;
        nslot += c;
    }
    const int slot = before + incl - 1;
    const WaveRuns runs = wave_runs(act ? slot : -1);
    int walker = 0;
    for (int lo = 0; lo < nslot; lo += kSlots) {
        const int cnt = min(kSlots, nslot - lo);
        if (head && slot >= lo && slot < lo + cnt) L.tet[slot - lo] = T;
        __syncthreads();
        {
            const int s = tid >> 3, part = tid & 7;
            if (s < cnt) stage_part<Real>(L, s, part, L.tet[s], a.topo, a.grad, F);
        }
        __syncthreads();
        const bool here = act && slot >= lo && slot < lo + cnt;
        double g6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // this lane's in-tet path integrals
        double r4[4] = {0.0, 0.0, 0.0, 0.0};             // this lane's end-point barycentrics
        if (here) {
            const int s = slot - lo;
            l[0] = 1.0 - l[1] - l[2] - l[3];
            const Real *cf = L.coef[s];
            Real E[3], B[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                E[d] = (Real)l[0] * cf[d] + (Real)l[1] * cf[3 + d] + (Real)l[2] * cf[6 + d] + (Real)l[3] * cf[9 + d];
                B[d] = (Real)l[0] * cf[12 + d] + (Real)l[1] * cf[15 + d] + (Real)l[2] * cf[18 + d] +
                       (Real)l[3] * cf[21 + d];
            }
            const Real h = a.h;
            Real vm[3], tau[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) {
                vm[d] = v[d] + h * E[d];
                tau[d] = h * B[d];
            }
            const Real t2 = tau[0] * tau[0] + tau[1] * tau[1] + tau[2] * tau[2];
            const Real sg = (Real)2 / ((Real)1 + t2);
            const Real vr[3] = {vm[0] + (vm[1] * tau[2] - vm[2] * tau[1]), vm[1] + (vm[2] * tau[0] - vm[0] * tau[2]),
                                vm[2] + (vm[0] * tau[1] - vm[1] * tau[0])};
            v[0] = vm[0] + sg * (vr[1] * tau[2] - vr[2] * tau[1]) + h * E[0];
            v[1] = vm[1] + sg * (vr[2] * tau[0] - vr[0] * tau[2]) + h * E[1];
            v[2] = vm[2] + sg * (vr[0] * tau[1] - vr[1] * tau[0]) + h * E[2];
            if (!(isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]))) atomicOr(a.status, (unsigned)ETPIC_DEV_NAN);
            const Real dx[3] = {a.dt_r * v[0], a.dt_r * v[1], a.dt_r * v[2]};
            const Real *gr = L.grad[s];
            double dl[4];
#pragma unroll
            for (int k = 1; k < 4; ++k)
                dl[k] = (double)(gr[3 * k - 3] * dx[0] + gr[3 * k - 2] * dx[1] + gr[3 * k - 1] * dx[2]);
            dl[0] = -(dl[1] + dl[2] + dl[3]);
            const bool stays = (l[0] + dl[0] >= 0.0) && (l[1] + dl[1] >= 0.0) && (l[2] + dl[2] >= 0.0) &&
                               (l[3] + dl[3] >= 0.0);
            if (stays) {
                double m[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) m[k] = l[k] + 0.5 * dl[k];
                const int le[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
#pragma unroll
                for (int e = 0; e < 6; ++e) g6[e] = m[le[e][0]] * dl[le[e][1]] - m[le[e][1]] * dl[le[e][0]];
#pragma unroll
                for (int k = 1; k < 4; ++k) l[k] += dl[k];
                a.lam1[p] = l[1];
                a.lam2[p] = l[2];
                a.lam3[p] = l[3];
                if (a.rho) {
                    r4[0] = 1.0 - l[1] - l[2] - l[3];
                    r4[1] = l[1];
                    r4[2] = l[2];
                    r4[3] = l[3];
                }
            } else {
                a.tet[p] = walker_mark(T);
                walker = 1;
            }
            a.v0[p] = v[0];
            a.v1[p] = v[1];
            a.v2[p] = v[2];
        }
        // wave-level segmented reduction over runs of equal slot, then one LDS
        // atomic per (run, edge) from the run's head lane
#pragma unroll
        for (int e = 0; e < 6; ++e) g6[e] = run_total(g6[e], runs);
        if (a.rho) {
#pragma unroll
            for (int k = 0; k < 4; ++k) r4[k] = run_total(r4[k], runs);
        }
        if (here && runs.head) {
            const int s = slot - lo;
#pragma unroll
            for (int e = 0; e < 6; ++e) unsafeAtomicAdd(&L.acc[s][e], g6[e]);
            if (a.rho) {
#pragma unroll
                for (int k = 0; k < 4; ++k) unsafeAtomicAdd(&L.racc[s][k], r4[k]);
            }
        }
        __syncthreads();
        for (int t = tid; t < cnt * 10; t += kBlock) {
            if (t < cnt * 6) {
                const int s = t / 6, e = t - 6 * s;
                const double val = L.acc[s][e];
                if (val != 0.0) unsafeAtomicAdd(&a.dG[L.edge[s][e]], a.qw * val);
            } else if (a.rho) {
                const int u = t - cnt * 6, s = u >> 2, k = u & 3;
                const double val = L.racc[s][k];
                if (val != 0.0) unsafeAtomicAdd(&a.rho[L.vert[s][k]], a.qw * val);
            }
        }
        __syncthreads();
    }
    if (__syncthreads_or(walker) && tid == 0) a.walk_queue[atomicAdd(&a.walk_ctr[0], 1u)] = blk;
}

// Walks the marked particles of the queued blocks: every piece of their path
// is deposited with global atomics, and the end point, reflected velocity and
// new tet are stored.  Blocks stride over the queue; the last block to finish
// resets the counters for the next step.
template <typename Real>
__global__ void __launch_bounds__(kBlock) k_walk(StepArgs<Real> a) {
    const unsigned count = __atomic_load_n(&a.walk_ctr[0], __ATOMIC_RELAXED);
    for (unsigned i = blockIdx.x; i < count; i += gridDim.x) {
        const int64_t p = (int64_t)a.walk_queue[i] * kBlock + threadIdx.x;
        if (p >= a.n) continue;
        const int marked = a.tet[p];
        if (marked > -2) continue;
        int T = walker_tet(marked);
        if (T >= a.nt) continue;
        double l[4];
        l[1] = a.lam1[p];
        l[2] = a.lam2[p];
        l[3] = a.lam3[p];
        l[0] = 1.0 - l[1] - l[2] - l[3];
        Real v[3] = {a.v0[p], a.v1[p], a.v2[p]};
        const Real dx[3] = {a.dt_r * v[0], a.dt_r * v[1], a.dt_r * v[2]};
        double d[3] = {(double)dx[0], (double)dx[1], (double)dx[2]};
        T = walk<Real>(a, T, l, d, v);
        a.tet[p] = T;
        a.lam1[p] = l[1];
        a.lam2[p] = l[2];
        a.lam3[p] = l[3];
        a.v0[p] = v[0];
        a.v1[p] = v[1];
        a.v2[p] = v[2];
        if (a.rho) {
            const TetTopo tp = a.topo[T];
            const double l0 = 1.0 - l[1] - l[2] - l[3];
            unsafeAtomicAdd(&a.rho[tp.v[0]], a.qw * l0);
            unsafeAtomicAdd(&a.rho[tp.v[1]], a.qw * l[1]);
            unsafeAtomicAdd(&a.rho[tp.v[2]], a.qw * l[2]);
            unsafeAtomicAdd(&a.rho[tp.v[3]], a.qw * l[3]);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&a.walk_ctr[1], 1u) == gridDim.x - 1) {
            a.walk_ctr[0] = 0u;
            a.walk_ctr[1] = 0u;
        }
    }
}

// ------------------------------------------------------------------ vertex charge
__global__ void __launch_bounds__(kBlock) k_charge(int64_t n, int64_t nt, const double *__restrict__ lam1,
                                                   const double *__restrict__ lam2, const double *__restrict__ lam3,
                                                   const int32_t *__restrict__ tet, const TetTopo *__restrict__ topo,
                                                   double qw, double *__restrict__ rho, unsigned *status) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int T = -1;
    double l[4] = {0.0, 0.0, 0.0, 0.0};
    if (p < n) {
        T = tet[p];
        if ((unsigned)T >= (unsigned)nt) {
            atomicOr(status, (unsigned)ETPIC_DEV_BADTET);
            T = -1;
        } else {
            l[1] = lam1[p];
            l[2] = lam2[p];
            l[3] = lam3[p];
            l[0] = 1.0 - l[1] - l[2] - l[3];
        }
    }
    const WaveRuns r = wave_runs(T);
#pragma unroll
    for (int k = 0; k < 4; ++k) l[k] = run_total(l[k], r);
    if (r.head && T >= 0) {
        const TetTopo tp = topo[T];
#pragma unroll
        for (int k = 0; k < 4; ++k) unsafeAtomicAdd(&rho[tp.v[k]], qw * l[k]);
    }
}

// ------------------------------------------------------------------ continuity residual
// r_k = sum_{e incident} (+dG_e if k is the head, -dG_e if the tail) - (rho_new_k - rho_old_k).
// out[0] = max |r|, out[1] = max |rho_old| as the bit patterns of non-negative doubles
// (which order like unsigned integers).
__global__ void __launch_bounds__(kBlock) k_gauss(int64_t nv, const int32_t *__restrict__ ptr,
                                                  const int32_t *__restrict__ code, const double *__restrict__ dG,
                                                  const double *__restrict__ rho_new,
                                                  const double *__restrict__ rho_old,
                                                  unsigned long long *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double r = 0.0, p = 0.0;
    if (k < nv) {
        double div = 0.0;
        for (int32_t i = ptr[k]; i < ptr[k + 1]; ++i) {
            const int32_t c = code[i];
            const double g = dG[c >> 1];
            div += (c & 1) ? g : -g;
        }
        r = fabs(div - (rho_new[k] - rho_old[k]));
        p = fabs(rho_old[k]);
    }
    // wave-level max then one atomic per wave
    for (int off = 32; off > 0; off >>= 1) {
        r = fmax(r, __shfl_xor(r, off));
        p = fmax(p, __shfl_xor(p, off));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&out[0], (unsigned long long)__double_as_longlong(r));
        atomicMax(&out[1], (unsigned long long)__double_as_longlong(p));
    }
}

// ------------------------------------------------------------------ counting sort
__global__ void __launch_bounds__(kBlock) k_fill_u32(unsigned *__restrict__ x, int64_t n, unsigned val) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = val;
}

__global__ void __launch_bounds__(kBlock) k_hist(int64_t n, int64_t nt, const int32_t *__restrict__ tet,
                                                 unsigned *__restrict__ count, unsigned *status) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int T = -1;
    if (p < n) {
        T = tet[p];
        if ((unsigned)T >= (unsigned)nt) {
            atomicOr(status, (unsigned)ETPIC_DEV_BADTET);
            T = -1;
        }
    }
    const WaveRuns r = wave_runs(T);
    if (r.head && T >= 0) atomicAdd(&count[T], (unsigned)(r.run_end - r.lane + 1));
}

constexpr int kScanTile = 1024;   // elements per block in the block-local scan (4 per thread)

// Exclusive scan of each 1024-element tile in place; tile totals to sums[].
__global__ void __launch_bounds__(kBlock) k_scan_tiles(unsigned *__restrict__ x, int64_t n,
                                                       unsigned *__restrict__ sums) {
    __shared__ unsigned s_wave[kBlock / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + threadIdx.x * 4;
    unsigned v[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) v[i] = (base + i < n) ? x[base + i] : 0u;
    unsigned tsum = v[0] + v[1] + v[2] + v[3];
    // inclusive wave scan of the thread sums
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    unsigned inc = tsum;
    for (int off = 1; off < 64; off <<= 1) {
        unsigned y = __shfl_up(inc, off);
        if (lane >= off) inc += y;
    }
    if (lane == 63) s_wave[wid] = inc;
    __syncthreads();
    unsigned wpre = 0;
    for (int w = 0; w < wid; ++w) wpre += s_wave[w];
    unsigned run = wpre + inc - tsum;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (base + i < n) x[base + i] = run;
        run += v[i];
    }
    if (threadIdx.x == kBlock - 1) sums[blockIdx.x] = wpre + inc;
}

// Exclusive scan of the (few) tile totals by a single block, looping over chunks.
__global__ void __launch_bounds__(kBlock) k_scan_sums(unsigned *__restrict__ sums, int64_t m) {
    __shared__ unsigned s_wave[kBlock / 64];
    __shared__ unsigned s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int64_t base = 0; base < m; base += kBlock) {
        const int64_t i = base + threadIdx.x;
        const unsigned v = i < m ? sums[i] : 0u;
        unsigned inc = v;
        for (int off = 1; off < 64; off <<= 1) {
            unsigned y = __shfl_up(inc, off);
            if (lane >= off) inc += y;
        }
        if (lane == 63) s_wave[wid] = inc;
        __syncthreads();
        unsigned wpre = 0;
        for (int w = 0; w < wid; ++w) wpre += s_wave[w];
        const unsigned carry = s_carry;
        if (i < m) sums[i] = carry + wpre + inc - v;
        __syncthreads();
        if (threadIdx.x == kBlock - 1) s_carry = carry + wpre + inc;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(kBlock) k_scan_add(unsigned *__restrict__ x, int64_t n,
                                                     const unsigned *__restrict__ sums) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] += sums[i / kScanTile];
}

template <typename Real>
__global__ void __launch_bounds__(kBlock) k_scatter(int64_t n, int64_t nt, const int32_t *__restrict__ tet,
                                                    unsigned *__restrict__ cursor, etpic_particles src,
                                                    etpic_particles dst) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int T = -1;
    if (p < n) {
        T = tet[p];
        if ((unsigned)T >= (unsigned)nt) T = -1;
    }
    // one cursor atomic per run of equal tet; lanes of a run keep their order
    const WaveRuns r = wave_runs(T);
    unsigned base = 0;
    if (r.head && T >= 0) base = atomicAdd(&cursor[T], (unsigned)(r.run_end - r.lane + 1));
    base = __shfl(base, r.head_lane);
    if (T < 0) return;
    const unsigned q = base + (unsigned)(r.lane - r.head_lane);
    dst.tet[q] = T;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        dst.lam[k][q] = src.lam[k][p];
        static_cast<Real *>(dst.vel[k])[q] = static_cast<const Real *>(src.vel[k])[p];
    }
    if (src.id && dst.id) dst.id[q] = src.id[p];
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

// =============================================================================== context
struct etpic_ctx {
    int device = 0;
    etpic::HostMesh host;
    bool has_mesh = false;
    TetTopo *d_topo = nullptr;
    double *d_grad64 = nullptr;
    void *d_coef = nullptr;          // nt*24 doubles (float table uses the first half)
    int32_t *d_v2e_ptr = nullptr;
    int32_t *d_v2e_code = nullptr;
    unsigned *d_status = nullptr;    // device status word
    unsigned *d_walk_queue = nullptr;  // kWalkQueueCap block indices
    unsigned *d_walk_ctr = nullptr;    // 2 counters of the walk queue
    unsigned long long *d_red = nullptr;  // 2 words for the residual maxima
    unsigned *d_count = nullptr;     // nt+1 counting-sort counters
    unsigned *d_tilesum = nullptr;   // scan tile totals
    int64_t tiles = 0;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> timing;   // recorded (start, stop) pairs
    std::vector<std::pair<hipEvent_t, hipEvent_t>> spare;    // created, unused pairs

    int timing_pair(hipEvent_t *a, hipEvent_t *b) {
        if (spare.empty()) {
            hipEvent_t x, y;
            HIP_TRY(hipEventCreate(&x));
            HIP_TRY(hipEventCreate(&y));
            spare.emplace_back(x, y);
        }
        *a = spare.back().first;
        *b = spare.back().second;
        spare.pop_back();
        timing.emplace_back(*a, *b);
        return ETPIC_OK;
    }

    template <typename Real>
    int launch_step(const etpic_particles *p, const etpic_species *sp, const etpic_fields *f, double c, double s,
                    double h, double dt, double *dG, double *rho, uint32_t flags, void *stream) {
        hipStream_t st = static_cast<hipStream_t>(stream);
        const int64_t nt = host.nt;
        StepArgs<Real> a{};
        a.n = p->n;
        a.nt = nt;
        a.lam1 = p->lam[0];
        a.lam2 = p->lam[1];
        a.lam3 = p->lam[2];
        a.v0 = static_cast<Real *>(p->vel[0]);
        a.v1 = static_cast<Real *>(p->vel[1]);
        a.v2 = static_cast<Real *>(p->vel[2]);
        a.tet = p->tet;
        a.grad = d_grad64;
        a.topo = d_topo;
        a.dG = dG;
        a.rho = rho;
        a.status = d_status;
        a.walk_queue = d_walk_queue;
        a.walk_ctr = d_walk_ctr;
        a.qw = sp->q * sp->w;
        a.h = (Real)h;
        a.dt_r = (Real)dt;
        hipEvent_t ev0 = nullptr, ev1 = nullptr;
        if (flags & ETPIC_STEP_TIMING) {
            if (int r = timing_pair(&ev0, &ev1)) return r;
            HIP_TRY(hipEventRecord(ev0, st));
        }
        FieldPtrs F{reinterpret_cast<const double2 *>(f->e_env), f->e_dc, reinterpret_cast<const double2 *>(f->b_env),
                    f->b_dc, c, s};
        k_step<Real><<<grid_for(p->n), kBlock, 0, st>>>(a, F, (flags & ETPIC_STEP_XCD_REMAP) ? 1 : 0);
        HIP_TRY(hipGetLastError());
        if (ev1) HIP_TRY(hipEventRecord(ev1, st));
        k_walk<Real><<<kWalkBlocks, kBlock, 0, st>>>(a);
        HIP_TRY(hipGetLastError());
        return ETPIC_OK;
    }


    void release() {
        (void)hipFree(d_topo);
        (void)hipFree(d_grad64);
        (void)hipFree(d_coef);
        (void)hipFree(d_v2e_ptr);
        (void)hipFree(d_v2e_code);
        (void)hipFree(d_count);
        (void)hipFree(d_tilesum);
        d_topo = nullptr;
        d_grad64 = nullptr;
        d_coef = nullptr;
        d_v2e_ptr = d_v2e_code = nullptr;
        d_count = d_tilesum = nullptr;
        has_mesh = false;
    }
};


namespace {

int set_device(const etpic_ctx *ctx) {
    HIP_TRY(hipSetDevice(ctx->device));
    return ETPIC_OK;
}

int check_particles(const etpic_ctx *ctx, const etpic_particles *p) {
    if (!p) return fail(ETPIC_EINVAL, "null particle descriptor");
    if (p->n < 0) return fail(ETPIC_EINVAL, "negative particle count");
    if (p->n > (int64_t)kWalkQueueCap * kBlock) return fail(ETPIC_EINVAL, "particle count above 2^30");
    if (p->n == 0) return ETPIC_OK;
    for (int k = 0; k < 3; ++k)
        if (!p->lam[k] || !p->vel[k]) return fail(ETPIC_EINVAL, "null particle array");
    if (!p->tet) return fail(ETPIC_EINVAL, "null tet array");
    (void)ctx;
    return ETPIC_OK;
}

}  // namespace

// =============================================================================== C ABI
extern "C" {

const char *etpic_last_error(void) { return g_last_error.c_str(); }

int etpic_create(etpic_ctx **out, int device) {
    if (!out) return fail(ETPIC_EINVAL, "null output handle");
    *out = nullptr;
    int ndev = 0;
    HIP_TRY(hipGetDeviceCount(&ndev));
    if (device < 0 || device >= ndev) return fail(ETPIC_EINVAL, "device %d not present (%d devices)", device, ndev);
    etpic_ctx *c = new etpic_ctx();
    c->device = device;
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) e = hipMalloc(&c->d_status, sizeof(unsigned));
    if (e == hipSuccess) e = hipMalloc(&c->d_red, 2 * sizeof(unsigned long long));
    if (e == hipSuccess) e = hipMalloc(&c->d_walk_queue, sizeof(unsigned) * kWalkQueueCap);
    if (e == hipSuccess) e = hipMalloc(&c->d_walk_ctr, 2 * sizeof(unsigned));
    if (e == hipSuccess) e = hipMemset(c->d_status, 0, sizeof(unsigned));
    if (e == hipSuccess) e = hipMemset(c->d_walk_ctr, 0, 2 * sizeof(unsigned));
    if (e == hipSuccess) e = hipDeviceSynchronize();
    if (e != hipSuccess) {
        (void)hipFree(c->d_status);
        (void)hipFree(c->d_red);
        (void)hipFree(c->d_walk_queue);
        (void)hipFree(c->d_walk_ctr);
        delete c;
        return fail(ETPIC_EHIP, "context setup: %s", hipGetErrorString(e));
    }
    *out = c;
    return ETPIC_OK;
}

int etpic_destroy(etpic_ctx *ctx) {
    if (!ctx) return ETPIC_OK;
    (void)hipSetDevice(ctx->device);
    (void)hipDeviceSynchronize();
    ctx->release();
    (void)hipFree(ctx->d_status);
    (void)hipFree(ctx->d_red);
    (void)hipFree(ctx->d_walk_queue);
    (void)hipFree(ctx->d_walk_ctr);
    for (auto &e : ctx->timing) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    for (auto &e : ctx->spare) {
        (void)hipEventDestroy(e.first);
        (void)hipEventDestroy(e.second);
    }
    delete ctx;
    return ETPIC_OK;
}

int etpic_mesh_upload(etpic_ctx *ctx, int64_t n_vert, const double *xyz_host, int64_t n_tet,
                      const int32_t *tet_vert_host) {
    if (!ctx) return fail(ETPIC_EINVAL, "null context");
    std::string err;
    etpic::HostMesh M;
    int rc = etpic::build_host_mesh(n_vert, xyz_host, n_tet, tet_vert_host, M, err);
    if (rc == -1) return fail(ETPIC_EINVAL, "mesh: %s", err.c_str());
    if (rc != 0) return fail(ETPIC_EMESH, "mesh: %s", err.c_str());
    if (int r = set_device(ctx)) return r;
    HIP_TRY(hipDeviceSynchronize());
    ctx->release();
    const int64_t nt = M.nt;
    HIP_TRY(hipMalloc(&ctx->d_topo, sizeof(TetTopo) * nt));
    HIP_TRY(hipMalloc(&ctx->d_grad64, sizeof(double) * 12 * nt));
    HIP_TRY(hipMalloc(&ctx->d_coef, sizeof(double) * 24 * nt));
    HIP_TRY(hipMalloc(&ctx->d_v2e_ptr, sizeof(int32_t) * (M.nv + 1)));
    HIP_TRY(hipMalloc(&ctx->d_v2e_code, sizeof(int32_t) * 2 * M.ne));
    HIP_TRY(hipMalloc(&ctx->d_count, sizeof(unsigned) * (nt + 1)));
    ctx->tiles = (nt + 1 + kScanTile - 1) / kScanTile;
    HIP_TRY(hipMalloc(&ctx->d_tilesum, sizeof(unsigned) * ctx->tiles));
    HIP_TRY(hipMemcpy(ctx->d_topo, M.topo.data(), sizeof(TetTopo) * nt, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(ctx->d_grad64, M.grad.data(), sizeof(double) * 12 * nt, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(ctx->d_v2e_ptr, M.v2e_ptr.data(), sizeof(int32_t) * (M.nv + 1), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(ctx->d_v2e_code, M.v2e_code.data(), sizeof(int32_t) * 2 * M.ne, hipMemcpyHostToDevice));
    ctx->host = std::move(M);
    ctx->has_mesh = true;
    return ETPIC_OK;
}

int etpic_mesh_canonical(int64_t n_vert, const double *xyz_host, int64_t n_tet, const int32_t *tet_vert_host,
                         int64_t counts_out[4], int32_t *edge_vert_host, int32_t *face_vert_host) {
    if (!counts_out) return fail(ETPIC_EINVAL, "null counts");
    std::string err;
    etpic::HostMesh M;
    int rc = etpic::build_host_mesh(n_vert, xyz_host, n_tet, tet_vert_host, M, err);
    if (rc == -1) return fail(ETPIC_EINVAL, "mesh: %s", err.c_str());
    if (rc != 0) return fail(ETPIC_EMESH, "mesh: %s", err.c_str());
    counts_out[0] = M.nv;
    counts_out[1] = M.ne;
    counts_out[2] = M.nf;
    counts_out[3] = M.nt;
    if (edge_vert_host) std::memcpy(edge_vert_host, M.edges.data(), sizeof(int32_t) * M.edges.size());
    if (face_vert_host) std::memcpy(face_vert_host, M.faces.data(), sizeof(int32_t) * M.faces.size());
    return ETPIC_OK;
}

int etpic_mesh_counts(const etpic_ctx *ctx, int64_t counts_out[4]) {
    if (!ctx || !counts_out) return fail(ETPIC_EINVAL, "null argument");
    if (!ctx->has_mesh) return fail(ETPIC_ESTATE, "no mesh uploaded");
    counts_out[0] = ctx->host.nv;
    counts_out[1] = ctx->host.ne;
    counts_out[2] = ctx->host.nf;
    counts_out[3] = ctx->host.nt;
    return ETPIC_OK;
}

int etpic_mesh_edges(const etpic_ctx *ctx, int32_t *edge_vert_host) {
    if (!ctx || !edge_vert_host) return fail(ETPIC_EINVAL, "null argument");
    if (!ctx->has_mesh) return fail(ETPIC_ESTATE, "no mesh uploaded");
    std::memcpy(edge_vert_host, ctx->host.edges.data(), sizeof(int32_t) * ctx->host.edges.size());
    return ETPIC_OK;
}

int etpic_mesh_faces(const etpic_ctx *ctx, int32_t *face_vert_host) {
    if (!ctx || !face_vert_host) return fail(ETPIC_EINVAL, "null argument");
    if (!ctx->has_mesh) return fail(ETPIC_ESTATE, "no mesh uploaded");
    std::memcpy(face_vert_host, ctx->host.faces.data(), sizeof(int32_t) * ctx->host.faces.size());
    return ETPIC_OK;
}

int etpic_gather_push_deposit(etpic_ctx *ctx, const etpic_particles *p, int precision, const etpic_species *sp,
                              const etpic_fields *f, int64_t step, double dt, double omega, double *dG,
                              double *rho, uint32_t flags, void *stream) {
    if (!ctx || !sp || !f || !dG) return fail(ETPIC_EINVAL, "null argument");
    if (!ctx->has_mesh) return fail(ETPIC_ESTATE, "no mesh uploaded");
    if (int r = check_particles(ctx, p)) return r;
    if (!f->e_env || !f->b_env) return fail(ETPIC_EINVAL, "null envelope DoFs");
    if (precision != ETPIC_FP64 && precision != ETPIC_MIXED) return fail(ETPIC_EINVAL, "bad precision %d", precision);
    if (!(std::isfinite(dt) && std::isfinite(omega) && sp->m != 0.0 && std::isfinite(sp->q) && std::isfinite(sp->m)))
        return fail(ETPIC_EINVAL, "non-finite dt / omega or zero mass");
    if (p->n == 0) return ETPIC_OK;
    if (int r = set_device(ctx)) return r;
    // carrier phase in float64 on the host (t_n = step*dt), argument reduced by libm
    const double t = (double)step * dt;
    const double c = std::cos(omega * t), s = std::sin(omega * t);
    const double h = sp->q * dt / (2.0 * sp->m);
    if (precision == ETPIC_FP64) return ctx->launch_step<double>(p, sp, f, c, s, h, dt, dG, rho, flags, stream);
    return ctx->launch_step<float>(p, sp, f, c, s, h, dt, dG, rho, flags, stream);
}

int etpic_vertex_charge(etpic_ctx *ctx, const etpic_particles *p, const etpic_species *sp, double *rho,
                        void *stream) {
    if (!ctx || !sp || !rho) return fail(ETPIC_EINVAL, "null argument");
    if (!ctx->has_mesh) return fail(ETPIC_ESTATE, "no mesh uploaded");
    if (int r = check_particles(ctx, p)) return r;
    if (p->n == 0) return ETPIC_OK;
    if (int r = set_device(ctx)) return r;
    k_charge<<<grid_for(p->n), kBlock, 0, static_cast<hipStream_t>(stream)>>>(
        p->n, ctx->host.nt, p->lam[0], p->lam[1], p->lam[2], p->tet, ctx->d_topo, sp->q * sp->w, rho,
        ctx->d_status);
    HIP_TRY(hipGetLastError());
    return ETPIC_OK;
}

int etpic_gauss_residual(etpic_ctx *ctx, const double *dG, const double *rho_new, const double *rho_old,
                         double out_host[2], void *stream) {
    if (!ctx || !dG || !rho_new || !rho_old || !out_host) return fail(ETPIC_EINVAL, "null argument");
    if (!ctx->has_mesh) return fail(ETPIC_ESTATE, "no mesh uploaded");
    if (int r = set_device(ctx)) return r;
    hipStream_t st = static_cast<hipStream_t>(stream);
    k_fill_u32<<<1, kBlock, 0, st>>>(reinterpret_cast<unsigned *>(ctx->d_red), 4, 0u);
    const int64_t nv = ctx->host.nv;
    k_gauss<<<grid_for(nv), kBlock, 0, st>>>(nv, ctx->d_v2e_ptr, ctx->d_v2e_code, dG, rho_new, rho_old, ctx->d_red);
    HIP_TRY(hipGetLastError());
    unsigned long long bits[2];
    HIP_TRY(hipMemcpyAsync(bits, ctx->d_red, sizeof bits, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    std::memcpy(out_host, bits, sizeof bits);
    return ETPIC_OK;
}

int etpic_sort(etpic_ctx *ctx, const etpic_particles *src, const etpic_particles *dst, int precision,
               void *stream) {
    if (!ctx || !src || !dst) return fail(ETPIC_EINVAL, "null argument");
    if (!ctx->has_mesh) return fail(ETPIC_ESTATE, "no mesh uploaded");
    if (int r = check_particles(ctx, src)) return r;
    if (int r = check_particles(ctx, dst)) return r;
    if (src->n != dst->n) return fail(ETPIC_EINVAL, "source and destination sizes differ");
    if (precision != ETPIC_FP64 && precision != ETPIC_MIXED) return fail(ETPIC_EINVAL, "bad precision %d", precision);
    if ((src->id == nullptr) != (dst->id == nullptr)) return fail(ETPIC_EINVAL, "id array given on one side only");
    for (int k = 0; k < 3; ++k)
        if (src->lam[k] == dst->lam[k] || src->vel[k] == dst->vel[k])
            return fail(ETPIC_EINVAL, "sort needs distinct source and destination buffers");
    if (src->tet == dst->tet) return fail(ETPIC_EINVAL, "sort needs distinct source and destination buffers");
    if (src->n == 0) return ETPIC_OK;
    if (int r = set_device(ctx)) return r;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t nt = ctx->host.nt, n = src->n, m = nt + 1;
    k_fill_u32<<<grid_for(m), kBlock, 0, st>>>(ctx->d_count, m, 0u);
    k_hist<<<grid_for(n), kBlock, 0, st>>>(n, nt, src->tet, ctx->d_count, ctx->d_status);
    k_scan_tiles<<<(unsigned)ctx->tiles, kBlock, 0, st>>>(ctx->d_count, m, ctx->d_tilesum);
    k_scan_sums<<<1, kBlock, 0, st>>>(ctx->d_tilesum, ctx->tiles);
    k_scan_add<<<grid_for(m), kBlock, 0, st>>>(ctx->d_count, m, ctx->d_tilesum);
    if (precision == ETPIC_FP64)
        k_scatter<double><<<grid_for(n), kBlock, 0, st>>>(n, nt, src->tet, ctx->d_count, *src, *dst);
    else
        k_scatter<float><<<grid_for(n), kBlock, 0, st>>>(n, nt, src->tet, ctx->d_count, *src, *dst);
    HIP_TRY(hipGetLastError());
    return ETPIC_OK;
}

int etpic_kernel_time(etpic_ctx *ctx, double *total_ms_out, int64_t *launches_out, int reset) {
    if (!ctx) return fail(ETPIC_EINVAL, "null context");
    if (int r = set_device(ctx)) return r;
    double total = 0.0;
    for (auto &e : ctx->timing) {
        HIP_TRY(hipEventSynchronize(e.second));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, e.first, e.second));
        total += ms;
    }
    if (total_ms_out) *total_ms_out = total;
    if (launches_out) *launches_out = (int64_t)ctx->timing.size();
    if (reset) {
        for (auto &e : ctx->timing) ctx->spare.push_back(e);
        ctx->timing.clear();
    }
    return ETPIC_OK;
}

int etpic_check(etpic_ctx *ctx, void *stream, uint32_t *device_flags) {
    if (!ctx) return fail(ETPIC_EINVAL, "null context");
    if (int r = set_device(ctx)) return r;
    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned word = 0;
    HIP_TRY(hipMemcpyAsync(&word, ctx->d_status, sizeof word, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    k_fill_u32<<<1, 64, 0, st>>>(ctx->d_status, 1, 0u);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
    if (device_flags) *device_flags = word;
    if (word & ETPIC_DEV_BADTET) return fail(ETPIC_EPARTICLE, "particle tet index out of range");
    if (word & ETPIC_DEV_HOPCAP) return fail(ETPIC_EWALK, "walk hop cap (%d) reached", ETPIC_HOP_CAP);
    if (word & ETPIC_DEV_NAN) return fail(ETPIC_ENAN, "non-finite velocity");
    return ETPIC_OK;
}

}  // extern "C"
