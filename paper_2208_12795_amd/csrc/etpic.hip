// etpic: envelope-tracking particle-mesh step for gfx950 (MI355X).
//
// Kernels (all launched on the caller's stream):
//   k_tet_coef    per tet and step: carrier-rotated Whitney coefficients.  With
//                 lam the barycentrics, E(x) = sum_i lam_i A_i and
//                 B(x) = sum_i lam_i C_i inside a tet (both expansions are affine
//                 in lam), where A_i, C_i fold the real parts Re{dof e^{jwt}} + dc
//                 of the 6 edge and 4 face DoFs into the gradients; the envelope
//                 may be interpolated in time between three snapshots.
//   k_push, k_push_rho, k_push_slices
//                 per particle, tet-sorted: gather from the coefficient row,
//                 Boris push, in-tet path-integral deposit reduced over runs
//                 of equal tet in each wavefront, float64 atomics; particles
//                 leaving their tet are queued.  k_push_rho also scatters the
//                 end-point vertex charge; the sliced form gives each
//                 wavefront several consecutive 64-particle slices.
//   k_walk        the queued particles: barycentric walk, reflection, deposit.
//   k_walk_coef   the walk of a step and the next step's coefficients in one
//                 launch (multi-step calls).
//   k_push_sort, k_push_sort_slices
//                 the same particle kernels reading the particles in their old
//                 order and writing them, pushed, at their tet-sorted places
//                 (the periodic re-sort folded into a step).
//   k_hist/k_scan*/k_scatter/k_run_stat   counting sort by tet.
//   k_tet_coef_env, k_push_ds, k_walk_ds
//                 the downshifted step: complex-envelope rows per tet, the
//                 carrier-exact velocity quadrature of interpolated samples
//                 with Adams-Bashforth positions, and its walk.
//   k_charge      vertex charge of the particles.
//   k_gauss       continuity residual D^T dG - (rho_new - rho_old).
//   k_locate, k_positions   Cartesian points <-> (tet, barycentrics).
//   k_adjoint     reverse of one float64 step (gradient w.r.t. the edge envelope).
//   k_field_spmv, k_nm_*, k_cocg_*   implicit envelope field step.
//   k_ns_*        Gauss-law (non-solenoidal) field solve: CG on the nodal operator.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>
#include <array>
#include <algorithm>
#include <complex>
#include <memory>
#include <mutex>
#include <type_traits>

#include "etpic.h"
#include "field_host.hpp"
#include "mesh_host.hpp"
#include "checkpoint_host.hpp"

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
constexpr int kTimingSets = 512;             // event sets of the step-timing pool
// Internal step flag (the public flags leave bit 31 free): the particle arrays
// hold fixed-point barycentrics (ETPIC_MIXED_FIXED).
constexpr uint32_t kFlagFixed = 1u << 31;
constexpr unsigned kWalkQueueCap = 1u << 23;  // entries of each walk queue; N_p <= 64 * kWalkQueueCap
constexpr unsigned kQueueSkip = 0xffffffffu;  // particle-queue entry to skip
// grid of the walk kernel (and the walk half of k_walk_coef): the walk is
// bound by its dependent loads and atomics, not by lanes, and fewer blocks
// leave the coefficient pass more of the chip and pay fewer end-of-walk fences
constexpr unsigned kWalkBlocks = 64;
constexpr int64_t kMinPushWaves = 16384;      // 256 CUs x 64 wavefronts
constexpr int64_t kInfinityCacheBytes = (int64_t)256 << 20;
constexpr int64_t kFloatRowBytes = 48 + 64 + 48;   // float coefficient, push and geometry rows per tet

// Runs of equal key among the 64 lanes of a wavefront (particles are kept
// sorted by tet, so neighbouring lanes mostly share a key).  head: first lane
// of a run; head_lane / run_end: first and last lane of this lane's run.
struct WaveRuns {
    int lane, head_lane, run_end;
    bool head;
};

__device__ __forceinline__ WaveRuns wave_runs(int key, int lane = threadIdx.x & 63) {
    WaveRuns r;
    r.lane = lane;
    const int prev = __shfl_up(key, 1);
    r.head = r.lane == 0 || key != prev;
    const unsigned long long hm = __ballot(r.head);
    const unsigned long long upto = r.lane == 63 ? ~0ull : ((2ull << r.lane) - 1ull);  // lanes 0..lane
    const unsigned long long after = hm & ~upto;
    r.head_lane = 63 - __clzll((long long)(hm & upto));
    r.run_end = after ? (__ffsll((unsigned long long)after) - 2) : 63;
    return r;
}

// Lane value x of the DPP source selected by kCtrl (row shift or row broadcast);
// lanes whose row is off in kRowMask, or whose source is out of the row, get 0.
template <int kCtrl, int kRowMask>
__device__ __forceinline__ double dpp_get(double x) {
    const long long b = __double_as_longlong(x);
    const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffffll), kCtrl, kRowMask, 0xf, true);
    const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), kCtrl, kRowMask, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// As dpp_get, but lanes whose row is off in kRowMask keep `old` (a value the
// caller no longer needs, so its registers take the result and no zeroing
// move is issued; the caller's factor for those lanes is 0).
template <int kCtrl, int kRowMask>
__device__ __forceinline__ double dpp_get_or(double old, double x) {
    const long long b = __double_as_longlong(x), o = __double_as_longlong(old);
    const int lo = __builtin_amdgcn_update_dpp((int)(o & 0xffffffffll), (int)(b & 0xffffffffll), kCtrl, kRowMask,
                                               0xf, true);
    const int hi = __builtin_amdgcn_update_dpp((int)(o >> 32), (int)(b >> 32), kCtrl, kRowMask, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// Segmented inclusive prefix sum over the wave: after the call the LAST lane of
// each run (lane == run_end) holds the run's total.  Hillis-Steele within rows
// of 16 lanes by DPP row shifts (1, 2, 4, 8), then the row broadcasts of lane 15
// (into rows 1, 3) and lane 31 (into rows 2, 3); a lane only adds a partial sum
// whose lanes all belong to its own run, selected by a 0/1 factor rather than a
// branch.  The broadcasts leave the rows they skip holding the previous round's
// fetched partial sum (finite), which their factor 0 discards.
__device__ __forceinline__ double run_total(double x, const WaveRuns &r) {
    const int h = r.head_lane, l = r.lane;
    double t = dpp_get<0x111, 0xf>(x);                                // row_shr:1
    x = fma(t, l - 1 >= h ? 1.0 : 0.0, x);
    t = dpp_get<0x112, 0xf>(x);                                       // row_shr:2
    x = fma(t, l - 2 >= h ? 1.0 : 0.0, x);
    t = dpp_get<0x114, 0xf>(x);                                       // row_shr:4
    x = fma(t, l - 4 >= h ? 1.0 : 0.0, x);
    t = dpp_get<0x118, 0xf>(x);                                       // row_shr:8
    x = fma(t, l - 8 >= h ? 1.0 : 0.0, x);
    t = dpp_get_or<0x142, 0xa>(t, x);                                 // row_bcast:15
    x = fma(t, (l & 16) != 0 && h < (l & 48) ? 1.0 : 0.0, x);
    t = dpp_get_or<0x143, 0xc>(t, x);                                 // row_bcast:31
    x = fma(t, l >= 32 && h < 32 ? 1.0 : 0.0, x);
    return x;
}

// ------------------------------------------------------------------ per-tet coefficients
// Inside a tet both field expansions are affine in the barycentrics:
//   E = sum_k l_k A_k,  A_k = sum_{j != k} sign(j - k) eps_{kj} grad l_j
//     (from W1_ij = l_i grad l_j - l_j grad l_i, edge (i<j) oriented i -> j);
//   B = sum_k l_k C_k,  C_k = 2 sum_{faces f containing k} beta_f (grad l_a x grad l_b)
//     (from W2 of face (a<b<c) = 2(l_a gb x gc + l_b gc x ga + l_c ga x gb); (k, a, b)
//     the cyclic order of f's ascending triple starting at k).
// eps, beta: the real parts Re{dof e^{jwt}} + dc of the edge and face DoFs at this
// step.  Two threads per tet: one for A_0..3, one for C_0..3.
//
// With kSnap = 3 the envelope itself is interpolated in time between three
// snapshots at the coarse field times t_{n-1}, t_n, t_{n+1} (the quadratic
// Lagrange basis N_{n,k}, eqs. newmark_L / newmark_N, used for the particle
// fields in the Particle Push section): dof(t) = sum_k w_k dof_k with the
// weights w_k = N_{n,k}(t) of the fine step's time, then modulated as above.
struct FieldPtrs {
    const double2 *e_env[3];
    const double *e_dc;
    const double2 *b_env[3];
    const double *b_dc;
    double w[3];   // snapshot weights (kSnap = 3)
    double c, s;   // cos(w t), sin(w t) of the fine step's time
    int xcd;       // coefficient pass: one contiguous tet range per XCD
};

template <int kSnap>
__device__ __forceinline__ double2 envelope(const double2 *const env[3], const double w[3], int64_t id) {
    if (kSnap == 1) return env[0][id];
    const double2 a = env[0][id], b = env[1][id], c = env[2][id];
    return make_double2(w[0] * a.x + w[1] * b.x + w[2] * c.x, w[0] * a.y + w[1] * b.y + w[2] * c.y);
}

// local edge index of the vertex pair {i, j}, i < j
__host__ __device__ constexpr int local_edge(int i, int j) { return i == 0 ? j - 1 : (i == 1 ? j + 1 : 5); }

template <int K, int kSnap>
__device__ __forceinline__ void coef_A(const int32_t *tp, const double g[4][3], const FieldPtrs &F, double A[3]) {
    A[0] = A[1] = A[2] = 0.0;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        if (j == K) continue;
        const int id = tp[local_edge(j < K ? j : K, j < K ? K : j)];
        const double2 z = envelope<kSnap>(F.e_env, F.w, id);
        double eps = z.x * F.c - z.y * F.s;
        if (F.e_dc) eps += F.e_dc[id];
        if (j < K) eps = -eps;
#pragma unroll
        for (int d = 0; d < 3; ++d) A[d] += eps * g[j][d];
    }
}

template <int K, int kSnap>
__device__ __forceinline__ void coef_C(const int32_t *tp, const double g[4][3], const FieldPtrs &F, double Cv[3]) {
    Cv[0] = Cv[1] = Cv[2] = 0.0;
    constexpr int lf[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        if (f == K) continue;
        const int a = lf[f][0] == K ? lf[f][1] : (lf[f][1] == K ? lf[f][2] : lf[f][0]);
        const int b = lf[f][0] == K ? lf[f][2] : (lf[f][1] == K ? lf[f][0] : lf[f][1]);
        const int id = tp[6 + f];
        const double2 z = envelope<kSnap>(F.b_env, F.w, id);
        double beta = z.x * F.c - z.y * F.s;
        if (F.b_dc) beta += F.b_dc[id];
        beta *= 2.0;
        Cv[0] += beta * (g[a][1] * g[b][2] - g[a][2] * g[b][1]);
        Cv[1] += beta * (g[a][2] * g[b][0] - g[a][0] * g[b][2]);
        Cv[2] += beta * (g[a][0] * g[b][1] - g[a][1] * g[b][0]);
    }
}

// What the particle kernel reads per tet besides this step's coefficients: the
// barycentric gradients grad l_1..3 (9 reals, in the kernel's precision) and the
// six global edge ids, packed in one row so that a run's lanes touch one
// contiguous record (float64: 9 doubles + 6 int32 = 96 B; float32: 9 floats,
// one pad, 6 int32 = 64 B).
template <typename Real>
struct PushRow;
template <>
struct PushRow<double> {
    static constexpr int kStride = 12;   // doubles per row
    static constexpr int kEdges = 9;     // first edge id at this Real offset
};
template <>
struct PushRow<float> {
    static constexpr int kStride = 16;
    static constexpr int kEdges = 10;
};

// The particle step's per-step coefficient row.  Inside a tet a Whitney edge
// field is E(x) = A_0 + beta x (x - r_0) (its Jacobian is antisymmetric,
// beta = sum over edges (i<j) of eps_ij grad l_i x grad l_j, half its curl) and
// a Whitney face field is B(x) = C_0 + b (x - r_0) (its Jacobian is b times
// the identity, b = div B / 3 = (sum_k C_k . grad l_k) / 3): A_0 (3), beta (3),
// C_0 (3), b, with x - r_0 = sum_{k>0} l_k (r_k - r_0) from the static
// geometry row.  10 reals; float rows are padded to 12 (16-byte aligned).
template <typename Real>
struct CoefRow;
template <>
struct CoefRow<double> {
    static constexpr int kStride = 10;
};
template <>
struct CoefRow<float> {
    static constexpr int kStride = 12;
};

// Static per-tet geometry row: the edge vectors r_1 - r_0, r_2 - r_0, r_3 - r_0
// of the canonical vertex order (9 reals, padded to 16-byte rows).
template <typename Real>
struct GeoRow;
template <>
struct GeoRow<double> {
    static constexpr int kStride = 10;
};
template <>
struct GeoRow<float> {
    static constexpr int kStride = 12;
};

// The coefficient pass reads the float64 push row (grad l_1..3 and the edge ids;
// grad l_0 = -(grad l_1 + grad l_2 + grad l_3), the sum the mesh tables define it
// by) and the four face ids of the tet: 112 B per tet.
// The dispatcher deals consecutive blocks round-robin over the 8 XCDs; this
// renumbering gives each XCD one contiguous range of the G blocks instead, so
// the tets (and the edges and faces they share) of an XCD's blocks stay in its
// L2.  The coefficient pass takes it when an XCD's share of the field DoFs
// fits its 4 MB L2; on larger meshes the round-robin order, whose neighbouring
// chunks run at the same time on different XCDs and share lines through the
// Infinity Cache, measured faster.
__device__ __forceinline__ unsigned xcd_block(unsigned c, unsigned G) {
    const unsigned q = G / 8, r = G % 8, x = c % 8, j = c / 8;
    return x * q + min(x, r) + j;
}

template <typename Real, int kSnap, bool kCompact = false>
__device__ __forceinline__ void tet_coef(int64_t nt, const double *__restrict__ prow,
                                         const int32_t *__restrict__ tetface, const FieldPtrs &F,
                                         Real *__restrict__ coef, unsigned blk) {
    // A block covers kTets tets.  Their push rows and face ids are staged in
    // LDS with coalesced 16-byte loads; then the block's first kTets lanes
    // build A_0..3 (edges) and the other kTets lanes C_0..3 (faces), so each
    // wavefront takes one branch with all its lanes; the 24-real rows go back
    // through LDS and out with coalesced stores.  (Each lane reading its own
    // 96-byte row and writing its own 96- or 48-byte half row strides every
    // load and store instruction over 64 rows.)  Row strides in LDS are odd
    // numbers of reals, so that the lanes' rows start in different banks.
    // kCompact: the particle step's 10-real row (CoefRow: A_0 and beta from the
    // edge lanes, C_0 and b from the face lanes) instead of A_0..3, C_0..3.
    constexpr int kTets = kBlock / 2;
    constexpr int kRow = PushRow<double>::kStride + 1;   // staged push row, doubles
    constexpr int kOut = kCompact ? 11 : 25;             // staged coefficient row, Reals
    constexpr int kPart0 = kCompact ? 6 : 12, kPart1 = kCompact ? 4 : 12;   // reals from each half
    constexpr int kOutRow = kCompact ? CoefRow<Real>::kStride : 24;       // row in memory, Reals
    constexpr int kIn = kTets * kRow + kTets * 4 / 2;    // rows + face ids, in doubles
    constexpr int kOutD = (kTets * kOut * (int)sizeof(Real) + 7) / 8;
    __shared__ double lds[kIn > kOutD ? kIn : kOutD];
    const int64_t T0 = (int64_t)blk * kTets;
    if (T0 >= nt) return;   // uniform over the block
    const int nloc = (int)min<int64_t>(kTets, nt - T0);
    double *srow = lds;
    int4 *sface = reinterpret_cast<int4 *>(lds + kTets * kRow);
    {
        const double2 *src = reinterpret_cast<const double2 *>(prow + T0 * PushRow<double>::kStride);
        constexpr int kHalf = PushRow<double>::kStride / 2;   // double2 per row
        for (int i = threadIdx.x; i < nloc * kHalf; i += kBlock) {
            const double2 v = src[i];
            const int t = i / kHalf, c = 2 * (i - t * kHalf);
            srow[t * kRow + c] = v.x;
            srow[t * kRow + c + 1] = v.y;
        }
        const int4 *tf = reinterpret_cast<const int4 *>(tetface) + T0;
        for (int i = threadIdx.x; i < nloc; i += kBlock) sface[i] = tf[i];
    }
    __syncthreads();
    const int part = (int)(threadIdx.x >= kTets);
    const int t = threadIdx.x & (kTets - 1);
    double o[12];
    if (t < nloc) {
        const double *row = srow + t * kRow;
        double g[4][3];
#pragma unroll
        for (int k = 1; k < 4; ++k)
#pragma unroll
            for (int d = 0; d < 3; ++d) g[k][d] = row[3 * (k - 1) + d];
#pragma unroll
        for (int d = 0; d < 3; ++d) g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
        int32_t tp[10];   // edge ids 0..5, face ids 6..9
        const int32_t *re = reinterpret_cast<const int32_t *>(row + PushRow<double>::kEdges);
#pragma unroll
        for (int k = 0; k < 6; ++k) tp[k] = re[k];
        const int4 fc = sface[t];
        tp[6] = fc.x;
        tp[7] = fc.y;
        tp[8] = fc.z;
        tp[9] = fc.w;
        // the DoFs first, all gathers in flight together (each edge serves
        // two of the A_k, each face three of the C_k), then the sums in the
        // order and with the operations of coef_A / coef_C
        if (part == 0) {
            double ev[6];
#pragma unroll
            for (int k = 0; k < 6; ++k) {
                const double2 z = envelope<kSnap>(F.e_env, F.w, tp[k]);
                ev[k] = z.x * F.c - z.y * F.s;
            }
            if (F.e_dc)
#pragma unroll
                for (int k = 0; k < 6; ++k) ev[k] += F.e_dc[tp[k]];
            if (kCompact) {
                // A_0 = E(r_0) = sum_j eps_0j grad l_j; beta = sum_(i<j) eps_ij grad l_i x grad l_j
#pragma unroll
                for (int d = 0; d < 6; ++d) o[d] = 0.0;
#pragma unroll
                for (int j = 1; j < 4; ++j)
#pragma unroll
                    for (int d = 0; d < 3; ++d) o[d] += ev[local_edge(0, j)] * g[j][d];
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = i + 1; j < 4; ++j) {
                        const double e = ev[local_edge(i, j)];
                        o[3] += e * (g[i][1] * g[j][2] - g[i][2] * g[j][1]);
                        o[4] += e * (g[i][2] * g[j][0] - g[i][0] * g[j][2]);
                        o[5] += e * (g[i][0] * g[j][1] - g[i][1] * g[j][0]);
                    }
            } else
#pragma unroll
            for (int K = 0; K < 4; ++K) {
                double *A = o + 3 * K;
                A[0] = A[1] = A[2] = 0.0;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    if (j == K) continue;
                    double eps = ev[local_edge(j < K ? j : K, j < K ? K : j)];
                    if (j < K) eps = -eps;
#pragma unroll
                    for (int d = 0; d < 3; ++d) A[d] += eps * g[j][d];
                }
            }
        } else {
            double bv[4];
#pragma unroll
            for (int f = 0; f < 4; ++f) {
                const double2 z = envelope<kSnap>(F.b_env, F.w, tp[6 + f]);
                bv[f] = z.x * F.c - z.y * F.s;
            }
            if (F.b_dc)
#pragma unroll
                for (int f = 0; f < 4; ++f) bv[f] += F.b_dc[tp[6 + f]];
            constexpr int lf[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
#pragma unroll
            for (int K = 0; K < 4; ++K) {
                double *Cv = o + 3 * K;
                Cv[0] = Cv[1] = Cv[2] = 0.0;
#pragma unroll
                for (int f = 0; f < 4; ++f) {
                    if (f == K) continue;
                    const int a = lf[f][0] == K ? lf[f][1] : (lf[f][1] == K ? lf[f][2] : lf[f][0]);
                    const int b = lf[f][0] == K ? lf[f][2] : (lf[f][1] == K ? lf[f][0] : lf[f][1]);
                    const double beta = bv[f] * 2.0;
                    Cv[0] += beta * (g[a][1] * g[b][2] - g[a][2] * g[b][1]);
                    Cv[1] += beta * (g[a][2] * g[b][0] - g[a][0] * g[b][2]);
                    Cv[2] += beta * (g[a][0] * g[b][1] - g[a][1] * g[b][0]);
                }
            }
            if (kCompact) {
                // C_0 stays in o[0..2]; b = (sum_k C_k . grad l_k) / 3
                double dv = 0.0;
#pragma unroll
                for (int K = 0; K < 4; ++K)
#pragma unroll
                    for (int d = 0; d < 3; ++d) dv += o[3 * K + d] * g[K][d];
                o[3] = dv * (1.0 / 3.0);
            }
        }
    }
    __syncthreads();   // every staged row read: the space takes the output
    Real *sout = reinterpret_cast<Real *>(lds);
    if (t < nloc) {
        // full rows: A_k at 3k, C_k at 12 + 3k; compact rows: A_0, beta, C_0, b
        if (part == 0) {
#pragma unroll
            for (int d = 0; d < kPart0; ++d) sout[t * kOut + d] = (Real)o[d];
        } else {
#pragma unroll
            for (int d = 0; d < kPart1; ++d) sout[t * kOut + kPart0 + d] = (Real)o[d];
        }
    }
    __syncthreads();
    Real *dst = coef + T0 * kOutRow;
    for (int i = threadIdx.x; i < nloc * kOutRow; i += kBlock) {
        const int tt = i / kOutRow, c = i - tt * kOutRow;
        dst[i] = c < kPart0 + kPart1 ? sout[tt * kOut + c] : (Real)0;
    }
}

template <typename Real, int kSnap = 1, bool kCompact = false>
__global__ void __launch_bounds__(kBlock) k_tet_coef(int64_t nt, const double *__restrict__ prow,
                                                     const int32_t *__restrict__ tetface, FieldPtrs F,
                                                     Real *__restrict__ coef) {
    tet_coef<Real, kSnap, kCompact>(nt, prow, tetface, F, coef,
                                    F.xcd ? xcd_block(blockIdx.x, gridDim.x) : blockIdx.x);
}

// ------------------------------------------------------------------ particle step
template <typename Real>
__device__ __forceinline__ const int32_t *push_row_edges(const Real *row) {
    return reinterpret_cast<const int32_t *>(row + PushRow<Real>::kEdges);
}

template <typename Real>
struct StepArgs {
    int64_t n, nt;
    double *lam1, *lam2, *lam3;
    Real *v0, *v1, *v2;
    int32_t *tet;
    const Real *coef;          // nt rows of CoefRow<Real>: A_0, beta, C_0, b of this step (k_tet_coef)
    const Real *gpush;         // nt rows of PushRow<Real>::kStride: grad l_1..3, then the 6 edge ids
    const Real *geo;           // nt rows of GeoRow<Real>: r_1 - r_0, r_2 - r_0, r_3 - r_0
    const double *grad;        // nt*12 float64 barycentric gradients grad l_0..3
    const TetTopo *topo;
    double *dG;
    double *rho;
    int fixed;                 // lam1..3 hold uint32 fixed-point barycentrics (float kernels only)
    double *tetG;              // nt*8 per-tet current slots (q w * the six path-integral sums of
                               // the tet's runs), or null: the runs then add to dG directly
    unsigned *status;
    unsigned *walk_queue;      // particles that left their tet
    unsigned *slice_queue;     // 64-particle slices whose walkers did not fit in walk_queue
    unsigned *walk_ctr;        // [0] walk_queue length, [1] walk blocks done, [2] slice_queue length
    int walk_by_slice;         // queue every walker by its slice (the overflow path)
    const double *gpush64;     // float64 push rows and tet-face ids: what the
    const int32_t *tetface;    // coefficient pass of the fused launch reads
    // Counting-sort scatter fused into the step (k_push_sort): the particles
    // read from the arrays above are written, pushed, at their sorted
    // positions cursor[T]++ of these arrays; the walk after it runs on them.
    double *o_lam1, *o_lam2, *o_lam3;
    Real *o_v0, *o_v1, *o_v2;
    int32_t *o_tet;
    const int64_t *id;
    int64_t *o_id;
    unsigned *cursor;          // exclusive prefix sums of the tet counts
    int scatter;               // the walk follows a scatter step: its queue
                               // overflow is handled by a scan of all particles
    double qw;
    Real h;                    // q dt / (2 m)
    Real dt_r;
};

// A particle that leaves its tet is marked in place (tet = -(T + 2)) by the
// step kernel, which keeps its start barycentrics and stores its new velocity;
// its wavefront's index goes to the walk queue.  k_walk then walks it.
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

// lambda_0 = 1 - (l1 + l2 + l3) with the rounding error of the sum carried
// along (Knuth's two-sum).  Near face 0 lambda_0 is small, and a plainly rounded
// sum leaves it uncertain by a unit in the last place of the sum; the crossing
// parameter lambda_0 / -dlambda_0 of a path leaving through that face would
// inherit that error divided by the step's barycentric length (~1e-5).
__device__ __forceinline__ double lam0_of(double l1, double l2, double l3) {
    const double s = l1 + l2;
    const double bs = s - l1;
    double e = (l1 - (s - bs)) + (l2 - bs);
    const double t = s + l3;
    const double bt = t - s;
    e += (s - (t - bt)) + (l3 - bt);
    return (1.0 - t) - e;
}

// Fixed-point barycentrics (the compact mixed form): lambda_k = u_k * 2^-32,
// u_k uint32, lambda_0 = 1 - the sum, which is exact.  Every such number and
// every difference of two of them is exact in float64.
constexpr double kFix = 2.3283064365386962890625e-10;   // 2^-32
constexpr double kFixScale = 4294967296.0;              // 2^32

__device__ __forceinline__ double fix_to_real(uint32_t u) { return (double)u * kFix; }

// The nearest fixed-point barycentrics to (l1, l2, l3) that keep lambda_0 =
// 1 - l1 - l2 - l3 >= 0: each rounded to the nearest multiple of 2^-32 (in
// [0, 1 - 2^-32]); if the three then sum past 1 (by at most the rounding of
// the three, for a point with lambda_0 >= 0) the largest gives up the excess.
// (A point far outside the tet, which no step stores, would have the excess
// taken from the largest remaining coordinates in turn, none below zero.)
__device__ __forceinline__ void fix_round3(double l1, double l2, double l3, uint32_t u[3]) {
    const double l[3] = {l1, l2, l3};
#pragma unroll
    for (int k = 0; k < 3; ++k) u[k] = (uint32_t)fmin(fmax(rint(l[k] * kFixScale), 0.0), kFixScale - 1.0);
    const uint64_t sum = (uint64_t)u[0] + u[1] + u[2];
    if (sum > (1ull << 32)) {
        uint64_t excess = sum - (1ull << 32);
        for (int pass = 0; pass < 3 && excess > 0; ++pass) {
            const int big = (u[0] >= u[1] && u[0] >= u[2]) ? 0 : (u[1] >= u[2] ? 1 : 2);
            const uint32_t take = (uint32_t)(excess < u[big] ? excess : u[big]);
#pragma unroll
            for (int k = 0; k < 3; ++k)
                if (k == big) u[k] -= take;
            excess -= take;
        }
    }
}

// Barycentric k of particle p from an array of either storage.
__device__ __forceinline__ double lam_at(const double *arr, int64_t p, int fixed) {
    return fixed ? fix_to_real(reinterpret_cast<const uint32_t *>(arr)[p]) : arr[p];
}

// Walk of the straight path with Cartesian remaining displacement d, starting in
// tet T at barycentrics l (l[0] is recomputed from l[1..3] by lam0_of).  Each piece is deposited.  At a face crossing the exit
// coordinate is set to exactly 0, the other three are rescaled to sum to one and
// handed to the neighbour's shared vertices; at a boundary face the remaining
// displacement and the velocity are reflected about the face normal.
// With kTrack (used by the adjoint) nothing is deposited and R accumulates the
// linear part of the step's reflections (R <- (I - 2 n n^T) R per wall hit):
// the end point is R (x + dt v) + const and the stored velocity is R v.
// kExtra further vectors ext[0..kExtra-1] (the velocity samples a multistep
// integrator keeps) are reflected with the velocity at a wall.
// With `fixed` the end point is rounded to the fixed-point barycentrics (as
// fix_round3) and the last piece runs to that rounded point, so that the
// deposit and the stored end point agree exactly.
template <typename Real, bool kTrack, int kExtra = 0>
__device__ __forceinline__ int walk(const StepArgs<Real> &a, int T, double l[4], double d[3], Real v[3], double *R,
                                   double (*ext)[3] = nullptr, bool fixed = false) {
    int hops = 0;
    l[0] = lam0_of(l[1], l[2], l[3]);
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
            if (fixed) {
                uint32_t u[3];
                fix_round3(l[1] + dl[1], l[2] + dl[2], l[3] + dl[3], u);
                double lq[4];
#pragma unroll
                for (int k = 1; k < 4; ++k) lq[k] = fix_to_real(u[k - 1]);
                lq[0] = 1.0 - lq[1] - lq[2] - lq[3];
#pragma unroll
                for (int k = 0; k < 4; ++k) dl[k] = lq[k] - l[k];
            }
            if (!kTrack) deposit_piece(a.dG, tp, l, dl, a.qw);
#pragma unroll
            for (int k = 0; k < 4; ++k) l[k] += dl[k];
            break;
        }
        double dlp[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) dlp[k] = smin * dl[k];
        if (!kTrack) deposit_piece(a.dG, tp, l, dlp, a.qw);
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
            for (int i = 0; i < kExtra; ++i) {
                const double xv = ext[i][0] * nh[0] + ext[i][1] * nh[1] + ext[i][2] * nh[2];
#pragma unroll
                for (int c = 0; c < 3; ++c) ext[i][c] -= 2.0 * xv * nh[c];
            }
            if (kTrack) {
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    const double col = nh[0] * R[j] + nh[1] * R[3 + j] + nh[2] * R[6 + j];
#pragma unroll
                    for (int i = 0; i < 3; ++i) R[3 * i + j] -= 2.0 * nh[i] * col;
                }
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


// q w * (the run's path-integral sums) onto the six edges of tet T, and
// q w * (its end-point barycentric sums) onto the four vertices if rho is kept.
template <typename Real, bool kRho, bool kSlots = false>
__device__ __forceinline__ void flush_run(const StepArgs<Real> &a, int T, const double g6[6], const double r4[4]) {
    if (kSlots) {
        double *slot = a.tetG + (int64_t)T * 8;
#pragma unroll
        for (int e = 0; e < 6; ++e)
            if (g6[e] != 0.0) unsafeAtomicAdd(&slot[e], a.qw * g6[e]);
    } else {
        const int32_t *ed = push_row_edges(a.gpush + (int64_t)T * PushRow<Real>::kStride);
#pragma unroll
        for (int e = 0; e < 6; ++e)
            if (g6[e] != 0.0) unsafeAtomicAdd(&a.dG[ed[e]], a.qw * g6[e]);
    }
    if (kRho) {
        const TetTopo *tp = a.topo + T;
#pragma unroll
        for (int k = 0; k < 4; ++k)
            if (r4[k] != 0.0) unsafeAtomicAdd(&a.rho[tp->v[k]], a.qw * r4[k]);
    }
}

// The six edge sums of the runs that end in this wavefront, added by the last
// six lanes of each run together (lane run_end - k adds local edge k, its sum
// fetched from the run's last lane): the wavefront issues one atomic
// instruction where the run-end lanes alone would issue six.  The run-end
// lanes hand their six sums over through a wavefront-private LDS row (three
// 16-byte stores, one 8-byte load per flushing lane), which costs fewer
// vector instructions than five 64-bit lane shuffles and their selects.  With kSlots the
// sums go to the run's per-tet current slots (8 * T + k: the six lanes of a
// run address one 64-byte line), else to the six edges.  A run shorter than
// six lanes leaves its remaining edges to its last lane.  `flush` marks the
// run-end lanes whose run is complete (the others stay open).
template <typename Real, bool kSlots>
__device__ __forceinline__ void flush_runs_together(const StepArgs<Real> &a, int T, const double g6[6],
                                                   const WaveRuns &r, bool flush) {
    __shared__ double2 s_sum[kBlock / 64][64 * 3];
    const int wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const unsigned long long fm = __ballot(flush);
    const bool mine = (fm >> r.run_end) & 1ull;
    const int k = r.run_end - r.lane;
    const int len = r.run_end - r.head_lane + 1;
    if (flush) {
        double2 *row = &s_sum[wv][3 * r.lane];
        row[0] = make_double2(g6[0], g6[1]);
        row[1] = make_double2(g6[2], g6[3]);
        row[2] = make_double2(g6[4], g6[5]);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    double val = 0.0;
    if (mine && k < 6 && k < len) {
        const double *sr = reinterpret_cast<const double *>(&s_sum[wv][3 * r.run_end]);
        val = sr[k];
        if (kSlots) {
            double *slot = a.tetG + (int64_t)T * 8;
            if (val != 0.0) unsafeAtomicAdd(&slot[k], a.qw * val);
            if (k == 0 && len < 6) {
                for (int j = len; j < 6; ++j)
                    if (g6[j] != 0.0) unsafeAtomicAdd(&slot[j], a.qw * g6[j]);
            }
        } else {
            const int32_t *ed = push_row_edges(a.gpush + (int64_t)T * PushRow<Real>::kStride);
            if (val != 0.0) unsafeAtomicAdd(&a.dG[ed[k]], a.qw * val);
            if (k == 0 && len < 6) {
                for (int j = len; j < 6; ++j)
                    if (g6[j] != 0.0) unsafeAtomicAdd(&a.dG[ed[j]], a.qw * g6[j]);
            }
        }
    }
}

// The per-tet current slots of a multi-step call added to the edges: dG[e] +=
// the slots that name edge e, in the fixed order of the edge's CSR (no atomics:
// every particle and walk kernel of the call has finished).  The same launch
// clears the other slot buffer, which the next call accumulates into.
__global__ void __launch_bounds__(kBlock) k_slots_to_edges(int64_t ne, const int32_t *__restrict__ ptr,
                                                           const int32_t *__restrict__ slot,
                                                           const double *__restrict__ tetG, double *__restrict__ dG,
                                                           double *__restrict__ clear, int64_t nclear) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ne; e += stride) {
        double s = 0.0;
        for (int32_t i = ptr[e]; i < ptr[e + 1]; ++i) s += tetG[slot[i]];
        if (s != 0.0) dG[e] += s;
    }
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nclear; i += stride) clear[i] = 0.0;
}


// ------------------------------------------------------------------ particle step
// One lane per particle, particles kept sorted by tet.  Each lane reads its
// tet's row of this step's coefficient table (lanes of a run share the row, so
// the loads coalesce), gathers E and B, applies the Boris update and, if the
// particle stays in its tet (the common case), computes the six in-tet path
// integrals.  These are summed over each run of equal tet within the
// wavefront (segmented scan by DPP lane moves); the run's last lane
// adds the sums to the edges with float64 global atomics.  There are no block
// barriers, so latency is hidden by occupancy alone.  Particles that leave
// their tet are marked and their 64-particle slice queued for k_walk.
//
// A wavefront handles kSlices consecutive slices of 64 particles.  With more
// than one, the run that reaches lane 63 stays open: its sums are parked in
// LDS and taken over by lane 0 of the next slice if the tet continues, so a
// tet holding thousands of particles is flushed a few times instead of once
// per wavefront (same-address atomics from many wavefronts serialise).  With
// about one wavefront's worth of particles per tet or fewer, one slice per
// wavefront keeps more wavefronts in flight and is faster.
// Whether a particle kernel adds its runs' sums to the per-tet current slots
// (added to the edges once per call) or straight to the edges: the slots cost
// one cache line per run instead of six, which pays in every form except the
// float64 kernels with several slices per wavefront, where the slot path's
// registers spill (measured: float64 4-slice kernel 1.20 -> 1.24 ms).
template <typename Real>
constexpr __host__ __device__ bool push_uses_slots(int slices) {
    return std::is_same<Real, float>::value || slices == 1;
}

// Element ln of a wavefront-uniform array: the scalar base plus a 32-bit byte
// offset, which the global loads and stores take as such (base in scalar
// registers, one offset register shared by every array of the same element
// size) instead of a 64-bit address per array and lane.
template <typename T>
__device__ __forceinline__ T *lane_at(T *base, unsigned ln) {
    return reinterpret_cast<T *>(reinterpret_cast<char *>(base) + ln * (unsigned)sizeof(T));
}

template <typename Real, int kSlices, bool kRho, bool kScatter = false, bool kFixed = false, bool kPipe = false>
__device__ __forceinline__ void push_slices(const StepArgs<Real> &a, int remap) {
    static_assert(!kFixed || std::is_same<Real, float>::value, "fixed-point barycentrics are a mixed-form storage");
    unsigned blk = blockIdx.x;
    if (remap) {
        // the dispatcher deals blocks round-robin over the 8 XCDs; give each XCD
        // one contiguous range of particles (hence of tets and edges in its L2)
        const unsigned G = gridDim.x, q = G / 8, r = G % 8, x = blk % 8, j = blk / 8;
        blk = x * q + min(x, r) + j;
    }
    // wv is the same in all lanes; readfirstlane tells the compiler so, which
    // keeps the slice loop and the per-slice array bases in scalar registers
    const int lane = threadIdx.x & 63, wv = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t first = ((int64_t)blk * (kBlock / 64) + wv) * kSlices;
    // the run still open at the end of the previous slice: its tet (wave-uniform)
    // and its sums, parked in LDS by lane 63 (6 path integrals, 4 barycentrics)
    __shared__ double s_carry[kBlock / 64][10];
    int carry_T = -1;
    // kPipe: the next slice's tet and state are requested before this slice's
    // tet rows, so that the rows' round trip overlaps those loads
    int nT = -1;
    double nl1 = 0.0, nl2 = 0.0, nl3 = 0.0;
    uint32_t nu1 = 0, nu2 = 0, nu3 = 0;
    Real nv0 = 0, nv1 = 0, nv2 = 0;
    auto fetch = [&](int64_t sl) {
        const int64_t bb = sl * 64;
        unsigned lq = lane;
        asm volatile("" : "+v"(lq));
        __builtin_assume(lq < 64u);
        nT = -1;
        if (bb + lq < a.n) {
            nT = __builtin_nontemporal_load(lane_at(a.tet + bb, lq));
            if (kFixed) {
                nu1 = __builtin_nontemporal_load(lane_at(reinterpret_cast<uint32_t *>(a.lam1) + bb, lq));
                nu2 = __builtin_nontemporal_load(lane_at(reinterpret_cast<uint32_t *>(a.lam2) + bb, lq));
                nu3 = __builtin_nontemporal_load(lane_at(reinterpret_cast<uint32_t *>(a.lam3) + bb, lq));
            } else {
                nl1 = __builtin_nontemporal_load(lane_at(a.lam1 + bb, lq));
                nl2 = __builtin_nontemporal_load(lane_at(a.lam2 + bb, lq));
                nl3 = __builtin_nontemporal_load(lane_at(a.lam3 + bb, lq));
            }
            nv0 = __builtin_nontemporal_load(lane_at(a.v0 + bb, lq));
            nv1 = __builtin_nontemporal_load(lane_at(a.v1 + bb, lq));
            nv2 = __builtin_nontemporal_load(lane_at(a.v2 + bb, lq));
        }
    };
    if (kPipe) fetch(first);
#pragma unroll 1
    for (int it = 0; it < kSlices; ++it) {
        const int64_t slice = first + it;
        if (slice * 64 >= a.n) break;
        // per-slice bases are wave-uniform: every array is addressed as a
        // scalar base plus the lane offset; the lane index is re-materialised in
        // every slice, so that the compiler does not keep per-lane addresses
        // alive across the loop.  The particle state is streamed with
        // non-temporal loads and stores, which leaves the caches to the per-tet
        // rows, the field DoFs and the current accumulator.
        const int64_t b0 = slice * 64;
        unsigned ln = lane;
        asm volatile("" : "+v"(ln));
        __builtin_assume(ln < 64u);
        const int64_t p = b0 + ln;
        double *__restrict__ lam1 = a.lam1 + b0, *__restrict__ lam2 = a.lam2 + b0, *__restrict__ lam3 = a.lam3 + b0;
        Real *__restrict__ v0 = a.v0 + b0, *__restrict__ v1 = a.v1 + b0, *__restrict__ v2 = a.v2 + b0;
        int32_t *__restrict__ tetp = a.tet + b0;
        // With one slice per wavefront the whole particle state is requested at
        // once, before the tet index is back: one HBM round trip instead of tet,
        // then barycentrics and rows, then velocities (the compiler issues them in
        // that order when they sit behind the tet test).  The sliced forms keep
        // the later loads: the extra live registers cost them more than the
        // round trip (measured on both).
        constexpr bool kEarly = kSlices == 1 || kPipe;
        constexpr bool kSlots = kPipe || push_uses_slots<Real>(kSlices);
        // the compact mixed form: barycentrics stored as uint32 fixed point
        constexpr bool fx = kFixed;
        uint32_t *__restrict__ f1 = reinterpret_cast<uint32_t *>(a.lam1) + b0;
        uint32_t *__restrict__ f2 = reinterpret_cast<uint32_t *>(a.lam2) + b0;
        uint32_t *__restrict__ f3 = reinterpret_cast<uint32_t *>(a.lam3) + b0;
        int T = -1;
        double sl1 = 0.0, sl2 = 0.0, sl3 = 0.0;
        uint32_t su1 = 0, su2 = 0, su3 = 0;
        Real sv0 = 0, sv1 = 0, sv2 = 0;
        auto load_state = [&]() {
            if (fx) {
                su1 = __builtin_nontemporal_load(lane_at(f1, ln));
                su2 = __builtin_nontemporal_load(lane_at(f2, ln));
                su3 = __builtin_nontemporal_load(lane_at(f3, ln));
            } else {
                sl1 = __builtin_nontemporal_load(lane_at(lam1, ln));
                sl2 = __builtin_nontemporal_load(lane_at(lam2, ln));
                sl3 = __builtin_nontemporal_load(lane_at(lam3, ln));
            }
            sv0 = __builtin_nontemporal_load(lane_at(v0, ln));
            sv1 = __builtin_nontemporal_load(lane_at(v1, ln));
            sv2 = __builtin_nontemporal_load(lane_at(v2, ln));
        };
        if (kPipe) {
            T = nT;
            sl1 = nl1;
            sl2 = nl2;
            sl3 = nl3;
            su1 = nu1;
            su2 = nu2;
            su3 = nu3;
            sv0 = nv0;
            sv1 = nv1;
            sv2 = nv2;
            if (it + 1 < kSlices) fetch(slice + 1);
        }
        if (p < a.n) {
            if (!kPipe) {
                T = __builtin_nontemporal_load(lane_at(tetp, ln));
                if (kEarly) load_state();
            }
            if ((unsigned)T >= (unsigned)a.nt) {
                atomicOr(a.status, (unsigned)ETPIC_DEV_BADTET);
                T = -1;
            }
        }
        const bool act = T >= 0;
        // scatter form: this lane's sorted position, from one cursor atomic
        // per run of equal tet (the lanes of a run keep their order)
        unsigned dq = 0;
        if (kScatter) {
            const WaveRuns r = wave_runs(T, ln);
            unsigned base = 0;
            if (r.head && act) base = atomicAdd(&a.cursor[T], (unsigned)(r.run_end - r.lane + 1));
            base = __shfl(base, r.head_lane);
            dq = base + (unsigned)(r.lane - r.head_lane);
        }
        double g6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};   // this lane's in-tet path integrals
        double r4[4] = {0.0, 0.0, 0.0, 0.0};             // this lane's end-point barycentrics
        int walker = 0;
        if (act) {
            double l[4];
            if (!kEarly) load_state();
            if (fx) {
                sl1 = fix_to_real(su1);
                sl2 = fix_to_real(su2);
                sl3 = fix_to_real(su3);
            }
            l[1] = sl1;
            l[2] = sl2;
            l[3] = sl3;
            l[0] = 1.0 - l[1] - l[2] - l[3];
            Real v[3] = {sv0, sv1, sv2};
            // E = A_0 + beta x u, B = C_0 + b u at u = x - r_0 = sum_{k>0} l_k (r_k - r_0)
            const Real *cf = a.coef + (int64_t)T * CoefRow<Real>::kStride;
            const Real *gm = a.geo + (int64_t)T * GeoRow<Real>::kStride;
            const Real x1 = (Real)l[1], x2 = (Real)l[2], x3 = (Real)l[3];
            Real u[3];
#pragma unroll
            for (int d = 0; d < 3; ++d) u[d] = x1 * gm[d] + x2 * gm[3 + d] + x3 * gm[6 + d];
            Real E[3], B[3];
            E[0] = cf[0] + (cf[4] * u[2] - cf[5] * u[1]);
            E[1] = cf[1] + (cf[5] * u[0] - cf[3] * u[2]);
            E[2] = cf[2] + (cf[3] * u[1] - cf[4] * u[0]);
#pragma unroll
            for (int d = 0; d < 3; ++d) B[d] = cf[6 + d] + cf[9] * u[d];
            // Boris: half kick, rotation (implicit midpoint in v x B), half kick
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
            // displacement and barycentric increments; lam0 is stored implicitly
            // (1 - lam1 - lam2 - lam3), so its increment is minus the sum of the
            // other three, in float64: deposit and stored end point see the same
            // four increments (continuity to float64 rounding)
            const Real dx[3] = {a.dt_r * v[0], a.dt_r * v[1], a.dt_r * v[2]};
            const Real *gr = a.gpush + (int64_t)T * PushRow<Real>::kStride;
            double dl[4];
#pragma unroll
            for (int k = 1; k < 4; ++k)
                dl[k] = (double)(gr[3 * k - 3] * dx[0] + gr[3 * k - 2] * dx[1] + gr[3 * k - 1] * dx[2]);
            dl[0] = -(dl[1] + dl[2] + dl[3]);
            const bool stays = (l[0] + dl[0] >= 0.0) && (l[1] + dl[1] >= 0.0) && (l[2] + dl[2] >= 0.0) &&
                               (l[3] + dl[3] >= 0.0);
            if (stays) {
                // compact form: the end point rounded to the fixed-point grid, and
                // the piece taken to that point, so that deposit and stored end
                // point agree exactly (the differences are exact in float64)
                uint32_t un[3] = {0, 0, 0};
                if (fx) {
                    fix_round3(l[1] + dl[1], l[2] + dl[2], l[3] + dl[3], un);
                    dl[1] = ((double)un[0] - (double)su1) * kFix;
                    dl[2] = ((double)un[1] - (double)su2) * kFix;
                    dl[3] = ((double)un[2] - (double)su3) * kFix;
                    dl[0] = -(dl[1] + dl[2] + dl[3]);
                }
                // path integral of W1_ij along the straight piece: m_i dl_j - m_j dl_i,
                // m the midpoint barycentrics (exact: the integrand is affine on the piece)
                double m[4];
#pragma unroll
                for (int k = 0; k < 4; ++k) m[k] = l[k] + 0.5 * dl[k];
                constexpr int le[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
#pragma unroll
                for (int e = 0; e < 6; ++e) g6[e] = m[le[e][0]] * dl[le[e][1]] - m[le[e][1]] * dl[le[e][0]];
#pragma unroll
                for (int k = 1; k < 4; ++k) l[k] += dl[k];
                if (kScatter) {
                    if (fx) {
                        __builtin_nontemporal_store(un[0], reinterpret_cast<uint32_t *>(a.o_lam1) + dq);
                        __builtin_nontemporal_store(un[1], reinterpret_cast<uint32_t *>(a.o_lam2) + dq);
                        __builtin_nontemporal_store(un[2], reinterpret_cast<uint32_t *>(a.o_lam3) + dq);
                    } else {
                        __builtin_nontemporal_store(l[1], &a.o_lam1[dq]);
                        __builtin_nontemporal_store(l[2], &a.o_lam2[dq]);
                        __builtin_nontemporal_store(l[3], &a.o_lam3[dq]);
                    }
                    a.o_tet[dq] = T;
                } else if (fx) {
                    __builtin_nontemporal_store(un[0], lane_at(f1, ln));
                    __builtin_nontemporal_store(un[1], lane_at(f2, ln));
                    __builtin_nontemporal_store(un[2], lane_at(f3, ln));
                } else {
                    __builtin_nontemporal_store(l[1], lane_at(lam1, ln));
                    __builtin_nontemporal_store(l[2], lane_at(lam2, ln));
                    __builtin_nontemporal_store(l[3], lane_at(lam3, ln));
                }
                if (kRho) {
                    r4[0] = 1.0 - l[1] - l[2] - l[3];
                    r4[1] = l[1];
                    r4[2] = l[2];
                    r4[3] = l[3];
                }
            } else if (kScatter) {
                // the walk starts from the old barycentrics at the new position
                if (fx) {
                    reinterpret_cast<uint32_t *>(a.o_lam1)[dq] = su1;
                    reinterpret_cast<uint32_t *>(a.o_lam2)[dq] = su2;
                    reinterpret_cast<uint32_t *>(a.o_lam3)[dq] = su3;
                } else {
                    a.o_lam1[dq] = l[1];
                    a.o_lam2[dq] = l[2];
                    a.o_lam3[dq] = l[3];
                }
                a.o_tet[dq] = walker_mark(T);
                walker = 1;
            } else {
                *lane_at(tetp, ln) = walker_mark(T);
                walker = 1;
            }
            if (kScatter) {
                __builtin_nontemporal_store(v[0], &a.o_v0[dq]);
                __builtin_nontemporal_store(v[1], &a.o_v1[dq]);
                __builtin_nontemporal_store(v[2], &a.o_v2[dq]);
                if (a.id) __builtin_nontemporal_store(__builtin_nontemporal_load(&a.id[p]), &a.o_id[dq]);
            } else {
                __builtin_nontemporal_store(v[0], lane_at(v0, ln));
                __builtin_nontemporal_store(v[1], lane_at(v1, ln));
                __builtin_nontemporal_store(v[2], lane_at(v2, ln));
            }
        }
        const WaveRuns runs = wave_runs(T, ln);
        // the open run continues into this slice: lane 0 takes over its sums;
        // otherwise it is complete and flushed now
        if (kSlices > 1 && carry_T >= 0) {
            __builtin_amdgcn_wave_barrier();
            if (ln == 0) {
                double cg[6], cr[4];
#pragma unroll
                for (int e = 0; e < 6; ++e) cg[e] = s_carry[wv][e];
#pragma unroll
                for (int k = 0; k < 4; ++k) cr[k] = s_carry[wv][6 + k];
                if (T == carry_T) {
#pragma unroll
                    for (int e = 0; e < 6; ++e) g6[e] += cg[e];
#pragma unroll
                    for (int k = 0; k < 4; ++k) r4[k] += cr[k];
                } else {
                    flush_run<Real, kRho, kPipe || push_uses_slots<Real>(kSlices)>(a, carry_T, cg, cr);
                }
            }
        }
        // segmented reduction over runs of equal tet; the run's last lane holds
        // its sums and adds them to HBM, except for the run reaching lane 63,
        // which stays open for the next slice
#pragma unroll
        for (int e = 0; e < 6; ++e) g6[e] = run_total(g6[e], runs);
        if (kRho) {
#pragma unroll
            for (int k = 0; k < 4; ++k) r4[k] = run_total(r4[k], runs);
        }
        const bool last = it == kSlices - 1 || (slice + 1) * 64 >= a.n;
        const bool flush = act && runs.lane == runs.run_end && (ln != 63 || last);
        if (kRho) {
            if (flush) flush_run<Real, kRho, kSlots>(a, T, g6, r4);
        } else {
            flush_runs_together<Real, kSlots>(a, T, g6, runs, flush);
        }
        if (!last) {
            carry_T = __builtin_amdgcn_readlane(T, 63);
            if (ln == 63) {
#pragma unroll
                for (int e = 0; e < 6; ++e) s_carry[wv][e] = g6[e];
#pragma unroll
                for (int k = 0; k < 4; ++k) s_carry[wv][6 + k] = r4[k];
            }
        }
        // walkers go to the particle queue (one atomic per wavefront); a
        // wavefront whose walkers do not all fit queues its slice instead
        const unsigned long long wmask = __ballot(walker);
        if (wmask) {
            const unsigned cnt = (unsigned)__popcll(wmask);
            unsigned base = 0;
            if (ln == 0) base = atomicAdd(&a.walk_ctr[0], cnt);
            base = __shfl(base, 0);
            const bool fits = (kScatter || !a.walk_by_slice) && base < kWalkQueueCap && cnt <= kWalkQueueCap - base;
            const unsigned rank = (unsigned)__popcll(wmask & ((1ull << ln) - 1ull));
            if (walker && base + rank < kWalkQueueCap)
                a.walk_queue[base + rank] = fits ? (kScatter ? dq : (unsigned)p) : kQueueSkip;
            // (after a scatter step the walkers of a slice are spread over the
            // output, so an overflow there makes the walk scan every particle)
            if (!kScatter && !fits && ln == 0) a.slice_queue[atomicAdd(&a.walk_ctr[2], 1u)] = (unsigned)slice;
        }
    }
}

// One slice per wavefront; without the vertex charge the kernel fits 64 VGPRs
// (8 wavefronts per SIMD), which the compiler does not choose by itself.
template <typename Real>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(7))) k_push(StepArgs<Real> a, int remap) {
    push_slices<Real, 1, false>(a, remap);
}

template <typename Real>
__global__ void __launch_bounds__(kBlock) k_push_rho(StepArgs<Real> a, int remap) {
    push_slices<Real, 1, true>(a, remap);
}

// The particle kernel's HBM access pattern and nothing else, to measure the
// streaming rate that pattern can reach: the same launch shape (one lane per
// particle, 64-particle slices, XCD-contiguous block ranges), the same
// non-temporal loads of tet, lambda_1..3 and v and non-temporal stores of
// lambda_1..3 and v back in place.  Each stored value is the loaded one plus
// zero times the tet index (zero is a run-time argument), so the particle
// state is left as it was and no load can be dropped.
template <typename Real>
__global__ void __launch_bounds__(kBlock) k_stream(int64_t n, double *__restrict__ lam1, double *__restrict__ lam2,
                                                   double *__restrict__ lam3, Real *__restrict__ v0,
                                                   Real *__restrict__ v1, Real *__restrict__ v2,
                                                   const int32_t *__restrict__ tet, double zero, int remap, int fixed) {
    unsigned blk = blockIdx.x;
    if (remap) blk = xcd_block(blk, gridDim.x);
    const int64_t p = (int64_t)blk * kBlock + threadIdx.x;
    if (p >= n) return;
    const double z = zero * (double)__builtin_nontemporal_load(&tet[p]);
    const Real a = __builtin_nontemporal_load(&v0[p]), b = __builtin_nontemporal_load(&v1[p]),
               c = __builtin_nontemporal_load(&v2[p]);
    if (fixed) {
        uint32_t *u1 = reinterpret_cast<uint32_t *>(lam1), *u2 = reinterpret_cast<uint32_t *>(lam2),
                 *u3 = reinterpret_cast<uint32_t *>(lam3);
        const uint32_t zi = (uint32_t)z;
        const uint32_t k1 = __builtin_nontemporal_load(&u1[p]), k2 = __builtin_nontemporal_load(&u2[p]),
                       k3 = __builtin_nontemporal_load(&u3[p]);
        __builtin_nontemporal_store(k1 + zi, &u1[p]);
        __builtin_nontemporal_store(k2 + zi, &u2[p]);
        __builtin_nontemporal_store(k3 + zi, &u3[p]);
    } else {
        const double l1 = __builtin_nontemporal_load(&lam1[p]), l2 = __builtin_nontemporal_load(&lam2[p]),
                     l3 = __builtin_nontemporal_load(&lam3[p]);
        __builtin_nontemporal_store(l1 + z, &lam1[p]);
        __builtin_nontemporal_store(l2 + z, &lam2[p]);
        __builtin_nontemporal_store(l3 + z, &lam3[p]);
    }
    __builtin_nontemporal_store(a + (Real)z, &v0[p]);
    __builtin_nontemporal_store(b + (Real)z, &v1[p]);
    __builtin_nontemporal_store(c + (Real)z, &v2[p]);
}

template <typename Real, int kSlices, bool kRho>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(7)))
k_push_slices(StepArgs<Real> a, int remap) {
    push_slices<Real, kSlices, kRho>(a, remap);
}

// The same kernels reading the particles in their old order and writing them,
// pushed, to their tet-sorted positions: the counting sort's scatter pass
// folded into the step.
template <typename Real, bool kRho>
__global__ void __launch_bounds__(kBlock) k_push_sort(StepArgs<Real> a, int remap) {
    push_slices<Real, 1, kRho, true>(a, remap);
}

template <typename Real, int kSlices, bool kRho>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(7)))
k_push_sort_slices(StepArgs<Real> a, int remap) {
    push_slices<Real, kSlices, kRho, true>(a, remap);
}

// Two slices per wavefront with the second slice's state requested before the
// first one's tet rows are read (float forms; in float64 the form needs 80
// VGPRs, six wavefronts per SIMD, and measured no gain worth it).  Chosen where
// the mesh's float rows outgrow the Infinity Cache, so that a wavefront's row
// reads are HBM round trips: there the state loads of one slice overlap the
// row round trip of the other.
template <bool kFixed>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(7)))
k_push_pipe(StepArgs<float> a, int remap) {
    push_slices<float, 2, false, false, kFixed, true>(a, remap);
}

// The compact mixed form (barycentrics stored as uint32 fixed point): the same
// kernels with that storage compiled in.
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(7)))
k_push_fixed(StepArgs<float> a, int remap) {
    push_slices<float, 1, false, false, true>(a, remap);
}

__global__ void __launch_bounds__(kBlock) k_push_rho_fixed(StepArgs<float> a, int remap) {
    push_slices<float, 1, true, false, true>(a, remap);
}

template <int kSlices, bool kRho>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(7)))
k_push_slices_fixed(StepArgs<float> a, int remap) {
    push_slices<float, kSlices, kRho, false, true>(a, remap);
}

template <bool kRho>
__global__ void __launch_bounds__(kBlock) k_push_sort_fixed(StepArgs<float> a, int remap) {
    push_slices<float, 1, kRho, true, true>(a, remap);
}

template <int kSlices, bool kRho>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(7)))
k_push_sort_slices_fixed(StepArgs<float> a, int remap) {
    push_slices<float, kSlices, kRho, true, true>(a, remap);
}

// Walk of one marked particle p: every piece of its path is deposited with
// global atomics, and the end point, reflected velocity and new tet are stored.
template <typename Real>
__device__ __forceinline__ void walk_particle(const StepArgs<Real> &a, int64_t p) {
    const int marked = a.tet[p];
    if (marked > -2) return;
    int T = walker_tet(marked);
    if (T >= a.nt) return;
    const bool fx = std::is_same<Real, float>::value && a.fixed;
    uint32_t *fl[3] = {reinterpret_cast<uint32_t *>(a.lam1), reinterpret_cast<uint32_t *>(a.lam2),
                       reinterpret_cast<uint32_t *>(a.lam3)};
    double l[4];
    if (fx) {
        l[1] = fix_to_real(fl[0][p]);
        l[2] = fix_to_real(fl[1][p]);
        l[3] = fix_to_real(fl[2][p]);
    } else {
        l[1] = a.lam1[p];
        l[2] = a.lam2[p];
        l[3] = a.lam3[p];
    }
    l[0] = 1.0 - l[1] - l[2] - l[3];
    Real v[3] = {a.v0[p], a.v1[p], a.v2[p]};
    const Real dx[3] = {a.dt_r * v[0], a.dt_r * v[1], a.dt_r * v[2]};
    double d[3] = {(double)dx[0], (double)dx[1], (double)dx[2]};
    T = walk<Real, false>(a, T, l, d, v, nullptr, nullptr, fx);
    a.tet[p] = T;
    if (fx) {
        // the walk ended on the fixed-point grid (rounding leaves such a point
        // as it is; a walk stopped at the hop cap is rounded onto the grid)
        uint32_t u[3];
        fix_round3(l[1], l[2], l[3], u);
        fl[0][p] = u[0];
        fl[1][p] = u[1];
        fl[2][p] = u[2];
    } else {
        a.lam1[p] = l[1];
        a.lam2[p] = l[2];
        a.lam3[p] = l[3];
    }
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

// Walks the queued particles, one lane each, then the particles of the
// overflow slices, one wavefront per slice.  The last block to finish resets
// the counters for the next step.
template <typename Real, typename WalkOne>
__device__ __forceinline__ void walk_queued(const StepArgs<Real> &a, unsigned blk, unsigned nblk, WalkOne walk_one) {
    const unsigned total = __atomic_load_n(&a.walk_ctr[0], __ATOMIC_RELAXED);
    if (a.scatter && (a.walk_by_slice || total > kWalkQueueCap)) {
        // after a scatter step whose walkers did not all fit in the queue:
        // every marked particle, found by a scan (one lane per particle)
        for (int64_t p = (int64_t)blk * kBlock + threadIdx.x; p < a.n; p += (int64_t)nblk * kBlock)
            walk_one(p);
    } else {
        const unsigned count = min(total, kWalkQueueCap);
        for (unsigned i = blk * kBlock + threadIdx.x; i < count; i += nblk * kBlock) {
            const unsigned q = a.walk_queue[i];
            if (q != kQueueSkip && (int64_t)q < a.n) walk_one((int64_t)q);
        }
        const unsigned slices = __atomic_load_n(&a.walk_ctr[2], __ATOMIC_RELAXED);
        const unsigned wpb = kBlock / 64;
        for (unsigned i = blk * wpb + (threadIdx.x >> 6); i < slices; i += nblk * wpb) {
            const int64_t p = (int64_t)a.slice_queue[i] * 64 + (threadIdx.x & 63);
            if (p < a.n) walk_one(p);
        }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        if (atomicAdd(&a.walk_ctr[1], 1u) == nblk - 1) {
            a.walk_ctr[0] = 0u;
            a.walk_ctr[1] = 0u;
            a.walk_ctr[2] = 0u;
        }
    }
}

template <typename Real>
__global__ void __launch_bounds__(kBlock) k_walk(StepArgs<Real> a) {
    walk_queued(a, blockIdx.x, gridDim.x, [&](int64_t p) { walk_particle(a, p); });
}

// The walk of one step and the coefficient pass of the next in one launch:
// blocks [0, kWalkBlocks) walk, the others build the next step's table.  The
// walk does not read the table and the table pass reads nothing the walk
// writes, so the two halves are independent; one launch saves the kernel
// boundary between them and lets the short, latency-bound walk hide behind
// the table pass.  (Used inside multi-step calls, where the next step's
// fields are known.)
template <typename Real, int kSnap>
__global__ void __launch_bounds__(kBlock) k_walk_coef(StepArgs<Real> a, int64_t nt, FieldPtrs F) {
    if (blockIdx.x < kWalkBlocks)
        walk_queued(a, blockIdx.x, kWalkBlocks, [&](int64_t p) { walk_particle(a, p); });
    else
        tet_coef<Real, kSnap, true>(nt, a.gpush64, a.tetface, F, const_cast<Real *>(a.coef),
                              F.xcd ? xcd_block(blockIdx.x - kWalkBlocks, gridDim.x - kWalkBlocks)
                                    : blockIdx.x - kWalkBlocks);
}

// ------------------------------------------------------------------ downshifted step
// The Particle Push section's other scheme: the velocity update integrates the
// carrier exactly against the envelope fields and velocities sampled along the
// trajectory and interpolated in time (Lagrange basis N_k on the nodes t_n,
// t_{n-1}, t_{n-2}):
//   v^{n+1} = v^n + q/m sum_k (Re E_k M^r_k + Im E_k M^i_k + Edc_k P_k)
//           + q/m sum_{j,k} v^{n-j} x (Re B_k L^r_jk + Im B_k L^i_jk + Bdc_k Q_jk),
// the positions advance by the Adams-Bashforth stencil in the velocities
// (eq. newtons), and the path is walked and deposited as in the fine-step
// scheme.  The weights M, L, P, Q of a step are computed on the host.
//
// The envelope samples need the complex per-tet coefficients (Re, Im and dc
// parts separately, the carrier being applied by the weights): rows of 72
// reals per tet, A_re, A_im, A_dc, C_re, C_im, C_dc, each 4 x 3 (A_k at 3k),
// built once per call since the fields are fixed within it.
constexpr int kEnvRow = 72;

__global__ void __launch_bounds__(kBlock) k_tet_coef_env(int64_t nt, const double *__restrict__ prow,
                                                         const int32_t *__restrict__ tetface, FieldPtrs F,
                                                         double *__restrict__ out) {
    // blockIdx.y: 0..2 the edge rows (Re, Im, dc), 3..5 the face rows
    const int part = blockIdx.y;
    const int64_t T = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (T >= nt) return;
    const double *row = prow + T * PushRow<double>::kStride;
    double g[4][3];
#pragma unroll
    for (int k = 1; k < 4; ++k)
#pragma unroll
        for (int d = 0; d < 3; ++d) g[k][d] = row[3 * (k - 1) + d];
#pragma unroll
    for (int d = 0; d < 3; ++d) g[0][d] = -(g[1][d] + g[2][d] + g[3][d]);
    int32_t tp[10];
    const int32_t *re = reinterpret_cast<const int32_t *>(row + PushRow<double>::kEdges);
#pragma unroll
    for (int k = 0; k < 6; ++k) tp[k] = re[k];
#pragma unroll
    for (int k = 0; k < 4; ++k) tp[6 + k] = tetface[4 * T + k];
    // the same expansions as the per-step coefficients, with (c, s) selecting
    // the real part (1, 0), the imaginary part (0, -1) or neither (0, 0), and
    // the dc DoFs kept only for the dc rows
    const int which = part % 3;
    FieldPtrs G = F;
    G.c = which == 0 ? 1.0 : 0.0;
    G.s = which == 1 ? -1.0 : 0.0;
    if (which != 2) {
        G.e_dc = nullptr;
        G.b_dc = nullptr;
    }
    double o[12];
    if (part < 3) {
        coef_A<0, 1>(tp, g, G, o);
        coef_A<1, 1>(tp, g, G, o + 3);
        coef_A<2, 1>(tp, g, G, o + 6);
        coef_A<3, 1>(tp, g, G, o + 9);
    } else {
        coef_C<0, 1>(tp, g, G, o);
        coef_C<1, 1>(tp, g, G, o + 3);
        coef_C<2, 1>(tp, g, G, o + 6);
        coef_C<3, 1>(tp, g, G, o + 9);
    }
    double *dst = out + T * kEnvRow + 12 * part;
#pragma unroll
    for (int d = 0; d < 12; ++d) dst[d] = o[d];
}

// History of the downshifted integrator: 48 arrays of length n in one
// caller-owned buffer (float64, or float32 in the mixed form), array i at
// hist + i * n.  Arrays 0..11: velocity ring,
// v^m in slot m mod 4 (components 3 slot + c); 12..29: E samples, the sample of
// step m in slot m mod 2 (12 + 9 slot + i, i = Re 0..2, Im 3..5, dc 6..8);
// 30..47: B samples likewise.
constexpr int kDsArrays = 48;

// Weights of one step, in float64 on the host.
struct DsWeights {
    double Mr[3], Mi[3], P[3], Lr[9], Li[9], Q[9];
    double ab[4];             // Adams-Bashforth coefficients times the step
};

template <typename Real>
struct DsArgs {
    const double *coef_env;   // nt * kEnvRow
    Real *hist;
    int64_t stride;           // n
    int vin[3];               // ring slots of v^{n-1}, v^{n-2}, v^{n-3} (-1: not used)
    int vout;                 // slot that receives v^n
    int sin_[2];              // sample slots of t_{n-1}, t_{n-2} (-1: not used)
    int sout;                 // slot that receives the sample of t_n
    int K, A;                 // interpolation nodes, Adams-Bashforth order
    Real Mr[3], Mi[3], P[3], Lr[9], Li[9], Q[9];
    Real ab[4];
    Real qm;
    int edc;                  // dc edge DoFs given (else the E dc samples are 0 and not stored)
};

template <typename Real>
__device__ __forceinline__ Real *ds_v(const DsArgs<Real> &d, int slot, int c) { return d.hist + (3 * slot + c) * d.stride; }
template <typename Real>
__device__ __forceinline__ Real *ds_e(const DsArgs<Real> &d, int slot, int i) { return d.hist + (12 + 9 * slot + i) * d.stride; }
template <typename Real>
__device__ __forceinline__ Real *ds_b(const DsArgs<Real> &d, int slot, int i) { return d.hist + (30 + 9 * slot + i) * d.stride; }

// Real = double: the float64 form.  Real = float: samples, velocities and the
// velocity update in float32, positions, the barycentric increments and the
// deposit in float64 (the mixed form of the fine-step kernel).
// (at most 128 VGPRs: 4 wavefronts per SIMD, which the float32 form does not
// reach by itself)
template <typename Real, bool kRho>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(4)))
k_push_ds(StepArgs<Real> a, DsArgs<Real> d, int remap) {
    unsigned blk = blockIdx.x;
    if (remap) {
        const unsigned G = gridDim.x, q = G / 8, r = G % 8, x = blk % 8, j = blk / 8;
        blk = x * q + min(x, r) + j;
    }
    const int ln = threadIdx.x & 63;
    const int64_t p = (int64_t)blk * kBlock + threadIdx.x;
    const int64_t slice = p >> 6;
    int T = -1;
    if (p < a.n) {
        T = a.tet[p];
        if ((unsigned)T >= (unsigned)a.nt) {
            atomicOr(a.status, (unsigned)ETPIC_DEV_BADTET);
            T = -1;
        }
    }
    const bool act = T >= 0;
    double g6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    double r4[4] = {0.0, 0.0, 0.0, 0.0};
    int walker = 0;
    if (act) {
        double l[4];
        l[1] = a.lam1[p];
        l[2] = a.lam2[p];
        l[3] = a.lam3[p];
        l[0] = 1.0 - l[1] - l[2] - l[3];
        // samples at t_n: sum_k lam_k of the tet's rows
        const double *row = d.coef_env + (int64_t)T * kEnvRow;
        const Real lr[4] = {(Real)l[0], (Real)l[1], (Real)l[2], (Real)l[3]};
        Real S[6][3];   // E re, im, dc; B re, im, dc
#pragma unroll
        for (int part = 0; part < 3; ++part)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                S[part][c] = (part == 2 && !d.edc)
                                 ? (Real)0
                                 : lr[0] * (Real)row[12 * part + c] + lr[1] * (Real)row[12 * part + 3 + c] +
                                       lr[2] * (Real)row[12 * part + 6 + c] + lr[3] * (Real)row[12 * part + 9 + c];
        Real V[4][3];
        V[0][0] = a.v0[p];
        V[0][1] = a.v1[p];
        V[0][2] = a.v2[p];
#pragma unroll
        for (int j = 0; j < 3; ++j)
#pragma unroll
            for (int c = 0; c < 3; ++c) V[j + 1][c] = d.vin[j] >= 0 ? ds_v(d, d.vin[j], c)[p] : (Real)0;
        Real acc[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) acc[c] = S[0][c] * d.Mr[0] + S[1][c] * d.Mi[0] + S[2][c] * d.P[0];
#pragma unroll
        for (int k = 1; k < 3; ++k) {
            if (k >= d.K) break;
            const int sl = d.sin_[k - 1];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                acc[c] += ds_e(d, sl, c)[p] * d.Mr[k] + ds_e(d, sl, 3 + c)[p] * d.Mi[k];
                if (d.edc) acc[c] += ds_e(d, sl, 6 + c)[p] * d.P[k];
            }
        }
        // the B rows are gathered only now: keeping the compiler from hoisting
        // all 72 row values ahead of use halves the live registers (4
        // wavefronts per SIMD instead of 2)
        asm volatile("" ::: "memory");
#pragma unroll
        for (int part = 3; part < 6; ++part)
#pragma unroll
            for (int c = 0; c < 3; ++c)
                S[part][c] = lr[0] * (Real)row[12 * part + c] + lr[1] * (Real)row[12 * part + 3 + c] +
                             lr[2] * (Real)row[12 * part + 6 + c] + lr[3] * (Real)row[12 * part + 9 + c];
        // magnetic part: sum_k (weighted B sample k) crossed with each v^{n-j}
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (k >= d.K) break;
            Real Bk[3][3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                if (k == 0) {
                    Bk[0][c] = S[3][c];
                    Bk[1][c] = S[4][c];
                    Bk[2][c] = S[5][c];
                } else {
                    const int sl = d.sin_[k - 1];
                    Bk[0][c] = ds_b(d, sl, c)[p];
                    Bk[1][c] = ds_b(d, sl, 3 + c)[p];
                    Bk[2][c] = ds_b(d, sl, 6 + c)[p];
                }
            }
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                if (j >= d.K) break;
                const int jk = j * d.K + k;
                Real Bw[3];
#pragma unroll
                for (int c = 0; c < 3; ++c) Bw[c] = Bk[0][c] * d.Lr[jk] + Bk[1][c] * d.Li[jk] + Bk[2][c] * d.Q[jk];
                acc[0] += V[j][1] * Bw[2] - V[j][2] * Bw[1];
                acc[1] += V[j][2] * Bw[0] - V[j][0] * Bw[2];
                acc[2] += V[j][0] * Bw[1] - V[j][1] * Bw[0];
            }
        }
        Real vn[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) vn[c] = V[0][c] + d.qm * acc[c];
        if (!(isfinite(vn[0]) && isfinite(vn[1]) && isfinite(vn[2]))) atomicOr(a.status, (unsigned)ETPIC_DEV_NAN);
        // history of the next steps: v^n and the samples of t_n
#pragma unroll
        for (int c = 0; c < 3; ++c) ds_v(d, d.vout, c)[p] = V[0][c];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            ds_e(d, d.sout, c)[p] = S[0][c];
            ds_e(d, d.sout, 3 + c)[p] = S[1][c];
            if (d.edc) ds_e(d, d.sout, 6 + c)[p] = S[2][c];
            ds_b(d, d.sout, c)[p] = S[3][c];
            ds_b(d, d.sout, 3 + c)[p] = S[4][c];
            ds_b(d, d.sout, 6 + c)[p] = S[5][c];
        }
        // Adams-Bashforth displacement and its barycentric increments (in
        // float64, the four summing to zero as in the fine-step kernel)
        Real dx[3] = {0, 0, 0};
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            if (i >= d.A) break;
#pragma unroll
            for (int c = 0; c < 3; ++c) dx[c] += d.ab[i] * V[i][c];
        }
        const Real *gr = a.gpush + (int64_t)T * PushRow<Real>::kStride;
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
            constexpr int le[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
#pragma unroll
            for (int e = 0; e < 6; ++e) g6[e] = m[le[e][0]] * dl[le[e][1]] - m[le[e][1]] * dl[le[e][0]];
#pragma unroll
            for (int k = 1; k < 4; ++k) l[k] += dl[k];
            a.lam1[p] = l[1];
            a.lam2[p] = l[2];
            a.lam3[p] = l[3];
            if (kRho) {
                r4[0] = 1.0 - l[1] - l[2] - l[3];
                r4[1] = l[1];
                r4[2] = l[2];
                r4[3] = l[3];
            }
        } else {
            a.tet[p] = walker_mark(T);
            walker = 1;
        }
        a.v0[p] = vn[0];
        a.v1[p] = vn[1];
        a.v2[p] = vn[2];
    }
    const WaveRuns runs = wave_runs(T, ln);
#pragma unroll
    for (int e = 0; e < 6; ++e) g6[e] = run_total(g6[e], runs);
    if (kRho) {
#pragma unroll
        for (int k = 0; k < 4; ++k) r4[k] = run_total(r4[k], runs);
    }
    if (act && runs.lane == runs.run_end) flush_run<Real, kRho>(a, T, g6, r4);
    // walkers to the particle queue, or their slice when it is full
    const unsigned long long wmask = __ballot(walker);
    if (wmask) {
        const unsigned cnt = (unsigned)__popcll(wmask);
        unsigned base = 0;
        if (ln == 0) base = atomicAdd(&a.walk_ctr[0], cnt);
        base = __shfl(base, 0);
        const bool fits = !a.walk_by_slice && base < kWalkQueueCap && cnt <= kWalkQueueCap - base;
        const unsigned rank = (unsigned)__popcll(wmask & ((1ull << ln) - 1ull));
        if (walker && base + rank < kWalkQueueCap) a.walk_queue[base + rank] = fits ? (unsigned)p : kQueueSkip;
        if (!fits && ln == 0) a.slice_queue[atomicAdd(&a.walk_ctr[2], 1u)] = (unsigned)slice;
    }
}

// Walk of a marked particle of a downshifted step: the Adams-Bashforth
// displacement is rebuilt from the ring (v^n is in its slot by now, the older
// samples are untouched), and at a wall the velocity samples the next steps
// use (v^n, v^{n-1}, v^{n-2}) are mirrored with v^{n+1}.
template <typename Real>
__device__ __forceinline__ void walk_particle_ds(const StepArgs<Real> &a, const DsArgs<Real> &d, int64_t p) {
    const int marked = a.tet[p];
    if (marked > -2) return;
    int T = walker_tet(marked);
    if (T >= a.nt) return;
    double l[4];
    l[1] = a.lam1[p];
    l[2] = a.lam2[p];
    l[3] = a.lam3[p];
    l[0] = 1.0 - l[1] - l[2] - l[3];
    int slot[4] = {d.vout, d.vin[0], d.vin[1], d.vin[2]};
    Real V[4][3];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) V[i][c] = slot[i] >= 0 ? ds_v(d, slot[i], c)[p] : (Real)0;
    // the particle kernel's displacement, in the same arithmetic
    Real dx[3] = {0, 0, 0};
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (i >= d.A) break;
#pragma unroll
        for (int c = 0; c < 3; ++c) dx[c] += d.ab[i] * V[i][c];
    }
    double dd[3] = {(double)dx[0], (double)dx[1], (double)dx[2]};
    double ext[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int c = 0; c < 3; ++c) ext[i][c] = (double)V[i][c];
    Real v[3] = {a.v0[p], a.v1[p], a.v2[p]};
    T = walk<Real, false, 3>(a, T, l, dd, v, nullptr, ext);
    a.tet[p] = T;
    a.lam1[p] = l[1];
    a.lam2[p] = l[2];
    a.lam3[p] = l[3];
    a.v0[p] = v[0];
    a.v1[p] = v[1];
    a.v2[p] = v[2];
#pragma unroll
    for (int i = 0; i < 3; ++i)
        if (slot[i] >= 0)
#pragma unroll
            for (int c = 0; c < 3; ++c) ds_v(d, slot[i], c)[p] = (Real)ext[i][c];
    if (a.rho) {
        const TetTopo tp = a.topo[T];
        const double l0 = 1.0 - l[1] - l[2] - l[3];
        unsafeAtomicAdd(&a.rho[tp.v[0]], a.qw * l0);
        unsafeAtomicAdd(&a.rho[tp.v[1]], a.qw * l[1]);
        unsafeAtomicAdd(&a.rho[tp.v[2]], a.qw * l[2]);
        unsafeAtomicAdd(&a.rho[tp.v[3]], a.qw * l[3]);
    }
}

template <typename Real>
__global__ void __launch_bounds__(kBlock) k_walk_ds(StepArgs<Real> a, DsArgs<Real> d) {
    walk_queued(a, blockIdx.x, gridDim.x, [&](int64_t p) { walk_particle_ds(a, d, p); });
}

// ------------------------------------------------------------------ adjoint step
// Reverse of one float64 step for every particle, given the state before the
// step (recomputed from a checkpoint) and the adjoints of the state after it.
// Recomputes gather, Boris and the walk's reflections, then back-propagates:
//   x_{k+1} = R (x_k + dt v+) + const, v_{k+1} = R v+         (walk, reflections R)
//   v+ = Boris(v_k, E, B)                                        (vjp written out)
//   E = sum_i l_i(x) A_i, B = sum_i l_i(x) C_i                  (affine in x)
// and accumulates the gradient with respect to the complex edge envelope,
// dL/dRe e_e + j dL/dIm e_e = (Ebar . W1_e(x_k)) e^{-j w t_k}, reduced over runs
// of equal tet before the float64 atomics.
struct AdjArgs {
    const double *lam1, *lam2, *lam3;
    const double *v0, *v1, *v2;
    const int32_t *tet;
    double *vb0, *vb1, *vb2;
    double *xb0, *xb1, *xb2;
    double *grad_e;
    double c, s, dt;
};

__global__ void __launch_bounds__(kBlock) k_adjoint(StepArgs<double> a, AdjArgs b) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int T = -1;
    if (p < a.n) {
        T = b.tet[p];
        if ((unsigned)T >= (unsigned)a.nt) {
            atomicOr(a.status, (unsigned)ETPIC_DEV_BADTET);
            T = -1;
        }
    }
    double ge[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) ge[k] = 0.0;
    if (T >= 0) {
        double l[4];
        l[1] = b.lam1[p];
        l[2] = b.lam2[p];
        l[3] = b.lam3[p];
        l[0] = 1.0 - l[1] - l[2] - l[3];
        const double v[3] = {b.v0[p], b.v1[p], b.v2[p]};
        const double *cf = a.coef + (int64_t)T * 24;
        double E[3], B[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            E[d] = l[0] * cf[d] + l[1] * cf[3 + d] + l[2] * cf[6 + d] + l[3] * cf[9 + d];
            B[d] = l[0] * cf[12 + d] + l[1] * cf[15 + d] + l[2] * cf[18 + d] + l[3] * cf[21 + d];
        }
        const double h = a.h;
        double vm[3], tau[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            vm[d] = v[d] + h * E[d];
            tau[d] = h * B[d];
        }
        const double t2 = tau[0] * tau[0] + tau[1] * tau[1] + tau[2] * tau[2];
        const double den = 1.0 + t2;
        const double sg = 2.0 / den;
        const double vr[3] = {vm[0] + (vm[1] * tau[2] - vm[2] * tau[1]), vm[1] + (vm[2] * tau[0] - vm[0] * tau[2]),
                              vm[2] + (vm[0] * tau[1] - vm[1] * tau[0])};
        double out[3];
        out[0] = vm[0] + sg * (vr[1] * tau[2] - vr[2] * tau[1]) + h * E[0];
        out[1] = vm[1] + sg * (vr[2] * tau[0] - vr[0] * tau[2]) + h * E[1];
        out[2] = vm[2] + sg * (vr[0] * tau[1] - vr[1] * tau[0]) + h * E[2];
        // reflections of this step (identity unless the particle left its tet)
        double R[9] = {1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0, 0.0, 1.0};
        const double dx[3] = {a.dt_r * out[0], a.dt_r * out[1], a.dt_r * out[2]};
        const double *gp = a.grad + (int64_t)T * 12;
        double g[4][3];
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int d = 0; d < 3; ++d) g[k][d] = gp[3 * k + d];
        {
            const double *gr = a.gpush + (int64_t)T * PushRow<double>::kStride;
            double dl[4];
#pragma unroll
            for (int k = 1; k < 4; ++k) dl[k] = gr[3 * k - 3] * dx[0] + gr[3 * k - 2] * dx[1] + gr[3 * k - 1] * dx[2];
            dl[0] = -(dl[1] + dl[2] + dl[3]);
            const bool stays = (l[0] + dl[0] >= 0.0) && (l[1] + dl[1] >= 0.0) && (l[2] + dl[2] >= 0.0) &&
                               (l[3] + dl[3] >= 0.0);
            if (!stays) {
                double lw[4] = {l[0], l[1], l[2], l[3]};
                double dw[3] = {dx[0], dx[1], dx[2]};
                double vw[3] = {out[0], out[1], out[2]};
                walk<double, true>(a, T, lw, dw, vw, R);
            }
        }
        const double xb[3] = {b.xb0[p], b.xb1[p], b.xb2[p]};
        const double vb[3] = {b.vb0[p], b.vb1[p], b.vb2[p]};
        double ob[3], xk[3];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            ob[i] = 0.0;
            xk[i] = 0.0;
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                ob[i] += R[3 * j + i] * (vb[j] + a.dt_r * xb[j]);
                xk[i] += R[3 * j + i] * xb[j];
            }
        }
        // Boris vjp: out = vm + vr x sig + h E, vr = vm + vm x tau, sig = 2 tau / (1 + |tau|^2)
        const double sig[3] = {sg * tau[0], sg * tau[1], sg * tau[2]};
        double Eb[3], Bb[3], vmb[3], vrb[3], sigb[3], taub[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            vmb[d] = ob[d];
            Eb[d] = h * ob[d];
        }
        vrb[0] = sig[1] * ob[2] - sig[2] * ob[1];
        vrb[1] = sig[2] * ob[0] - sig[0] * ob[2];
        vrb[2] = sig[0] * ob[1] - sig[1] * ob[0];
        sigb[0] = ob[1] * vr[2] - ob[2] * vr[1];
        sigb[1] = ob[2] * vr[0] - ob[0] * vr[2];
        sigb[2] = ob[0] * vr[1] - ob[1] * vr[0];
        vmb[0] += vrb[0] + (tau[1] * vrb[2] - tau[2] * vrb[1]);
        vmb[1] += vrb[1] + (tau[2] * vrb[0] - tau[0] * vrb[2]);
        vmb[2] += vrb[2] + (tau[0] * vrb[1] - tau[1] * vrb[0]);
        taub[0] = vrb[1] * vm[2] - vrb[2] * vm[1];
        taub[1] = vrb[2] * vm[0] - vrb[0] * vm[2];
        taub[2] = vrb[0] * vm[1] - vrb[1] * vm[0];
        const double st = sigb[0] * tau[0] + sigb[1] * tau[1] + sigb[2] * tau[2];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            taub[d] += 2.0 * sigb[d] / den - 4.0 * st * tau[d] / (den * den);
            Bb[d] = h * taub[d];
            Eb[d] += h * vmb[d];
        }
        // gather vjp: position and edge DoFs
        double Eg[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const double ae = cf[3 * k] * Eb[0] + cf[3 * k + 1] * Eb[1] + cf[3 * k + 2] * Eb[2];
            const double cb = cf[12 + 3 * k] * Bb[0] + cf[12 + 3 * k + 1] * Bb[1] + cf[12 + 3 * k + 2] * Bb[2];
#pragma unroll
            for (int d = 0; d < 3; ++d) xk[d] += g[k][d] * (ae + cb);
            Eg[k] = Eb[0] * g[k][0] + Eb[1] * g[k][1] + Eb[2] * g[k][2];
        }
        constexpr int le[6][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            const double we = l[le[e][0]] * Eg[le[e][1]] - l[le[e][1]] * Eg[le[e][0]];
            ge[2 * e] = we * b.c;
            ge[2 * e + 1] = -we * b.s;
        }
        b.vb0[p] = vmb[0];
        b.vb1[p] = vmb[1];
        b.vb2[p] = vmb[2];
        b.xb0[p] = xk[0];
        b.xb1[p] = xk[1];
        b.xb2[p] = xk[2];
    }
    const WaveRuns runs = wave_runs(T);
#pragma unroll
    for (int k = 0; k < 12; ++k) ge[k] = run_total(ge[k], runs);
    if (T >= 0 && runs.lane == runs.run_end) {
        const TetTopo *tp = a.topo + T;
#pragma unroll
        for (int e = 0; e < 6; ++e) {
            unsafeAtomicAdd(&b.grad_e[2 * (int64_t)tp->e[e]], ge[2 * e]);
            unsafeAtomicAdd(&b.grad_e[2 * (int64_t)tp->e[e] + 1], ge[2 * e + 1]);
        }
    }
}

// ------------------------------------------------------------------ point location
// Particles enter as Cartesian points; the step works on (tet, barycentrics).
// A point is located by a straight walk from the centroid of a start tet (the
// caller's hint, else the tet of the point's start-grid cell) to the point:
// each hop leaves the current tet through the face whose barycentric reaches
// zero first and enters the neighbour.  The final barycentrics are recomputed
// from the point itself, lam_k = grad l_k . (x - r_0) (k = 1..3).  A walk that
// reaches a boundary face or the hop cap marks the point as not located; a
// point within kLocateTol (in barycentric terms) outside a boundary face counts
// as on it, so points on the domain boundary are located.
constexpr int kLocateHopCap = 4096;
constexpr double kLocateTol = 1e-10;

struct GridArgs {
    const int32_t *cell;
    double lo[3], inv[3];
    int dims[3];
};

__global__ void __launch_bounds__(kBlock) k_locate(int64_t n, const double *__restrict__ x0,
                                                   const double *__restrict__ x1, const double *__restrict__ x2,
                                                   const int32_t *__restrict__ hint, int64_t nt,
                                                   const TetTopo *__restrict__ topo, const double *__restrict__ grad,
                                                   const double *__restrict__ xyz, GridArgs G,
                                                   double *__restrict__ lam1, double *__restrict__ lam2,
                                                   double *__restrict__ lam3, int32_t *__restrict__ tet,
                                                   unsigned *__restrict__ fails, int fixed) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const double x[3] = {x0[p], x1[p], x2[p]};
    bool ok = isfinite(x[0]) && isfinite(x[1]) && isfinite(x[2]);
    int T = hint ? hint[p] : -1;
    if (ok && (unsigned)T >= (unsigned)nt) {
        int64_t c[3];
#pragma unroll
        for (int d = 0; d < 3; ++d) {
            const double f = floor((x[d] - G.lo[d]) * G.inv[d]);
            c[d] = (int64_t)fmin(fmax(f, 0.0), (double)(G.dims[d] - 1));
        }
        T = G.cell[c[0] + (int64_t)G.dims[0] * (c[1] + (int64_t)G.dims[1] * c[2])];
    }
    if (ok) {
        // start at the centroid of T (barycentrics 1/4) with displacement x - centroid
        double l[4] = {0.25, 0.25, 0.25, 0.25}, d[3] = {x[0], x[1], x[2]};
        {
            const TetTopo tp = topo[T];
#pragma unroll
            for (int k = 0; k < 4; ++k)
#pragma unroll
                for (int c = 0; c < 3; ++c) d[c] -= 0.25 * xyz[3 * (int64_t)tp.v[k] + c];
        }
        int hops = 0;
        for (;;) {
            const double *gp = grad + (int64_t)T * 12;
            const TetTopo tp = topo[T];
            double dl[4];
#pragma unroll
            for (int k = 1; k < 4; ++k) dl[k] = gp[3 * k] * d[0] + gp[3 * k + 1] * d[1] + gp[3 * k + 2] * d[2];
            dl[0] = -(dl[1] + dl[2] + dl[3]);
            double smin = 1.0;
            int kmin = -1;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (dl[k] < 0.0 && l[k] + dl[k] < 0.0 && !(tp.n[k] < 0 && l[k] + dl[k] >= -kLocateTol)) {
                    const double sk = l[k] > 0.0 ? l[k] / (-dl[k]) : 0.0;
                    if (kmin < 0 || sk < smin) {
                        smin = sk;
                        kmin = k;
                    }
                }
            if (kmin < 0) break;
            int nb = -1;
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (k == kmin) nb = tp.n[k];
            if (nb < 0 || ++hops > kLocateHopCap) {
                ok = false;
                break;
            }
            double lc[4], sum = 0.0;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                lc[k] = (k == kmin) ? 0.0 : fmax(l[k] + smin * dl[k], 0.0);
                sum += lc[k];
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) d[c] -= smin * d[c];
            const TetTopo tn = topo[nb];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                double v = 0.0;
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (tp.v[i] == tn.v[j]) v = lc[i] / sum;
                l[j] = v;
            }
            T = nb;
        }
    }
    if (!ok) {
        tet[p] = -1;
        atomicAdd(fails, 1u);
        return;
    }
    const TetTopo tp = topo[T];
    const double *r0 = xyz + 3 * (int64_t)tp.v[0];
    const double dx[3] = {x[0] - r0[0], x[1] - r0[1], x[2] - r0[2]};
    const double *gp = grad + (int64_t)T * 12;
    const double l1 = gp[3] * dx[0] + gp[4] * dx[1] + gp[5] * dx[2];
    const double l2 = gp[6] * dx[0] + gp[7] * dx[1] + gp[8] * dx[2];
    const double l3 = gp[9] * dx[0] + gp[10] * dx[1] + gp[11] * dx[2];
    if (fixed) {
        uint32_t u[3];
        fix_round3(l1, l2, l3, u);
        reinterpret_cast<uint32_t *>(lam1)[p] = u[0];
        reinterpret_cast<uint32_t *>(lam2)[p] = u[1];
        reinterpret_cast<uint32_t *>(lam3)[p] = u[2];
    } else {
        lam1[p] = l1;
        lam2[p] = l2;
        lam3[p] = l3;
    }
    tet[p] = T;
}

// x = sum_k lam_k r_k of every particle (lam_0 = 1 - lam_1 - lam_2 - lam_3).
__global__ void __launch_bounds__(kBlock) k_positions(int64_t n, int64_t nt, const double *__restrict__ lam1,
                                                      const double *__restrict__ lam2, const double *__restrict__ lam3,
                                                      const int32_t *__restrict__ tet, const TetTopo *__restrict__ topo,
                                                      const double *__restrict__ xyz, double *__restrict__ x0,
                                                      double *__restrict__ x1, double *__restrict__ x2,
                                                      unsigned *__restrict__ status, int fixed) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const int T = tet[p];
    if ((unsigned)T >= (unsigned)nt) {
        atomicOr(status, (unsigned)ETPIC_DEV_BADTET);
        x0[p] = x1[p] = x2[p] = NAN;
        return;
    }
    const double a1 = lam_at(lam1, p, fixed), a2 = lam_at(lam2, p, fixed), a3 = lam_at(lam3, p, fixed);
    const double l[4] = {1.0 - a1 - a2 - a3, a1, a2, a3};
    const TetTopo tp = topo[T];
    double x[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 4; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) x[c] += l[k] * xyz[3 * (int64_t)tp.v[k] + c];
    x0[p] = x[0];
    x1[p] = x[1];
    x2[p] = x[2];
}

// ------------------------------------------------------------------ vertex charge
__global__ void __launch_bounds__(kBlock) k_charge(int64_t n, int64_t nt, const double *__restrict__ lam1,
                                                   const double *__restrict__ lam2, const double *__restrict__ lam3,
                                                   const int32_t *__restrict__ tet, const TetTopo *__restrict__ topo,
                                                   double qw, double *__restrict__ rho, unsigned *status, int fixed) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int T = -1;
    double l[4] = {0.0, 0.0, 0.0, 0.0};
    if (p < n) {
        T = tet[p];
        if ((unsigned)T >= (unsigned)nt) {
            atomicOr(status, (unsigned)ETPIC_DEV_BADTET);
            T = -1;
        } else {
            l[1] = lam_at(lam1, p, fixed);
            l[2] = lam_at(lam2, p, fixed);
            l[3] = lam_at(lam3, p, fixed);
            l[0] = 1.0 - l[1] - l[2] - l[3];
        }
    }
    const WaveRuns r = wave_runs(T);
#pragma unroll
    for (int k = 0; k < 4; ++k) l[k] = run_total(l[k], r);
    if (r.lane == r.run_end && T >= 0) {
        const TetTopo tp = topo[T];
#pragma unroll
        for (int k = 0; k < 4; ++k) unsafeAtomicAdd(&rho[tp.v[k]], qw * l[k]);
    }
}

// The same over kSlices consecutive slices of 64 particles per wavefront: the
// run of one tet that reaches lane 63 of a slice is carried (as a
// wavefront-uniform partial sum) into the next slice instead of being flushed,
// so a tet holding thousands of sorted particles costs kSlices times fewer
// same-address atomics.
template <int kSlices>
__global__ void __launch_bounds__(kBlock) k_charge_slices(int64_t n, int64_t nt, const double *__restrict__ lam1,
                                                          const double *__restrict__ lam2,
                                                          const double *__restrict__ lam3,
                                                          const int32_t *__restrict__ tet,
                                                          const TetTopo *__restrict__ topo, double qw,
                                                          double *__restrict__ rho, unsigned *status, int fixed) {
    const int lane = threadIdx.x & 63;
    const int64_t base = (((int64_t)blockIdx.x * kBlock + threadIdx.x) >> 6) * 64 * kSlices;
    auto flush = [&](int T, const double v[4]) {
        const TetTopo tp = topo[T];
#pragma unroll
        for (int k = 0; k < 4; ++k) unsafeAtomicAdd(&rho[tp.v[k]], qw * v[k]);
    };
    int carry_t = -1;   // tet of the carried run (uniform over the wavefront), -1: none
    double carry[4] = {0.0, 0.0, 0.0, 0.0};
    for (int s = 0; s < kSlices; ++s) {
        const int64_t p = base + (int64_t)s * 64 + lane;
        int T = -1;
        double l[4] = {0.0, 0.0, 0.0, 0.0};
        if (p < n) {
            T = tet[p];
            if ((unsigned)T >= (unsigned)nt) {
                atomicOr(status, (unsigned)ETPIC_DEV_BADTET);
                T = -1;
            } else {
                l[1] = lam_at(lam1, p, fixed);
                l[2] = lam_at(lam2, p, fixed);
                l[3] = lam_at(lam3, p, fixed);
                l[0] = 1.0 - l[1] - l[2] - l[3];
            }
        }
        const int t0 = __shfl(T, 0);
        if (carry_t >= 0 && carry_t != t0) {   // the carried run ended with the previous slice
            if (lane == 0) flush(carry_t, carry);
            carry_t = -1;
        }
        const WaveRuns r = wave_runs(T);
#pragma unroll
        for (int k = 0; k < 4; ++k) l[k] = run_total(l[k], r);
        const int first_end = __shfl(r.run_end, 0);
        if (carry_t >= 0 && lane == first_end)   // the slice's first run continues the carried one
#pragma unroll
            for (int k = 0; k < 4; ++k) l[k] += carry[k];
        const int t63 = __shfl(T, 63);
        double last[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) last[k] = __shfl(l[k], 63);
        const bool keep = s + 1 < kSlices && t63 >= 0;   // the run through lane 63 may go on
        if (lane == r.run_end && T >= 0 && !(keep && r.run_end == 63)) flush(T, l);
        carry_t = keep ? t63 : -1;
#pragma unroll
        for (int k = 0; k < 4; ++k) carry[k] = keep ? last[k] : 0.0;
    }
    if (carry_t >= 0 && lane == 0) flush(carry_t, carry);
}

// ------------------------------------------------------------------ continuity residual
// r_k = sum_{e incident} (+dG_e if k is the head, -dG_e if the tail) - (rho_new_k - rho_old_k).
// out[0] = max |r|, out[1] = max |rho_old| as the bit patterns of non-negative doubles
// (which order like unsigned integers).  The maxima propagate NaN: a non-finite
// dG or rho makes the residual NaN (whose bit pattern orders above +inf), never
// a passing number.
__device__ __forceinline__ double max_keep_nan(double a, double b) { return (a != a || a > b) ? a : b; }

// |r_k| of vertex k: the signed sum of its incident edge currents (CSR of
// (edge << 1 | head) codes) minus its change of charge.
__device__ __forceinline__ double gauss_r(int64_t k, const int32_t *__restrict__ ptr,
                                          const int32_t *__restrict__ code, const double *__restrict__ dG,
                                          const double *__restrict__ rho_new, const double *__restrict__ rho_old) {
    double div = 0.0;
    for (int32_t i = ptr[k]; i < ptr[k + 1]; ++i) {
        const int32_t c = code[i];
        const double g = dG[c >> 1];
        div += (c & 1) ? g : -g;
    }
    return fabs(div - (rho_new[k] - rho_old[k]));
}

__global__ void __launch_bounds__(kBlock) k_gauss(int64_t nv, const int32_t *__restrict__ ptr,
                                                  const int32_t *__restrict__ code, const double *__restrict__ dG,
                                                  const double *__restrict__ rho_new,
                                                  const double *__restrict__ rho_old,
                                                  unsigned long long *__restrict__ out) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double r = 0.0, p = 0.0;
    if (k < nv) {
        r = gauss_r(k, ptr, code, dG, rho_new, rho_old);
        p = fabs(rho_old[k]);
    }
    // wave-level max then one atomic per wave; a NaN operand wins
    for (int off = 32; off > 0; off >>= 1) {
        r = max_keep_nan(r, __shfl_xor(r, off));
        p = max_keep_nan(p, __shfl_xor(p, off));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&out[0], (unsigned long long)__double_as_longlong(r));
        atomicMax(&out[1], (unsigned long long)__double_as_longlong(p));
    }
}

// The same maxima in two passes without atomics, for the allocation-free
// entry point: k_gauss_part leaves one (max|r|, max|rho_old|) pair per block
// (grid-stride over the vertices, kResBlocks blocks at most) in part[2 * block],
// k_gauss_final reduces the pairs into out[0..1].  Every partial is written
// before it is read, so nothing needs clearing between calls.
constexpr int kResBlocks = 1024;

__global__ void __launch_bounds__(kBlock) k_gauss_part(int64_t nv, const int32_t *__restrict__ ptr,
                                                       const int32_t *__restrict__ code,
                                                       const double *__restrict__ dG,
                                                       const double *__restrict__ rho_new,
                                                       const double *__restrict__ rho_old, double *__restrict__ part) {
    double r = 0.0, p = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; k < nv; k += (int64_t)gridDim.x * blockDim.x) {
        r = max_keep_nan(gauss_r(k, ptr, code, dG, rho_new, rho_old), r);
        p = max_keep_nan(fabs(rho_old[k]), p);
    }
    for (int off = 32; off > 0; off >>= 1) {
        r = max_keep_nan(r, __shfl_xor(r, off));
        p = max_keep_nan(p, __shfl_xor(p, off));
    }
    __shared__ double wr[kBlock / 64], wp[kBlock / 64];
    if ((threadIdx.x & 63) == 0) {
        wr[threadIdx.x >> 6] = r;
        wp[threadIdx.x >> 6] = p;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) {
            r = max_keep_nan(r, wr[w]);
            p = max_keep_nan(p, wp[w]);
        }
        part[2 * blockIdx.x] = r;
        part[2 * blockIdx.x + 1] = p;
    }
}

__global__ void __launch_bounds__(kBlock) k_gauss_final(const double *__restrict__ part, int nblk,
                                                        double *__restrict__ out) {
    double r = 0.0, p = 0.0;
    for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
        r = max_keep_nan(r, part[2 * b]);
        p = max_keep_nan(p, part[2 * b + 1]);
    }
    for (int off = 32; off > 0; off >>= 1) {
        r = max_keep_nan(r, __shfl_xor(r, off));
        p = max_keep_nan(p, __shfl_xor(p, off));
    }
    __shared__ double wr[kBlock / 64], wp[kBlock / 64];
    if ((threadIdx.x & 63) == 0) {
        wr[threadIdx.x >> 6] = r;
        wp[threadIdx.x >> 6] = p;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kBlock / 64; ++w) {
            r = max_keep_nan(r, wr[w]);
            p = max_keep_nan(p, wp[w]);
        }
        out[0] = r;
        out[1] = p;
    }
}

constexpr size_t kScratchDoubles = 2 * (size_t)kResBlocks + 2;

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

// sum over tets of count^2 (count = particles in the tet), accumulated into
// *out: sum(count^2) / N_p is the mean length of the same-tet run a particle
// belongs to, which picks the slices per wavefront of the particle kernel.
__global__ void __launch_bounds__(kBlock) k_run_stat(int64_t nt, const unsigned *__restrict__ count,
                                                     unsigned long long *__restrict__ out) {
    unsigned long long c2 = 0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < nt; t += (int64_t)gridDim.x * blockDim.x) {
        const unsigned long long c = count[t];
        c2 += c * c;
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) c2 += __shfl_xor(c2, off);
    __shared__ unsigned long long s_part[kBlock / 64];
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = c2;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long sum = 0;
#pragma unroll
        for (int w = 0; w < kBlock / 64; ++w) sum += s_part[w];
        if (sum) atomicAdd(out, sum);
    }
}

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

// hsrc / hdst (optional): nh further arrays of length n at stride n, of the
// velocity type, moved with the particles (the downshifted history).
template <typename Real>
__global__ void __launch_bounds__(kBlock) k_scatter(int64_t n, int64_t nt, const int32_t *__restrict__ tet,
                                                    unsigned *__restrict__ cursor, etpic_particles src,
                                                    etpic_particles dst, const Real *__restrict__ hsrc = nullptr,
                                                    Real *__restrict__ hdst = nullptr, int nh = 0, int fixed = 0) {
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
        if (fixed)
            reinterpret_cast<uint32_t *>(dst.lam[k])[q] = reinterpret_cast<const uint32_t *>(src.lam[k])[p];
        else
            dst.lam[k][q] = src.lam[k][p];
        static_cast<Real *>(dst.vel[k])[q] = static_cast<const Real *>(src.vel[k])[p];
    }
    if (src.id && dst.id) dst.id[q] = src.id[p];
    for (int i = 0; i < nh; ++i) hdst[(int64_t)i * n + q] = hsrc[(int64_t)i * n + p];
}

// ------------------------------------------------------------------ field update
// Implicit envelope field step on the Whitney edge space (a side path of the
// particle step, timed separately).  Eliminating B~ from the envelope Maxwell
// equations (Formulation: the curl equations with the carrier) and testing
// with W1 gives
//   M e'' + 2 j w M e' + (K - w^2 M) e = f,   f = -e^{-j w t} g''
// (M = eps-mass, K = curl-curl, g the deposited edge DoFs of G), stepped with
// Newmark-beta (gamma = 1/2, beta = 1/4, Formulation) in acceleration form:
//   A a_{n+1} = f_{n+1} - M (2 j w v* - w^2 u*) - K u*,   A = (1 + j w dt - w^2 dt^2/4) M + (dt^2/4) K,
//   u* = u + dt v + dt^2/4 a,  v* = v + dt/2 a,  u_{n+1} = u* + dt^2/4 a_{n+1},  v_{n+1} = v* + dt/2 a_{n+1}.
// A is complex symmetric: Jacobi-preconditioned COCG.  The face envelope
// follows the discrete envelope Faraday law (j w + d/dt) b = -C e with the
// trapezoidal rule.
__device__ __forceinline__ double2 cmul(double2 a, double2 b) { return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x); }
__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
    const double d = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / d, (a.y * b.x - a.x * b.y) / d);
}

constexpr int kRowLanes = 8;   // lanes per CSR row

struct FieldCsr {
    int64_t ne;
    const int32_t *rowptr, *col;
    const double *M, *K;
    const uint8_t *dir;
};

// Row-wise (M x1)_i and (K x2)_i with kRowLanes lanes per row, summed across
// those lanes; every lane of the group returns the totals.
__device__ __forceinline__ void csr_row2(const FieldCsr &S, int64_t row, int sub, const double2 *__restrict__ x1,
                                         const double2 *__restrict__ x2, double2 &m1, double2 &k2) {
    m1 = make_double2(0.0, 0.0);
    k2 = make_double2(0.0, 0.0);
    if (row < S.ne) {
        for (int32_t j = S.rowptr[row] + sub; j < S.rowptr[row + 1]; j += kRowLanes) {
            const int32_t c = S.col[j];
            const double mv = S.M[j], kv = S.K[j];
            const double2 a = x1[c], b = x2[c];
            m1.x += mv * a.x;
            m1.y += mv * a.y;
            k2.x += kv * b.x;
            k2.y += kv * b.y;
        }
    }
#pragma unroll
    for (int off = kRowLanes / 2; off > 0; off >>= 1) {
        m1.x += __shfl_xor(m1.x, off);
        m1.y += __shfl_xor(m1.y, off);
        k2.x += __shfl_xor(k2.x, off);
        k2.y += __shfl_xor(k2.y, off);
    }
}

// block-level sum of up to 4 doubles into partial[blockIdx.x * 4 + k]
__device__ __forceinline__ void block_sum4(double v[4], double *partial) {
    __shared__ double sh[kBlock / 64][4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0)
#pragma unroll
        for (int k = 0; k < 4; ++k) sh[wid][k] = v[k];
    __syncthreads();
    if (threadIdx.x < 4) {
        double s = 0.0;
        for (int w = 0; w < kBlock / 64; ++w) s += sh[w][threadIdx.x];
        partial[blockIdx.x * 4 + threadIdx.x] = s;
    }
}

// y = alpha M x + beta K x (complex alpha, real beta)
__global__ void __launch_bounds__(kBlock) k_field_spmv(FieldCsr S, double2 alpha, double beta,
                                                       const double2 *__restrict__ x, double2 *__restrict__ y) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t row = t / kRowLanes;
    const int sub = (int)(t % kRowLanes);
    double2 m, k;
    csr_row2(S, row, sub, x, x, m, k);
    if (row < S.ne && sub == 0) y[row] = cadd(cmul(alpha, m), cscale(k, beta));
}

// Newmark predictor: us = u + dt v + dt^2/4 a, vs = v + dt/2 a, w = 2 j w vs - w^2 us
__global__ void __launch_bounds__(kBlock) k_nm_predict(int64_t ne, const double2 *__restrict__ u,
                                                       const double2 *__restrict__ v, const double2 *__restrict__ a,
                                                       double2 *__restrict__ us, double2 *__restrict__ vs,
                                                       double2 *__restrict__ w, double dt, double omega) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ne) return;
    const double2 ui = u[i], vi = v[i], ai = a[i];
    const double2 usi = cadd(cadd(ui, cscale(vi, dt)), cscale(ai, 0.25 * dt * dt));
    const double2 vsi = cadd(vi, cscale(ai, 0.5 * dt));
    us[i] = usi;
    vs[i] = vsi;
    w[i] = csub(cmul(make_double2(0.0, 2.0 * omega), vsi), cscale(usi, omega * omega));
}

// rhs = f - M w - K us with f = -e^{-j w t} g'';  boundary rows 0
__global__ void __launch_bounds__(kBlock) k_nm_rhs(FieldCsr S, const double2 *__restrict__ w,
                                                   const double2 *__restrict__ us, const double *__restrict__ gdd,
                                                   double c, double s, double2 *__restrict__ rhs) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t row = t / kRowLanes;
    const int sub = (int)(t % kRowLanes);
    double2 m, k;
    csr_row2(S, row, sub, w, us, m, k);
    if (row < S.ne && sub == 0) {
        double2 r = make_double2(0.0, 0.0);
        if (!S.dir[row]) {
            const double g = gdd ? gdd[row] : 0.0;
            // -e^{-j w t} g = -(c - j s) g
            r = make_double2(-c * g - m.x - k.x, s * g - m.y - k.y);
        }
        rhs[row] = r;
    }
}

// COCG start: x = 0, r = rhs, z = Dinv r, p = q = 0; partials r.z (re, im),
// |r|^2, |b|^2 (= |r|^2); clears the done flag and the iteration count.
__global__ void __launch_bounds__(kBlock) k_cocg_init(int64_t ne, const double2 *__restrict__ rhs,
                                                      const double2 *__restrict__ dinv, double2 *__restrict__ x,
                                                      double2 *__restrict__ r, double2 *__restrict__ z,
                                                      double2 *__restrict__ p, double2 *__restrict__ q,
                                                      double *__restrict__ partial, double *__restrict__ sc) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    if (i < ne) {
        const double2 ri = rhs[i];
        const double2 zi = cmul(dinv[i], ri);
        x[i] = make_double2(0.0, 0.0);
        r[i] = ri;
        z[i] = zi;
        p[i] = make_double2(0.0, 0.0);
        q[i] = make_double2(0.0, 0.0);
        const double2 rz = cmul(ri, zi);
        v[0] = rz.x;
        v[1] = rz.y;
        v[2] = ri.x * ri.x + ri.y * ri.y;
        v[3] = v[2];
    }
    if (i == 0) {
        sc[10] = 0.0;
        sc[11] = 0.0;
    }
    block_sum4(v, partial);
}

// faces: (1 + j w dt/2) b_new = (1 - j w dt/2) b - dt/2 C (u + u_new), u_new = us + dt^2/4 x,
// (C e)_f = e_ab + e_bc - e_ac
__global__ void __launch_bounds__(kBlock) k_nm_faraday(int64_t nf, const int32_t *__restrict__ fe,
                                                       const double2 *__restrict__ u, const double2 *__restrict__ us,
                                                       const double2 *__restrict__ x, double2 *__restrict__ b,
                                                       double dt, double omega) {
    const int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    const double q = 0.25 * dt * dt;
    double2 cs = make_double2(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const int32_t e = fe[3 * f + k];
        const double2 sum = cadd(u[e], cadd(us[e], cscale(x[e], q)));
        cs = (k == 2) ? csub(cs, sum) : cadd(cs, sum);
    }
    const double2 num = csub(cmul(make_double2(1.0, -0.5 * omega * dt), b[f]), cscale(cs, 0.5 * dt));
    b[f] = cdiv(num, make_double2(1.0, 0.5 * omega * dt));
}

// u = us + dt^2/4 x, v = vs + dt/2 x, a = x
__global__ void __launch_bounds__(kBlock) k_nm_correct(int64_t ne, const double2 *__restrict__ us,
                                                       const double2 *__restrict__ vs, const double2 *__restrict__ x,
                                                       double2 *__restrict__ u, double2 *__restrict__ v,
                                                       double2 *__restrict__ a, double dt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ne) return;
    const double2 xi = x[i];
    u[i] = cadd(us[i], cscale(xi, 0.25 * dt * dt));
    v[i] = cadd(vs[i], cscale(xi, 0.5 * dt));
    a[i] = xi;
}

// ---- non-solenoidal field of the quasi-Helmholtz split (eq. ns_equation):
// Jacobi-preconditioned CG on the nodal operator D^T [*eps] D, real because
// the operator is real (the carrier phase multiplies the solution).
struct NsCsr {
    int64_t nv;
    const int32_t *rowptr, *col;
    const double *S;
};

// The CG kernels run on at most kNsBlocks blocks (grid-stride loops), so that
// every block can sum all block partials of the previous kernel itself, in
// the same fixed order: the scalars of the iteration need no kernel of their
// own and no cross-block synchronisation.  Partials: 4 doubles per block.
// Scalars sc (written by thread 0 of block 0 only, read by the next kernel):
// sc[0], sc[1] rho = r.z of even / odd iterations, sc[8] |r|^2, sc[9] |b|^2,
// sc[10] done flag, sc[11] iterations taken.
constexpr int kNsBlocks = 512;
constexpr int kNsThreads = 1024;   // product kernels: 16 wavefronts per block, enough rows in flight for one pass
constexpr int kNsVecThreads = 256; // vector kernels (one node per lane): more, smaller blocks

// Block-level sum of 4 doubles into partial[blockIdx.x * 4 + k].
__device__ __forceinline__ void ns_block_sum4(double v[4], double *partial) {
    __shared__ double sh[kNsThreads / 64][4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
        for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off);
    if ((threadIdx.x & 63) == 0)
#pragma unroll
        for (int k = 0; k < 4; ++k) sh[threadIdx.x >> 6][k] = v[k];
    __syncthreads();
    if (threadIdx.x < 4) {
        double t = 0.0;
        for (int w = 0; w < (int)(blockDim.x / 64); ++w) t += sh[w][threadIdx.x];
        partial[blockIdx.x * 4 + threadIdx.x] = t;
    }
}

// Every thread gets the sums of the nb partials (fixed order).
__device__ __forceinline__ void all_sum4(int64_t nb, const double *__restrict__ partial, double tot[4]) {
    __shared__ double sh[kNsThreads / 64][4];
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
        for (int w = 0; w < (int)(blockDim.x / 64); ++w) t += sh[w][threadIdx.x];
        res[threadIdx.x] = t;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k) tot[k] = res[k];
}

// Right-hand side of a nodal solve: b = -(gs (D^T G + rho0) + D^T w_comp)
// at the nodes off the wall, 0 on it; every pointer may be NULL.  w is a
// complex edge vector of which component comp (0 re, 1 im) is taken.
struct NsRhs {
    const double *G, *rho0;
    double gs;
    const double2 *w;
    int comp;
};

// (D^T G)_i sums +-G over the edges at node i (+ where i is the head).
__device__ __forceinline__ double ns_rhs(int64_t i, const int32_t *__restrict__ ptr, const int32_t *__restrict__ code,
                                         const NsRhs &R, const uint8_t *__restrict__ wall) {
    if (wall[i]) return 0.0;
    double div = R.rho0 ? R.rho0[i] : 0.0;
    double dw = 0.0;
    for (int32_t k = ptr[i]; k < ptr[i + 1]; ++k) {
        const int32_t c = code[k];
        if (R.G) {
            const double g = R.G[c >> 1];
            div += (c & 1) ? g : -g;
        }
        if (R.w) {
            const double2 wv = R.w[c >> 1];
            const double g = R.comp ? wv.y : wv.x;
            dw += (c & 1) ? g : -g;
        }
    }
    return -(R.gs * div + dw);
}

// Cold start: x = 0, r = b, z = Dinv b, p = q = 0; partials r.z, 0, |r|^2, |b|^2.
__global__ void __launch_bounds__(kNsVecThreads) k_ns_start(int64_t nv, const int32_t *__restrict__ ptr,
                                                     const int32_t *__restrict__ code, NsRhs R,
                                                     const uint8_t *__restrict__ wall,
                                                     const double *__restrict__ dinv, double *__restrict__ x,
                                                     double *__restrict__ r, double *__restrict__ z,
                                                     double *__restrict__ p, double *__restrict__ q,
                                                     double *__restrict__ partial, double *__restrict__ sc) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x) {
        const double b = ns_rhs(i, ptr, code, R, wall);
        const double zi = dinv[i] * b;
        x[i] = 0.0;
        r[i] = b;
        z[i] = zi;
        p[i] = 0.0;
        q[i] = 0.0;
        v[0] += b * zi;
        v[2] += b * b;
        v[3] += b * b;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc[10] = 0.0;
        sc[11] = 0.0;
    }
    ns_block_sum4(v, partial);
}

// Warm start from the x left by the previous solve: r = b - S x, z = Dinv r,
// p = q = 0; partials r.z, 0, |r|^2, |b|^2.  kRowLanes lanes per row.
__global__ void __launch_bounds__(kNsThreads) k_ns_start_warm(NsCsr S, const int32_t *__restrict__ ptr,
                                                          const int32_t *__restrict__ code, NsRhs R,
                                                          const uint8_t *__restrict__ wall,
                                                          const double *__restrict__ dinv,
                                                          const double *__restrict__ x, double *__restrict__ r,
                                                          double *__restrict__ z, double *__restrict__ p,
                                                          double *__restrict__ q, double *__restrict__ partial,
                                                          double *__restrict__ sc) {
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t / kRowLanes < S.nv; t += stride) {
        const int64_t row = t / kRowLanes;
        const int sub = (int)(t % kRowLanes);
        double sx = 0.0;
        for (int32_t j = S.rowptr[row] + sub; j < S.rowptr[row + 1]; j += kRowLanes) sx += S.S[j] * x[S.col[j]];
#pragma unroll
        for (int off = kRowLanes / 2; off > 0; off >>= 1) sx += __shfl_xor(sx, off);
        if (sub == 0) {
            const double b = ns_rhs(row, ptr, code, R, wall);
            const double ri = b - sx;
            const double zi = dinv[row] * ri;
            r[row] = ri;
            z[row] = zi;
            p[row] = 0.0;
            q[row] = 0.0;
            v[0] += ri * zi;
            v[2] += ri * ri;
            v[3] += b * b;
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc[10] = 0.0;
        sc[11] = 0.0;
    }
    ns_block_sum4(v, partial);
}

// Iteration k, first half.  From the partials of the previous update (or of
// the start, k = 0): |r|^2 and rho_new = r.z; done once |r|^2 <= tol^2 |b|^2
// (or not finite, or b = 0), then every block returns.  Otherwise beta = rho_new /
// rho_old, p = z + beta p and q = A p = A z + beta q (the direction update
// folded into the product, so no separate pass over p is needed), with the
// partials of p . q.  check_only: the convergence test alone (after the last
// allowed iteration).  Returns at once if an earlier launch found convergence.
__global__ void __launch_bounds__(kNsThreads) k_ns_apply(NsCsr S, double *__restrict__ sc,
                                                     const double *__restrict__ z, double *__restrict__ p,
                                                     double *__restrict__ q, const double *__restrict__ pin,
                                                     int64_t nb_in, double *__restrict__ pout, int k, double tol2,
                                                     int check_only) {
    if (sc[10] != 0.0) return;
    double tot[4];
    all_sum4(nb_in, pin, tot);
    const double b2 = k == 0 ? tot[3] : sc[9];
    const double r2 = tot[2], rn = tot[0];
    const bool done = b2 == 0.0 || !(r2 > tol2 * b2);   // no source: x = 0, done
    const double ro = sc[(k + 1) & 1];
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc[8] = r2;
        if (k == 0) sc[9] = b2;
        sc[k & 1] = rn;
        sc[10] = done ? 1.0 : 0.0;
        sc[11] = (double)k;
    }
    if (done || check_only) return;
    const double be = (k == 0 || ro == 0.0) ? 0.0 : rn / ro;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t / kRowLanes < S.nv; t += stride) {
        const int64_t row = t / kRowLanes;
        const int sub = (int)(t % kRowLanes);
        double az = 0.0;
        for (int32_t j = S.rowptr[row] + sub; j < S.rowptr[row + 1]; j += kRowLanes) az += S.S[j] * z[S.col[j]];
#pragma unroll
        for (int off = kRowLanes / 2; off > 0; off >>= 1) az += __shfl_xor(az, off);
        if (sub == 0) {
            const double pn = z[row] + be * p[row];
            const double qn = az + be * q[row];
            p[row] = pn;
            q[row] = qn;
            v[0] += pn * qn;
        }
    }
    ns_block_sum4(v, pout);
}

// Iteration k, second half: alpha = rho_new / (p . q) from the partials of the
// product; x += alpha p, r -= alpha q, z = Dinv r, with the partials of r . z
// and |r|^2.  Returns at once if the first half found convergence.
__global__ void __launch_bounds__(kNsVecThreads) k_ns_update(int64_t nv, const double *__restrict__ sc,
                                                      const double *__restrict__ dinv, const double *__restrict__ p,
                                                      const double *__restrict__ q, double *__restrict__ x,
                                                      double *__restrict__ r, double *__restrict__ z,
                                                      const double *__restrict__ pin, int64_t nb_in,
                                                      double *__restrict__ pout, int k) {
    if (sc[10] != 0.0) return;
    double tot[4];
    all_sum4(nb_in, pin, tot);
    const double pq = tot[0];
    const double al = pq != 0.0 ? sc[k & 1] / pq : 0.0;
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nv; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] += al * p[i];
        const double ri = r[i] - al * q[i];
        r[i] = ri;
        const double zi = dinv[i] * ri;
        z[i] = zi;
        v[0] += ri * zi;
        v[2] += ri * ri;
    }
    ns_block_sum4(v, pout);
}

// ---- COCG of the field step, two launches per iteration on at most
// kNsBlocks blocks, so that every block sums the previous launch's partials
// itself (as the nodal CG): no scalar kernels, the convergence test on the
// device.  Scalars sc: [0..1], [2..3] rho = r^T z (complex, unconjugated) of
// even / odd iterations, [8] |r|^2, [9] |b|^2, [10] done, [11] iterations.
//
// Iteration k, first half: done once |r_k|^2 <= tol^2 |b|^2 (or b = 0, or not
// finite); beta = rho_k / rho_{k-1}, p = z + beta p, q = A z + beta q (= A p,
// the direction update folded into the product), partials p^T q.
// A = alpha M + beta_k K.  check_only: the test alone.
__global__ void __launch_bounds__(kNsThreads) k_cocg_apply(FieldCsr S, double2 alpha, double beta_k,
                                                       double *__restrict__ sc, const double2 *__restrict__ z,
                                                       double2 *__restrict__ p, double2 *__restrict__ q,
                                                       const double *__restrict__ pin, int64_t nb_in,
                                                       double *__restrict__ pout, int k, double tol2,
                                                       int check_only) {
    if (sc[10] != 0.0) return;
    double tot[4];
    all_sum4(nb_in, pin, tot);
    const double b2 = k == 0 ? tot[3] : sc[9];
    const double r2 = tot[2];
    const double2 rn = make_double2(tot[0], tot[1]);
    const bool done = b2 == 0.0 || !(r2 > tol2 * b2);
    const int o = 2 * ((k + 1) & 1);
    const double2 ro = make_double2(sc[o], sc[o + 1]);
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        sc[8] = r2;
        if (k == 0) sc[9] = b2;
        sc[2 * (k & 1)] = rn.x;
        sc[2 * (k & 1) + 1] = rn.y;
        sc[10] = done ? 1.0 : 0.0;
        sc[11] = (double)k;
    }
    if (done || check_only) return;
    const double2 be = (k == 0 || (ro.x == 0.0 && ro.y == 0.0)) ? make_double2(0.0, 0.0) : cdiv(rn, ro);
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t / kRowLanes < S.ne; t += stride) {
        const int64_t row = t / kRowLanes;
        const int sub = (int)(t % kRowLanes);
        double2 m, kk;
        csr_row2(S, row, sub, z, z, m, kk);
        if (sub == 0) {
            const double2 pn = cadd(z[row], cmul(be, p[row]));
            const double2 qn = cadd(cadd(cmul(alpha, m), cscale(kk, beta_k)), cmul(be, q[row]));
            p[row] = pn;
            q[row] = qn;
            const double2 pq = cmul(pn, qn);
            v[0] += pq.x;
            v[1] += pq.y;
        }
    }
    ns_block_sum4(v, pout);
}

// Iteration k, second half: alpha = rho_k / (p^T q); x += alpha p, r -= alpha q,
// z = Dinv r; partials r^T z (re, im), |r|^2.
__global__ void __launch_bounds__(kNsVecThreads) k_cocg_update(int64_t ne, const double *__restrict__ sc,
                                                        const double2 *__restrict__ dinv,
                                                        const double2 *__restrict__ p, const double2 *__restrict__ q,
                                                        double2 *__restrict__ x, double2 *__restrict__ r,
                                                        double2 *__restrict__ z, const double *__restrict__ pin,
                                                        int64_t nb_in, double *__restrict__ pout, int k) {
    if (sc[10] != 0.0) return;
    double tot[4];
    all_sum4(nb_in, pin, tot);
    const double2 pq = make_double2(tot[0], tot[1]);
    const double2 rho = make_double2(sc[2 * (k & 1)], sc[2 * (k & 1) + 1]);
    const double2 al = (pq.x == 0.0 && pq.y == 0.0) ? make_double2(0.0, 0.0) : cdiv(rho, pq);
    double v[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ne; i += (int64_t)gridDim.x * blockDim.x) {
        x[i] = cadd(x[i], cmul(al, p[i]));
        const double2 ri = csub(r[i], cmul(al, q[i]));
        r[i] = ri;
        const double2 zi = cmul(dinv[i], ri);
        z[i] = zi;
        const double2 rz = cmul(ri, zi);
        v[0] += rz.x;
        v[1] += rz.y;
        v[2] += ri.x * ri.x + ri.y * ri.y;
    }
    ns_block_sum4(v, pout);
}

// x_out = e^{-j w t} x on the nodes, e_out = e^{-j w t} D x on the edges
// (edge e from ev[2e] to ev[2e+1]), edc_out = D x (+ edc_add): the same field
// as real, unmodulated DoFs.  Every pointer may be NULL.
__global__ void __launch_bounds__(kBlock) k_ns_out(int64_t ne, int64_t nv, const int32_t *__restrict__ ev,
                                                   const double *__restrict__ x, double c, double s,
                                                   double2 *__restrict__ x_out, double2 *__restrict__ e_out,
                                                   double *__restrict__ edc_out, const double *__restrict__ edc_add) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if ((e_out || edc_out) && i < ne) {
        const double d = x[ev[2 * i + 1]] - x[ev[2 * i]];
        if (e_out) e_out[i] = make_double2(c * d, -s * d);
        if (edc_out) edc_out[i] = edc_add ? d + edc_add[i] : d;
    }
    if (x_out && i < nv) {
        const double xi = x[i];
        x_out[i] = make_double2(c * xi, -s * xi);
    }
}

// e_out = u + D (xr + j xi) on the edges (edge e from ev[2e] to ev[2e+1])
__global__ void __launch_bounds__(kBlock) k_ns_combine(int64_t ne, const int32_t *__restrict__ ev,
                                                       const double *__restrict__ xr, const double *__restrict__ xi,
                                                       const double2 *__restrict__ u, double2 *__restrict__ e_out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= ne) return;
    const int32_t a = ev[2 * i], b = ev[2 * i + 1];
    const double2 ui = u[i];
    e_out[i] = make_double2(ui.x + xr[b] - xr[a], ui.y + xi[b] - xi[a]);
}

// Source of the field step from the running path integral: with h1, h2 the
// values of G one and two steps back, gdd = (G - 2 h1 + h2) / dt^2 (written
// into gdd, which may be h2)
__global__ void __launch_bounds__(kBlock) k_em_gdd(int64_t ne, const double *__restrict__ G,
                                                   const double *__restrict__ h1, const double *h2, double *gdd,
                                                   double inv_dt2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ne) gdd[i] = ((G[i] - 2.0 * h1[i]) + h2[i]) * inv_dt2;
}

// history shift after a field step: h2 = h1, h1 = G
__global__ void __launch_bounds__(kBlock) k_em_shift(int64_t ne, const double *__restrict__ G, double *__restrict__ h1,
                                                     double *__restrict__ h2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ne) {
        h2[i] = h1[i];
        h1[i] = G[i];
    }
}

// Solenoidal source: gs = gdd + Re m, m = [*eps] D y with D^T [*eps] D y =
// -D^T gdd at the inner nodes (gs may be gdd)
__global__ void __launch_bounds__(kBlock) k_sol_add(int64_t ne, const double *gdd, const double2 *__restrict__ m,
                                                    double *gs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ne) gs[i] = gdd[i] + m[i].x;
}

// e += u: the solenoidal and non-solenoidal halves of the field summed
__global__ void __launch_bounds__(kBlock) k_em_add(int64_t ne, const double2 *__restrict__ u, double2 *__restrict__ e) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < ne) {
        const double2 a = u[i], b = e[i];
        e[i] = make_double2(a.x + b.x, a.y + b.y);
    }
}

inline unsigned grid_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

// =============================================================================== context

// Device memory carved from one caller-owned buffer.  Every table and scratch
// array the library keeps on the device lives in such a buffer (context
// workspace, mesh tables, field solver, Gauss-law solver, downshifted rows); the
// library itself allocates no device memory.  A layout takes its arrays in a
// fixed order, each on a 256-byte boundary; with a null base it only counts
// the bytes, which is how the size queries are answered.
struct Carve {
    char *base = nullptr;
    size_t cap = 0, used = 0;
    template <typename T>
    T *take(size_t count) {
        const size_t off = (used + 255) & ~(size_t)255;
        used = off + sizeof(T) * std::max<size_t>(count, 1);
        return base ? reinterpret_cast<T *>(base + off) : nullptr;
    }
};

// Device state of the field update (allocated by etpic_field_setup).
struct FieldState {
    bool ready = false;
    double dt = 0, omega = 0, eps = 0, mu = 0;
    int64_t ne = 0, nf = 0, nnz = 0;
    int32_t *rowptr = nullptr, *col = nullptr, *face_edge = nullptr;
    double *M = nullptr, *K = nullptr;
    uint8_t *dir = nullptr;
    double2 *dinv = nullptr;
    double2 *vec = nullptr;     // 9 work vectors of ne: us, vs, w, rhs, x, r, z, p, q
    double *partial = nullptr;  // two sets of 4 per block: nb blocks (the start, the update), then kNsBlocks
    double *sc = nullptr;       // 12 scalars of the iteration
    int64_t nb = 0;

    double2 *v(int k) const { return vec + (size_t)k * ne; }
    FieldCsr csr() const { return FieldCsr{ne, rowptr, col, M, K, dir}; }
    void release() { *this = FieldState(); }   // the memory is the caller's
};

// Device state of the non-solenoidal solve (allocated by etpic_ns_setup).
struct NsState {
    bool ready = false;
    double eps = 0;
    int64_t nv = 0, ne = 0, nnz = 0, n_wall = 0;
    int32_t *rowptr = nullptr, *col = nullptr, *ev = nullptr;
    double *S = nullptr, *dinv = nullptr;
    uint8_t *wall = nullptr;
    double *vec = nullptr;      // 8 vectors of nv: x, r, z, p, q, the solutions (re, im) of the correction and
                                // that of the source projection
    double *partial = nullptr;  // two sets of 4 per block (kNsBlocks blocks)
    double *sc = nullptr;       // 12 scalars of the iteration
    double *bzero = nullptr;    // 2*N_f zeros: the face envelope of a loop without external fields
    double *ezero = nullptr;    // 2*N_e zeros: its edge envelope

    double *v(int k) const { return vec + (size_t)k * nv; }
    NsCsr csr() const { return NsCsr{nv, rowptr, col, S}; }
    void release() { *this = NsState(); }   // the memory is the caller's
};

// Device pointers of one (snap[1] NULL) or three envelope snapshots; the dc
// DoFs are those of snap[0] (one snapshot) or snap[1] (three).
FieldPtrs field_ptrs(const etpic_fields *const snap[3], const double w[3], double c, double s) {
    FieldPtrs F{};
    const bool three = snap[1] != nullptr;
    for (int k = 0; k < 3; ++k) {
        const etpic_fields *f = three ? snap[k] : snap[0];
        F.e_env[k] = reinterpret_cast<const double2 *>(f->e_env);
        F.b_env[k] = reinterpret_cast<const double2 *>(f->b_env);
        F.w[k] = w[k];
    }
    const etpic_fields *dc = three ? snap[1] : snap[0];
    F.e_dc = dc->e_dc;
    F.b_dc = dc->b_dc;
    F.c = c;
    F.s = s;
    return F;
}

// One step of a multi-step call: the envelope snapshots (snap[1] NULL for
// one snapshot), their weights and the gather time.
struct StepPlan {
    const etpic_fields *snap[3];
    double w[3];
    double t;
};

// Launch of one kernel of a timed step sequence.  With events the kernel's
// own dispatch carries them (hipExtLaunchKernel binds e0 to its start and e1
// to its end), so timing inserts no marker packets between the kernels of a
// step; without, a plain launch.  Errors are left for hipGetLastError.
template <typename... P, typename... A>
void launch_timed(void (*k)(P...), dim3 grid, hipStream_t st, hipEvent_t e0, hipEvent_t e1, A... args) {
    if (e0)
        hipExtLaunchKernelGGL(k, grid, dim3(kBlock), 0, st, e0, e1, 0, static_cast<P>(args)...);
    else
        hipLaunchKernelGGL(k, grid, dim3(kBlock), 0, st, static_cast<P>(args)...);
}

struct etpic_ctx {
    int device = 0;
    etpic::HostMesh host;
    bool has_mesh = false;
    uint64_t mesh_hash = 0;   // hash of the uploaded mesh (particle checkpoints resume on it only)
    TetTopo *d_topo = nullptr;
    double *d_grad64 = nullptr;
    double *d_gpush64 = nullptr;     // nt rows of PushRow<double>
    float *d_gpush32 = nullptr;       // nt rows of PushRow<float>
    double *d_geo64 = nullptr;        // nt rows of GeoRow<double>
    float *d_geo32 = nullptr;         // nt rows of GeoRow<float>
    int32_t *d_tetface = nullptr;     // nt*4 face ids (face k opposite vertex k)
    void *d_coef = nullptr;          // nt*24 doubles: the step's CoefRow rows, or A_0..3, C_0..3 for the adjoint
    double *d_coef_env = nullptr;    // nt*kEnvRow complex-envelope rows (bound by etpic_ds_rows_bind)
    int32_t *d_v2e_ptr = nullptr;
    int32_t *d_v2e_code = nullptr;
    int32_t *d_e2s_ptr = nullptr;    // edge -> tet-slot CSR (ne+1)
    int32_t *d_e2s_slot = nullptr;   // its slots, 8 * tet + local edge (6 nt)
    double *d_tetG[2] = {nullptr, nullptr};  // per-tet current slots (nt*8 each), alternate per call
    int tetG_cur = 0;
    double *d_xyz = nullptr;         // 3*nv vertex coordinates
    int32_t *d_grid = nullptr;       // start tets of the point-location grid
    GridArgs grid{};
    bool has_ws = false;             // context workspace bound (etpic_workspace_bind)
    unsigned *d_status = nullptr;    // device status word
    unsigned *d_walk_queue = nullptr;  // kWalkQueueCap particle indices
    unsigned *d_slice_queue = nullptr; // kWalkQueueCap slice indices
    unsigned *d_walk_ctr = nullptr;    // 3 counters of the walk queues
    unsigned long long *d_red = nullptr;  // 2 words for the residual maxima
    double *d_scratch = nullptr;          // device address of `scratch` on this device
    // mean same-tet run length from the last sort (sum count^2 / N_p), read
    // back without blocking: the device word, its pinned host copy, the event
    // that marks the copy, and the value in use (0 until a sort has been seen)
    unsigned long long *d_runstat = nullptr;
    unsigned long long *h_runstat = nullptr;
    hipEvent_t runstat_ev = nullptr;
    bool runstat_pending = false;
    int64_t runstat_n = 0;
    double run_len = 0.0;
    int last_slices = 0;             // slices per wavefront of the last particle-kernel launch
    unsigned *d_count = nullptr;     // nt+1 counting-sort counters
    unsigned *d_tilesum = nullptr;   // scan tile totals
    int64_t tiles = 0;
    FieldState field;
    NsState ns;
    // Timing of steps run with ETPIC_STEP_TIMING: per step a set of start and
    // stop events of its kernels, interval k = 0 coefficient pass, 1 particle
    // kernel, 2 walk, 3 edge gather of the per-tet sums, each bound to its
    // kernel's dispatch (launch_timed); `has` marks the intervals launched
    // (a coefficient pass that ran inside the previous walk launch has none),
    // `sorting` whether the particle kernel also sorted (k_push_sort).  The
    // sets are created with the context (a fixed pool of kTimingSets, the
    // vectors reserved so that pointers to sets stay valid);
    // etpic_kernel_time returns the read sets to the pool.
    struct TimingSet {
        std::array<hipEvent_t, 8> ev{};
        unsigned has = 0;
        bool sorting = false;
    };
    std::vector<TimingSet> timing;
    std::vector<TimingSet> spare;
    // host-side systems built by a size query, kept for the setup call that follows
    std::unique_ptr<etpic::FieldSystem> field_pending;
    double field_pending_eps = 0, field_pending_mu = 0;
    std::unique_ptr<etpic::NsSystem> ns_pending;
    double ns_pending_eps = 0;

    int timing_events(TimingSet **ts, bool sorting = false) {
        if (spare.empty())
            return fail(ETPIC_EINVAL, "step timing: all %d event sets in use (etpic_kernel_time returns them)",
                        kTimingSets);
        timing.push_back(spare.back());
        spare.pop_back();
        timing.back().has = 0;
        timing.back().sorting = sorting;
        *ts = &timing.back();
        return ETPIC_OK;
    }
    // start / stop event of interval k of a timing set (none without a set)
    static hipEvent_t ev_start(TimingSet *ts, int k) {
        if (!ts) return nullptr;
        ts->has |= 1u << k;
        return ts->ev[2 * k];
    }
    static hipEvent_t ev_stop(TimingSet *ts, int k) { return ts ? ts->ev[2 * k + 1] : nullptr; }

    template <typename Real>
    StepArgs<Real> step_args(const etpic_particles *p, const etpic_species *sp, double dt, double *dG,
                             double *rho) const {
        StepArgs<Real> a{};
        a.n = p->n;
        a.nt = host.nt;
        a.lam1 = p->lam[0];
        a.lam2 = p->lam[1];
        a.lam3 = p->lam[2];
        a.v0 = static_cast<Real *>(p->vel[0]);
        a.v1 = static_cast<Real *>(p->vel[1]);
        a.v2 = static_cast<Real *>(p->vel[2]);
        a.tet = p->tet;
        a.coef = static_cast<const Real *>(d_coef);
        a.gpush = gpush_table<Real>();
        a.geo = geo_table<Real>();
        a.grad = d_grad64;
        a.topo = d_topo;
        a.dG = dG;
        a.rho = rho;
        a.status = d_status;
        a.walk_queue = d_walk_queue;
        a.slice_queue = d_slice_queue;
        a.walk_ctr = d_walk_ctr;
        a.gpush64 = d_gpush64;
        a.tetface = d_tetface;
        a.qw = sp->q * sp->w;
        a.h = (Real)(sp->q * dt / (2.0 * sp->m));
        a.dt_r = (Real)dt;
        return a;
    }

    // One step: carrier phase in float64 on the host (t = step*dt, argument
    // reduced by libm), per-tet coefficients, particle kernel, walk kernel.
    template <typename Real>
    int step(const etpic_particles *p, const etpic_species *sp, const etpic_fields *f, int64_t step, double dt,
             double omega, double *dG, double *rho, uint32_t flags, void *stream) {
        StepPlan plan{{f, nullptr, nullptr}, {1.0, 0.0, 0.0}, (double)step * dt};
        return run_steps<Real>(p, sp, &plan, 1, dt, omega, dG, rho, flags, stream);
    }

    // XCD-contiguous coefficient pass when an eighth of the edge and face DoFs
    // (complex edge and face envelopes, dc face DoFs) fits one 4 MB L2
    int coef_xcd() const { return (16 * host.ne + 24 * host.nf) / 8 <= (int64_t)4 << 20 ? 1 : 0; }

    template <typename Real>
    int launch_coef(const StepPlan &plan, double omega, hipStream_t s, TimingSet *ts = nullptr) {
        const int64_t nt = host.nt;
        FieldPtrs F = field_ptrs(plan.snap, plan.w, std::cos(omega * plan.t), std::sin(omega * plan.t));
        F.xcd = coef_xcd();
        hipEvent_t e0 = ev_start(ts, 0), e1 = ev_stop(ts, 0);
        Real *coef = static_cast<Real *>(d_coef);
        if (plan.snap[1])
            launch_timed(k_tet_coef<Real, 3, true>, grid_for(2 * nt), s, e0, e1, nt, d_gpush64, d_tetface, F, coef);
        else
            launch_timed(k_tet_coef<Real, 1, true>, grid_for(2 * nt), s, e0, e1, nt, d_gpush64, d_tetface, F, coef);
        HIP_TRY(hipGetLastError());
        return ETPIC_OK;
    }

    template <typename Real, bool kRho, bool kSort>
    bool launch_push(const StepArgs<Real> &a, int slices, int remap, hipStream_t st, TimingSet *ts = nullptr) {
        const int64_t n = a.n;
        hipEvent_t e0 = ev_start(ts, 1), e1 = ev_stop(ts, 1);
        if constexpr (std::is_same<Real, float>::value) {
            if (a.fixed) {
                switch (slices) {
                case 16:
                    if (kSort)
                        launch_timed(k_push_sort_slices_fixed<16, kRho>, grid_for((n + 15) / 16), st, e0, e1, a, remap);
                    else
                        launch_timed(k_push_slices_fixed<16, kRho>, grid_for((n + 15) / 16), st, e0, e1, a, remap);
                    break;
                case 4:
                    if (kSort)
                        launch_timed(k_push_sort_slices_fixed<4, kRho>, grid_for((n + 3) / 4), st, e0, e1, a, remap);
                    else
                        launch_timed(k_push_slices_fixed<4, kRho>, grid_for((n + 3) / 4), st, e0, e1, a, remap);
                    break;
                case 2:
                    if (!kSort && !kRho) {
                        launch_timed(k_push_pipe<true>, grid_for((n + 1) / 2), st, e0, e1, a, remap);
                        break;
                    }
                    [[fallthrough]];
                default:
                    if (kSort)
                        launch_timed(k_push_sort_fixed<kRho>, grid_for(n), st, e0, e1, a, remap);
                    else if (kRho)
                        launch_timed(k_push_rho_fixed, grid_for(n), st, e0, e1, a, remap);
                    else
                        launch_timed(k_push_fixed, grid_for(n), st, e0, e1, a, remap);
                    slices = 1;
                    break;
                }
                last_slices = slices;
                return slices == 2 || push_uses_slots<Real>(slices);
            }
        }
        switch (slices) {
        case 16:
            if (kSort)
                launch_timed(k_push_sort_slices<Real, 16, kRho>, grid_for((n + 15) / 16), st, e0, e1, a, remap);
            else
                launch_timed(k_push_slices<Real, 16, kRho>, grid_for((n + 15) / 16), st, e0, e1, a, remap);
            break;
        case 4:
            if (kSort)
                launch_timed(k_push_sort_slices<Real, 4, kRho>, grid_for((n + 3) / 4), st, e0, e1, a, remap);
            else
                launch_timed(k_push_slices<Real, 4, kRho>, grid_for((n + 3) / 4), st, e0, e1, a, remap);
            break;
        case 2:
            if constexpr (std::is_same<Real, float>::value) {
                if (!kSort && !kRho) {
                    launch_timed(k_push_pipe<false>, grid_for((n + 1) / 2), st, e0, e1, a, remap);
                    break;
                }
            }
            [[fallthrough]];
        default:
            if (kSort)
                launch_timed(k_push_sort<Real, kRho>, grid_for(n), st, e0, e1, a, remap);
            else if (kRho)
                launch_timed(k_push_rho<Real>, grid_for(n), st, e0, e1, a, remap);
            else
                launch_timed(k_push<Real>, grid_for(n), st, e0, e1, a, remap);
            slices = 1;
            break;
        }
        last_slices = slices;
        return slices == 2 || push_uses_slots<Real>(slices);
    }

    // Counting sort, first half: tet counts of src, the run-length statistic
    // for the slice choice (unless one is still in flight), and the exclusive
    // prefix sums of the counts in d_count (the scatter cursors).
    int sort_count(const etpic_particles *src, hipStream_t st) {
        const int64_t nt = host.nt, n = src->n, m = nt + 1;
        k_fill_u32<<<grid_for(m), kBlock, 0, st>>>(d_count, m, 0u);
        k_hist<<<grid_for(n), kBlock, 0, st>>>(n, nt, src->tet, d_count, d_status);
        if (!runstat_pending) {
            k_fill_u32<<<1, kBlock, 0, st>>>(reinterpret_cast<unsigned *>(d_runstat), 2, 0u);
            k_run_stat<<<(unsigned)std::min<int64_t>(grid_for(nt), 256), kBlock, 0, st>>>(nt, d_count, d_runstat);
            HIP_TRY(hipMemcpyAsync(h_runstat, d_runstat, sizeof(unsigned long long), hipMemcpyDeviceToHost, st));
            HIP_TRY(hipEventRecord(runstat_ev, st));
            runstat_pending = true;
            runstat_n = n;
        }
        k_scan_tiles<<<(unsigned)tiles, kBlock, 0, st>>>(d_count, m, d_tilesum);
        k_scan_sums<<<1, kBlock, 0, st>>>(d_tilesum, tiles);
        k_scan_add<<<grid_for(m), kBlock, 0, st>>>(d_count, m, d_tilesum);
        HIP_TRY(hipGetLastError());
        return ETPIC_OK;
    }

    template <typename Real>
    int sort(const etpic_particles *src, const etpic_particles *dst, hipStream_t st, const Real *hsrc = nullptr,
             Real *hdst = nullptr, int nh = 0, int fixed = 0) {
        if (int r = sort_count(src, st)) return r;
        k_scatter<Real><<<grid_for(src->n), kBlock, 0, st>>>(src->n, host.nt, src->tet, d_count, *src, *dst, hsrc,
                                                              hdst, nh, fixed);
        HIP_TRY(hipGetLastError());
        return ETPIC_OK;
    }

    // nsteps consecutive steps, step j at time plans[j].t with the envelope
    // sum_k w[k] snap[k] of plans[j]; rho (if any) after the last step.  Each
    // step is coefficient pass, particle kernel, walk kernel on the caller's
    // stream; between two steps of the call the walk and the next step's
    // coefficient pass share one launch (k_walk_coef).
    // With src, the particles of src are first counting-sorted by tet into p,
    // the scatter folded into the first step's particle kernel.
    template <typename Real>
    int run_steps(const etpic_particles *p, const etpic_species *sp, const StepPlan *plans, int nsteps, double dt,
                  double omega, double *dG, double *rho, uint32_t flags, void *stream,
                  const etpic_particles *src = nullptr) {
        hipStream_t st = static_cast<hipStream_t>(stream);
        const int remap = (flags & ETPIC_STEP_XCD_REMAP) ? 1 : 0;
        const int64_t n = p->n, nt = host.nt;
        const unsigned coef_blocks = grid_for(2 * nt);
        if (src)
            if (int r = sort_count(src, st)) return r;
        // ts: this step's timing set; ta: the same where every kernel is timed
        TimingSet *ts = nullptr;
        const bool time_all = (flags & ETPIC_STEP_TIMING_ALL) != 0;
        if (flags & (ETPIC_STEP_TIMING | ETPIC_STEP_TIMING_ALL))
            if (int r = timing_events(&ts, src != nullptr)) return r;
        TimingSet *ta = time_all ? ts : nullptr;
        if (int r = launch_coef<Real>(plans[0], omega, st, ta)) return r;
        double *slots = d_tetG[tetG_cur];
        bool used_slots = false;
        for (int j = 0; j < nsteps; ++j) {
            StepArgs<Real> a = step_args<Real>(p, sp, dt, dG, j == nsteps - 1 ? rho : nullptr);
            a.walk_by_slice = (flags & ETPIC_STEP_WALK_BY_SLICE) ? 1 : 0;
            a.fixed = (flags & kFlagFixed) ? 1 : 0;
            a.tetG = slots;
            if (j == 0 && src) {
                // read src, write p at the sorted positions; the walk then runs on p
                StepArgs<Real> as = a;
                as.lam1 = src->lam[0];
                as.lam2 = src->lam[1];
                as.lam3 = src->lam[2];
                as.v0 = static_cast<Real *>(src->vel[0]);
                as.v1 = static_cast<Real *>(src->vel[1]);
                as.v2 = static_cast<Real *>(src->vel[2]);
                as.tet = src->tet;
                as.o_lam1 = p->lam[0];
                as.o_lam2 = p->lam[1];
                as.o_lam3 = p->lam[2];
                as.o_v0 = static_cast<Real *>(p->vel[0]);
                as.o_v1 = static_cast<Real *>(p->vel[1]);
                as.o_v2 = static_cast<Real *>(p->vel[2]);
                as.o_tet = p->tet;
                as.id = src->id;
                as.o_id = p->id;
                as.cursor = d_count;
                if (as.rho)
                    used_slots |= launch_push<Real, true, true>(as, push_slices_for(flags, n, true), remap, st, ts);
                else
                    used_slots |= launch_push<Real, false, true>(as, push_slices_for(flags, n, true), remap, st, ts);
                a.scatter = 1;
            } else if (a.rho) {
                used_slots |= launch_push<Real, true, false>(a, push_slices_for(flags, n), remap, st, ts);
            } else {
                used_slots |= launch_push<Real, false, false>(a, push_slices_for(flags, n), remap, st, ts);
            }
            HIP_TRY(hipGetLastError());
            hipEvent_t w0 = ev_start(ta, 2), w1 = ev_stop(ta, 2);
            if (j + 1 < nsteps) {
                const StepPlan &nx = plans[j + 1];
                FieldPtrs F = field_ptrs(nx.snap, nx.w, std::cos(omega * nx.t), std::sin(omega * nx.t));
                F.xcd = coef_xcd();
                if (nx.snap[1])
                    launch_timed(k_walk_coef<Real, 3>, kWalkBlocks + coef_blocks, st, w0, w1, a, nt, F);
                else
                    launch_timed(k_walk_coef<Real, 1>, kWalkBlocks + coef_blocks, st, w0, w1, a, nt, F);
            } else {
                launch_timed(k_walk<Real>, kWalkBlocks, st, w0, w1, a);
                if (used_slots) {
                    // the call's per-tet sums onto the edges; the other slot
                    // buffer is cleared for the next call
                    HIP_TRY(hipGetLastError());
                    const int64_t ne = host.ne;
                    const unsigned gb = (unsigned)std::min<int64_t>(grid_for(std::max<int64_t>(ne, 8 * nt)), 4096);
                    launch_timed(k_slots_to_edges, gb, st, ev_start(ta, 3), ev_stop(ta, 3), ne, d_e2s_ptr,
                                 d_e2s_slot, slots, dG, d_tetG[tetG_cur ^ 1], 8 * nt);
                    tetG_cur ^= 1;
                }
            }
            HIP_TRY(hipGetLastError());
            // the next step's coefficient pass ran inside this launch (booked
            // as walk): its set has no coefficient interval
            if (ts && j + 1 < nsteps) {
                if (int r = timing_events(&ts)) return r;
                ta = time_all ? ts : nullptr;
            }
        }
        return ETPIC_OK;
    }

    template <typename Real>
    const Real *gpush_table() const;
    template <typename Real>
    const Real *geo_table() const;

    // Slices per wavefront of the particle kernel: forced by a flag, else from
    // the mean same-tet run length of the last sort (one slice while runs fit
    // in a wavefront; 4 or 16 for longer runs), kept to >= kMinPushWaves
    // wavefronts so that the chip stays full.
    int push_slices_for(uint32_t flags, int64_t n, bool sorting = false) {
        if (flags & ETPIC_STEP_SLICES_16) return last_slices = 16;
        if (flags & ETPIC_STEP_SLICES_4) return last_slices = 4;
        if (flags & ETPIC_STEP_SLICES_2) return last_slices = 2;
        if (flags & ETPIC_STEP_SLICES_1) return last_slices = 1;
        // The particle kernel adds a run's currents to its tet's slots, so
        // long runs cost it few same-address atomics: one slice measured
        // fastest up to hundreds of particles per tet (5e7 on 40^3 x 6 tets,
        // the 2e8 bunch), and slices are kept for thousands.  The sorting
        // form takes one cursor atomic per run and tet, which slices divide:
        // it keeps them from a hundred particles per tet on
        if (sorting) return last_slices = slices_from_runs(n, 96.0, 256.0);
        int s = slices_from_runs(n, 1024.0, 4096.0);
        // one slice: two pipelined ones (float forms; float64 keeps one) where
        // the float rows of the mesh (coefficient 48 B, push 64 B, geometry 48 B
        // per tet) outgrow the 256 MB Infinity Cache (measured: large box
        // mixed 4.09 -> 3.89 ms, compact 3.96 -> 3.79 ms; on the bench mesh,
        // whose rows fit, 2-5 % slower)
        if (s == 1 && host.nt * (int64_t)kFloatRowBytes > kInfinityCacheBytes && n / 128 >= kMinPushWaves) s = 2;
        return last_slices = s;
    }

    // 1, 4 or 16 slices from the last sort's mean same-tet run length (read
    // back without blocking: a statistic still in flight leaves the previous):
    // 4 from run length lo on, 16 from hi on
    int slices_from_runs(int64_t n, double lo, double hi) {
        if (runstat_pending && hipEventQuery(runstat_ev) == hipSuccess) {
            run_len = runstat_n > 0 ? (double)*h_runstat / (double)runstat_n : 0.0;
            runstat_pending = false;
        }
        (void)hipGetLastError();   // an unfinished query is not an error
        int s = run_len >= hi ? 16 : (run_len >= lo ? 4 : 1);
        while (s > 1 && n / (64 * (int64_t)s) < kMinPushWaves) s /= 4;
        return s;
    }

    // nsteps downshifted steps from step0 (t_n = n dt), hist0 of them taken
    // before; the complex-envelope rows are built once for the call.
    template <typename Real>
    int ds_steps(const etpic_particles *p, void *hist, const etpic_species *sp, const etpic_fields *f,
                 int64_t step0, int nsteps, int hist0, double dt, double omega, double *dG, double *rho,
                 uint32_t flags, void *stream) {
        hipStream_t st = static_cast<hipStream_t>(stream);
        const int remap = (flags & ETPIC_STEP_XCD_REMAP) ? 1 : 0;
        const int64_t n = p->n, nt = host.nt;
        if (!d_coef_env)
            return fail(ETPIC_ESTATE, "no downshifted rows bound (etpic_ds_rows_bytes, etpic_ds_rows_bind)");
        TimingSet *ts = nullptr;
        const bool time_all = (flags & ETPIC_STEP_TIMING_ALL) != 0;
        if (flags & (ETPIC_STEP_TIMING | ETPIC_STEP_TIMING_ALL))
            if (int r = timing_events(&ts)) return r;
        TimingSet *ta = time_all ? ts : nullptr;
        {
            const etpic_fields *snap[3] = {f, nullptr, nullptr};
            const double w1[3] = {1.0, 0.0, 0.0};
            const FieldPtrs F = field_ptrs(snap, w1, 1.0, 0.0);
            launch_timed(k_tet_coef_env, dim3(grid_for(nt), 6), st, ev_start(ta, 0), ev_stop(ta, 0), nt, d_gpush64,
                         d_tetface, F, d_coef_env);
            HIP_TRY(hipGetLastError());
        }
        for (int j = 0; j < nsteps; ++j) {
            const int64_t sn = step0 + j;
            const int H = hist0 + j;
            StepArgs<Real> a = step_args<Real>(p, sp, dt, dG, j == nsteps - 1 ? rho : nullptr);
            a.walk_by_slice = (flags & ETPIC_STEP_WALK_BY_SLICE) ? 1 : 0;
            DsArgs<Real> d{};
            d.coef_env = d_coef_env;
            d.hist = static_cast<Real *>(hist);
            d.stride = n;
            d.K = std::min(H, 2) + 1;
            d.A = std::min(H, 3) + 1;
            auto mod = [](int64_t x, int m) { return (int)(((x % m) + m) % m); };
            for (int i = 0; i < 3; ++i) d.vin[i] = i < H ? mod(sn - 1 - i, 4) : -1;
            d.vout = mod(sn, 4);
            for (int i = 0; i < 2; ++i) d.sin_[i] = i < H ? mod(sn - 1 - i, 2) : -1;
            d.sout = mod(sn, 2);
            DsWeights W;
            ds_weights(d.K, d.A, (double)sn * dt, dt, omega, W);
            for (int k = 0; k < 3; ++k) {
                d.Mr[k] = (Real)W.Mr[k];
                d.Mi[k] = (Real)W.Mi[k];
                d.P[k] = (Real)W.P[k];
            }
            for (int k = 0; k < 9; ++k) {
                d.Lr[k] = (Real)W.Lr[k];
                d.Li[k] = (Real)W.Li[k];
                d.Q[k] = (Real)W.Q[k];
            }
            for (int k = 0; k < 4; ++k) d.ab[k] = (Real)W.ab[k];
            d.qm = (Real)(sp->q / sp->m);
            d.edc = f->e_dc ? 1 : 0;
            if (a.rho)
                launch_timed(k_push_ds<Real, true>, grid_for(n), st, ev_start(ts, 1), ev_stop(ts, 1), a, d, remap);
            else
                launch_timed(k_push_ds<Real, false>, grid_for(n), st, ev_start(ts, 1), ev_stop(ts, 1), a, d, remap);
            HIP_TRY(hipGetLastError());
            launch_timed(k_walk_ds<Real>, kWalkBlocks, st, ev_start(ta, 2), ev_stop(ta, 2), a, d);
            HIP_TRY(hipGetLastError());
            if (ts && j + 1 < nsteps) {
                if (int r = timing_events(&ts)) return r;
                ta = time_all ? ts : nullptr;
            }
        }
        return ETPIC_OK;
    }

    // Weights of one downshifted step [t0, t0 + h] with K Lagrange nodes at
    // t0, t0 - h, t0 - 2h, in closed form: with s = (t - t0) / h the basis
    // polynomials have the monomial coefficients below, and
    // J_p = int_0^1 s^p e^{j theta s} ds (theta = w h) comes from its power
    // series for |theta| < 1 and from the integration-by-parts recurrence
    // J_p = (e^{j theta} - p J_{p-1}) / (j theta) above.
    static void ds_weights(int K, int A, double t0, double h, double omega, DsWeights &d) {
        using cplx = std::complex<double>;
        double cf[3][3] = {{0.0}};
        if (K == 1) {
            cf[0][0] = 1.0;
        } else if (K == 2) {
            cf[0][0] = 1.0, cf[0][1] = 1.0;      // 1 + s
            cf[1][1] = -1.0;                     // -s
        } else {
            cf[0][0] = 1.0, cf[0][1] = 1.5, cf[0][2] = 0.5;   // (s + 1)(s + 2) / 2
            cf[1][1] = -2.0, cf[1][2] = -1.0;                 // -s (s + 2)
            cf[2][1] = 0.5, cf[2][2] = 0.5;                   // s (s + 1) / 2
        }
        const double th = omega * h;
        cplx J[5];
        const cplx jt(0.0, th);
        if (std::fabs(th) < 1.0) {
            for (int q = 0; q < 5; ++q) {
                cplx sum = 0.0, term = 1.0;   // (j theta)^m / m!
                for (int m = 0; m < 30; ++m) {
                    sum += term / (double)(q + m + 1);
                    term *= jt / (double)(m + 1);
                }
                J[q] = sum;
            }
        } else {
            const cplx e = std::exp(jt);
            J[0] = (e - 1.0) / jt;
            for (int q = 1; q < 5; ++q) J[q] = (e - (double)q * J[q - 1]) / jt;
        }
        const cplx ph(std::cos(omega * t0), std::sin(omega * t0));
        for (int k = 0; k < 3; ++k) d.Mr[k] = d.Mi[k] = d.P[k] = 0.0;
        for (int k = 0; k < 9; ++k) d.Lr[k] = d.Li[k] = d.Q[k] = 0.0;
        for (int k = 0; k < K; ++k) {
            cplx mu = 0.0;
            double pk = 0.0;
            for (int q = 0; q < 3; ++q) {
                mu += cf[k][q] * J[q];
                pk += cf[k][q] / (q + 1);
            }
            mu *= h * ph;
            d.Mr[k] = mu.real();
            d.Mi[k] = -mu.imag();
            d.P[k] = h * pk;
            for (int jj = 0; jj < K; ++jj) {
                cplx la = 0.0;
                double qk = 0.0;
                for (int q1 = 0; q1 < 3; ++q1)
                    for (int q2 = 0; q2 < 3; ++q2) {
                        la += cf[jj][q1] * cf[k][q2] * J[q1 + q2];
                        qk += cf[jj][q1] * cf[k][q2] / (q1 + q2 + 1);
                    }
                la *= h * ph;
                d.Lr[jj * K + k] = la.real();
                d.Li[jj * K + k] = -la.imag();
                d.Q[jj * K + k] = h * qk;
            }
        }
        static const double kAB[4][4] = {{1.0, 0.0, 0.0, 0.0},
                                         {1.5, -0.5, 0.0, 0.0},
                                         {23.0 / 12.0, -16.0 / 12.0, 5.0 / 12.0, 0.0},
                                         {55.0 / 24.0, -59.0 / 24.0, 37.0 / 24.0, -9.0 / 24.0}};
        for (int i = 0; i < 4; ++i) d.ab[i] = h * kAB[A - 1][i];
    }

    // Forgets the mesh and everything derived from it (the buffers are the
    // caller's: nothing is freed here).
    void release() {
        d_topo = nullptr;
        d_grad64 = nullptr;
        d_gpush64 = nullptr;
        d_gpush32 = nullptr;
        d_geo64 = nullptr;
        d_geo32 = nullptr;
        d_tetface = nullptr;
        d_coef = nullptr;
        d_coef_env = nullptr;
        d_v2e_ptr = d_v2e_code = nullptr;
        d_e2s_ptr = d_e2s_slot = nullptr;
        d_tetG[0] = d_tetG[1] = nullptr;
        tetG_cur = 0;
        d_xyz = nullptr;
        d_grid = nullptr;
        grid = GridArgs{};
        d_count = d_tilesum = nullptr;
        field.release();
        ns.release();
        field_pending.reset();
        ns_pending.reset();
        has_mesh = false;
    }
};


// File-scope scratch of the allocation-free residual (each GPU holds its own
// copy for the life of the process): kResBlocks partial pairs, then the
// result pair (16 KB).  Host code never passes this name to a kernel or a
// copy: on the host it is a stand-in, not a device address.  The device
// address is taken once per device with hipGetSymbolAddress (scratch_address,
// called by etpic_create with the device current) and used everywhere instead.
static __device__ __align__(256) double scratch[kScratchDoubles];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mutex;
double *g_scratch_addr[kMaxDevices] = {};

// The device address of `scratch` on the current device `device`.
int scratch_address(int device, double **out) {
    if (device < 0 || device >= kMaxDevices) return fail(ETPIC_EINVAL, "device %d beyond %d", device, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_addr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(ETPIC_EHIP, "address of the residual scratch: %s", hipGetErrorString(e));
        g_scratch_addr[device] = static_cast<double *>(p);
    }
    *out = g_scratch_addr[device];
    return ETPIC_OK;
}
}  // namespace

template <>
const double *etpic_ctx::gpush_table<double>() const { return d_gpush64; }
template <>
const float *etpic_ctx::gpush_table<float>() const { return d_gpush32; }
template <>
const double *etpic_ctx::geo_table<double>() const { return d_geo64; }
template <>
const float *etpic_ctx::geo_table<float>() const { return d_geo32; }

namespace {

// Makes the context's device current; every call that launches kernels goes
// through here, so it also requires the context workspace (status word, walk
// queues, reduction words) to be bound.
int set_device(const etpic_ctx *ctx) {
    if (!ctx->has_ws) return fail(ETPIC_ESTATE, "no workspace bound (etpic_workspace_bytes, etpic_workspace_bind)");
    HIP_TRY(hipSetDevice(ctx->device));
    return ETPIC_OK;
}

// The device only (setup calls that copy tables but launch nothing).
int set_device_only(const etpic_ctx *ctx) {
    HIP_TRY(hipSetDevice(ctx->device));
    return ETPIC_OK;
}

// ETPIC_FP64, ETPIC_MIXED, and ETPIC_MIXED_FIXED where the entry point has the
// fixed-point form.
int check_precision(int precision, bool fixed_ok) {
    if (precision == ETPIC_FP64 || precision == ETPIC_MIXED) return ETPIC_OK;
    if (precision == ETPIC_MIXED_FIXED) {
        if (fixed_ok) return ETPIC_OK;
        return fail(ETPIC_EINVAL, "this entry point has no fixed-point (ETPIC_MIXED_FIXED) form");
    }
    return fail(ETPIC_EINVAL, "bad precision %d", precision);
}

// Public step flags: bit 31 is the library's own.
uint32_t step_flags(uint32_t flags, int precision) {
    return (flags & ~kFlagFixed) | (precision == ETPIC_MIXED_FIXED ? kFlagFixed : 0u);
}

int check_particles(const etpic_ctx *ctx, const etpic_particles *p) {
    if (!p) return fail(ETPIC_EINVAL, "null particle descriptor");
    if (p->n < 0) return fail(ETPIC_EINVAL, "negative particle count");
    if (p->n > (int64_t)kWalkQueueCap * 64) return fail(ETPIC_EINVAL, "particle count above 2^29");
    if (p->n == 0) return ETPIC_OK;
    for (int k = 0; k < 3; ++k)
        if (!p->lam[k] || !p->vel[k]) return fail(ETPIC_EINVAL, "null particle array");
    if (!p->tet) return fail(ETPIC_EINVAL, "null tet array");
    (void)ctx;
    return ETPIC_OK;
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Workspace of the differentiation entry points: ncp checkpoints and
// checkpoint_every segment slots, each a float64 particle state (lam, v, tet),
// then a scratch current accumulator.
struct AdjLayout {
    size_t arr8, arr4, state, slots_off, dG_off, total;
    int ncp;
};

AdjLayout adj_layout(int64_t n, int64_t ne, int nsteps, int every) {
    AdjLayout L{};
    L.arr8 = align256(sizeof(double) * (size_t)n);
    L.arr4 = align256(sizeof(int32_t) * (size_t)n);
    L.state = 6 * L.arr8 + L.arr4;
    L.ncp = (nsteps + every - 1) / every;
    L.slots_off = (size_t)L.ncp * L.state;
    L.dG_off = L.slots_off + (size_t)every * L.state;
    L.total = L.dG_off + align256(sizeof(double) * (size_t)ne);
    return L;
}

etpic_particles state_view(void *ws, size_t off, const AdjLayout &L, int64_t n) {
    char *b = static_cast<char *>(ws) + off;
    etpic_particles q{};
    q.n = n;
    for (int k = 0; k < 3; ++k) {
        q.lam[k] = reinterpret_cast<double *>(b + k * L.arr8);
        q.vel[k] = b + (3 + k) * L.arr8;
    }
    q.tet = reinterpret_cast<int32_t *>(b + 6 * L.arr8);
    q.id = nullptr;
    return q;
}

int copy_state(const etpic_particles &src, const etpic_particles &dst, int64_t n, hipStream_t st) {
    for (int k = 0; k < 3; ++k) {
        HIP_TRY(hipMemcpyAsync(dst.lam[k], src.lam[k], sizeof(double) * n, hipMemcpyDeviceToDevice, st));
        HIP_TRY(hipMemcpyAsync(dst.vel[k], src.vel[k], sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    }
    HIP_TRY(hipMemcpyAsync(dst.tet, src.tet, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, st));
    return ETPIC_OK;
}

int check_step_args(const etpic_ctx *ctx, const etpic_species *sp, const etpic_fields *f, double dt, double omega) {
    if (!ctx || !sp || !f) return fail(ETPIC_EINVAL, "null argument");
    if (!ctx->has_mesh) return fail(ETPIC_ESTATE, "no mesh uploaded");
    if (!f->e_env || !f->b_env) return fail(ETPIC_EINVAL, "null envelope DoFs");
    if (!(std::isfinite(dt) && std::isfinite(omega) && sp->m != 0.0 && std::isfinite(sp->q) && std::isfinite(sp->m)))
        return fail(ETPIC_EINVAL, "non-finite dt / omega or zero mass");
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
    // host-side resources only: the pinned word the run-length statistic is
    // read into, its event, the step-timing events; device memory comes from
    // the caller (etpic_workspace_bind, etpic_mesh_upload, ...)
    hipError_t e = hipSetDevice(device);
    if (e == hipSuccess) e = hipHostMalloc(&c->h_runstat, sizeof(unsigned long long), hipHostMallocDefault);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&c->runstat_ev, hipEventDisableTiming);
    c->spare.reserve(kTimingSets);
    c->timing.reserve(kTimingSets);
    for (int k = 0; k < kTimingSets && e == hipSuccess; ++k) {
        etpic_ctx::TimingSet set{};
        int made = 0;
        for (auto &x : set.ev) {
            // timing only: no system-scope fence when the event completes (no
            // cache writeback and invalidation between the kernels it times)
            e = hipEventCreateWithFlags(&x, hipEventDisableSystemFence);
            if (e != hipSuccess) break;
            ++made;
        }
        if (e != hipSuccess)
            for (int i = 0; i < made; ++i) (void)hipEventDestroy(set.ev[i]);
        else
            c->spare.push_back(set);
    }
    int rs = ETPIC_OK;
    if (e == hipSuccess) rs = scratch_address(device, &c->d_scratch);
    if (e != hipSuccess || rs != ETPIC_OK) {
        if (c->h_runstat) (void)hipHostFree(c->h_runstat);
        if (c->runstat_ev) (void)hipEventDestroy(c->runstat_ev);
        for (auto &set : c->spare)
            for (auto x : set.ev) (void)hipEventDestroy(x);
        delete c;
        if (rs != ETPIC_OK) return rs;
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
    (void)hipHostFree(ctx->h_runstat);
    (void)hipEventDestroy(ctx->runstat_ev);
    for (auto &e : ctx->timing)
        for (auto x : e.ev) (void)hipEventDestroy(x);
    for (auto &e : ctx->spare)
        for (auto x : e.ev) (void)hipEventDestroy(x);
    delete ctx;
    return ETPIC_OK;
}

}  // extern "C"

namespace {

// Context workspace: the status word, the residual and run-length words, the
// walk counters and the two walk queues.
struct WsPtrs {
    unsigned *status, *walk_ctr, *walk_queue, *slice_queue;
    unsigned long long *red, *runstat;
};
WsPtrs ws_layout(Carve &cv) {
    WsPtrs w;
    w.status = cv.take<unsigned>(1);
    w.walk_ctr = cv.take<unsigned>(3);
    w.red = cv.take<unsigned long long>(2);
    w.runstat = cv.take<unsigned long long>(1);
    w.walk_queue = cv.take<unsigned>(kWalkQueueCap);
    w.slice_queue = cv.take<unsigned>(kWalkQueueCap);
    return w;
}

int check_buffer(const void *buf, size_t bytes, size_t need, const char *what) {
    if (!buf) return fail(ETPIC_EINVAL, "%s: null buffer", what);
    if (reinterpret_cast<uintptr_t>(buf) & 255u) return fail(ETPIC_EINVAL, "%s: buffer not 256-byte aligned", what);
    if (bytes < need) return fail(ETPIC_EINVAL, "%s: buffer of %zu bytes, %zu needed", what, bytes, need);
    return ETPIC_OK;
}

// Mesh tables, in this order: tet topology, float64 gradients, float64 and
// float32 push rows, float64 and float32 geometry rows, tet-face ids, the
// coefficient table, vertex coordinates,
// point-location start grid, vertex -> edge CSR, sort counters and tile sums,
// edge -> tet-slot CSR, two per-tet current slot buffers.
struct MeshPtrs {
    TetTopo *topo;
    double *grad64, *gpush64, *geo64;
    float *gpush32, *geo32;
    int32_t *tetface;
    void *coef;
    double *xyz;
    int32_t *grid, *v2e_ptr, *v2e_code;
    unsigned *count, *tilesum;
    int32_t *e2s_ptr, *e2s_slot;
    double *tetG[2];
};
MeshPtrs mesh_layout(Carve &cv, const etpic::HostMesh &M, size_t grid_cells) {
    const int64_t nt = M.nt;
    MeshPtrs m;
    m.topo = cv.take<TetTopo>(nt);
    m.grad64 = cv.take<double>(12 * nt);
    m.gpush64 = cv.take<double>((size_t)PushRow<double>::kStride * nt);
    m.gpush32 = cv.take<float>((size_t)PushRow<float>::kStride * nt);
    m.geo64 = cv.take<double>((size_t)GeoRow<double>::kStride * nt);
    m.geo32 = cv.take<float>((size_t)GeoRow<float>::kStride * nt);
    m.tetface = cv.take<int32_t>(4 * nt);
    m.coef = cv.take<double>(24 * nt);
    m.xyz = cv.take<double>(3 * M.nv);
    m.grid = cv.take<int32_t>(grid_cells);
    m.v2e_ptr = cv.take<int32_t>(M.nv + 1);
    m.v2e_code = cv.take<int32_t>(2 * M.ne);
    m.count = cv.take<unsigned>(nt + 1);
    m.tilesum = cv.take<unsigned>((nt + 1 + kScanTile - 1) / kScanTile);
    m.e2s_ptr = cv.take<int32_t>(M.ne + 1);
    m.e2s_slot = cv.take<int32_t>(6 * nt);
    m.tetG[0] = cv.take<double>(8 * nt);
    m.tetG[1] = cv.take<double>(8 * nt);
    return m;
}

int host_mesh(int64_t n_vert, const double *xyz_host, int64_t n_tet, const int32_t *tet_vert_host,
              etpic::HostMesh &M, etpic::StartGrid &sg) {
    if (!xyz_host || !tet_vert_host) return fail(ETPIC_EINVAL, "mesh: null array");
    std::string err;
    int rc = etpic::build_host_mesh(n_vert, xyz_host, n_tet, tet_vert_host, M, err);
    if (rc == -1) return fail(ETPIC_EINVAL, "mesh: %s", err.c_str());
    if (rc != 0) return fail(ETPIC_EMESH, "mesh: %s", err.c_str());
    etpic::build_start_grid(M, xyz_host, 2.0, sg);
    return ETPIC_OK;
}

}  // namespace

extern "C" {

int etpic_workspace_bytes(size_t *bytes) {
    if (!bytes) return fail(ETPIC_EINVAL, "null argument");
    Carve cv;
    (void)ws_layout(cv);
    *bytes = cv.used;
    return ETPIC_OK;
}

int etpic_workspace_bind(etpic_ctx *ctx, void *dev_buf, size_t bytes) {
    if (!ctx) return fail(ETPIC_EINVAL, "null context");
    size_t need = 0;
    (void)etpic_workspace_bytes(&need);
    if (int r = check_buffer(dev_buf, bytes, need, "workspace")) return r;
    if (int r = set_device_only(ctx)) return r;
    HIP_TRY(hipDeviceSynchronize());
    Carve cv;
    cv.base = static_cast<char *>(dev_buf);
    cv.cap = bytes;
    const WsPtrs w = ws_layout(cv);
    ctx->d_status = w.status;
    ctx->d_walk_ctr = w.walk_ctr;
    ctx->d_red = w.red;
    ctx->d_runstat = w.runstat;
    ctx->d_walk_queue = w.walk_queue;
    ctx->d_slice_queue = w.slice_queue;
    HIP_TRY(hipMemset(ctx->d_status, 0, sizeof(unsigned)));
    HIP_TRY(hipMemset(ctx->d_walk_ctr, 0, 3 * sizeof(unsigned)));
    HIP_TRY(hipDeviceSynchronize());
    ctx->runstat_pending = false;
    ctx->has_ws = true;
    return ETPIC_OK;
}

int etpic_mesh_sizes(int64_t n_vert, const double *xyz_host, int64_t n_tet, const int32_t *tet_vert_host,
                     int64_t counts_out[4], size_t *dev_bytes) {
    if (!counts_out || !dev_bytes) return fail(ETPIC_EINVAL, "null output");
    etpic::HostMesh M;
    etpic::StartGrid sg;
    if (int r = host_mesh(n_vert, xyz_host, n_tet, tet_vert_host, M, sg)) return r;
    counts_out[0] = M.nv;
    counts_out[1] = M.ne;
    counts_out[2] = M.nf;
    counts_out[3] = M.nt;
    Carve cv;
    (void)mesh_layout(cv, M, sg.cell.size());
    *dev_bytes = cv.used;
    return ETPIC_OK;
}

int etpic_mesh_upload(etpic_ctx *ctx, int64_t n_vert, const double *xyz_host, int64_t n_tet,
                      const int32_t *tet_vert_host, void *dev_buf, size_t bytes) {
    if (!ctx) return fail(ETPIC_EINVAL, "null context");
    etpic::HostMesh M;
    etpic::StartGrid sg;
    if (int r = host_mesh(n_vert, xyz_host, n_tet, tet_vert_host, M, sg)) return r;
    size_t need = 0;
    {
        Carve cv;
        (void)mesh_layout(cv, M, sg.cell.size());
        need = cv.used;
    }
    if (int r = check_buffer(dev_buf, bytes, need, "mesh")) return r;
    if (int r = set_device_only(ctx)) return r;
    HIP_TRY(hipDeviceSynchronize());
    ctx->release();
    Carve cv;
    cv.base = static_cast<char *>(dev_buf);
    cv.cap = bytes;
    const MeshPtrs m = mesh_layout(cv, M, sg.cell.size());
    const int64_t nt = M.nt;
    ctx->d_topo = m.topo;
    ctx->d_grad64 = m.grad64;
    ctx->d_gpush64 = m.gpush64;
    ctx->d_gpush32 = m.gpush32;
    ctx->d_geo64 = m.geo64;
    ctx->d_geo32 = m.geo32;
    ctx->d_tetface = m.tetface;
    ctx->d_coef = m.coef;
    ctx->d_xyz = m.xyz;
    ctx->d_grid = m.grid;
    ctx->d_v2e_ptr = m.v2e_ptr;
    ctx->d_v2e_code = m.v2e_code;
    ctx->d_count = m.count;
    ctx->d_tilesum = m.tilesum;
    ctx->tiles = (nt + 1 + kScanTile - 1) / kScanTile;
    ctx->d_e2s_ptr = m.e2s_ptr;
    ctx->d_e2s_slot = m.e2s_slot;
    ctx->d_tetG[0] = m.tetG[0];
    ctx->d_tetG[1] = m.tetG[1];
    ctx->tetG_cur = 0;
    {
        constexpr int s64 = PushRow<double>::kStride, s32 = PushRow<float>::kStride;
        std::vector<double> gp64((size_t)nt * s64, 0.0);
        std::vector<float> gp32((size_t)nt * s32, 0.0f);
        std::vector<int32_t> tf((size_t)nt * 4);
        for (int64_t t = 0; t < nt; ++t) {
            for (int k = 0; k < 9; ++k) {
                gp64[s64 * t + k] = M.grad[12 * t + 3 + k];
                gp32[s32 * t + k] = (float)M.grad[12 * t + 3 + k];
            }
            std::memcpy(&gp64[s64 * t + PushRow<double>::kEdges], M.topo[t].e, sizeof(int32_t) * 6);
            std::memcpy(&gp32[s32 * t + PushRow<float>::kEdges], M.topo[t].e, sizeof(int32_t) * 6);
            std::memcpy(&tf[4 * t], M.topo[t].f, sizeof(int32_t) * 4);
        }
        HIP_TRY(hipMemcpy(ctx->d_gpush64, gp64.data(), sizeof(double) * s64 * nt, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(ctx->d_gpush32, gp32.data(), sizeof(float) * s32 * nt, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(ctx->d_tetface, tf.data(), sizeof(int32_t) * 4 * nt, hipMemcpyHostToDevice));
        // geometry rows: the edge vectors from local vertex 0 (canonical order)
        constexpr int g64 = GeoRow<double>::kStride, g32 = GeoRow<float>::kStride;
        std::vector<double> ge64((size_t)nt * g64, 0.0);
        std::vector<float> ge32((size_t)nt * g32, 0.0f);
        for (int64_t t = 0; t < nt; ++t) {
            const int64_t v0 = M.topo[t].v[0];
            for (int k = 1; k < 4; ++k)
                for (int c = 0; c < 3; ++c) {
                    const double d = xyz_host[3 * (int64_t)M.topo[t].v[k] + c] - xyz_host[3 * v0 + c];
                    ge64[g64 * t + 3 * (k - 1) + c] = d;
                    ge32[g32 * t + 3 * (k - 1) + c] = (float)d;
                }
        }
        HIP_TRY(hipMemcpy(ctx->d_geo64, ge64.data(), sizeof(double) * g64 * nt, hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(ctx->d_geo32, ge32.data(), sizeof(float) * g32 * nt, hipMemcpyHostToDevice));
    }
    HIP_TRY(hipMemcpy(ctx->d_xyz, xyz_host, sizeof(double) * 3 * M.nv, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(ctx->d_grid, sg.cell.data(), sizeof(int32_t) * sg.cell.size(), hipMemcpyHostToDevice));
    ctx->grid.cell = ctx->d_grid;
    for (int d = 0; d < 3; ++d) {
        ctx->grid.lo[d] = sg.lo[d];
        ctx->grid.inv[d] = sg.inv[d];
        ctx->grid.dims[d] = sg.dims[d];
    }
    HIP_TRY(hipMemcpy(ctx->d_topo, M.topo.data(), sizeof(TetTopo) * nt, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(ctx->d_grad64, M.grad.data(), sizeof(double) * 12 * nt, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(ctx->d_v2e_ptr, M.v2e_ptr.data(), sizeof(int32_t) * (M.nv + 1), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(ctx->d_v2e_code, M.v2e_code.data(), sizeof(int32_t) * 2 * M.ne, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(ctx->d_e2s_ptr, M.e2s_ptr.data(), sizeof(int32_t) * (M.ne + 1), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(ctx->d_e2s_slot, M.e2s_slot.data(), sizeof(int32_t) * 6 * nt, hipMemcpyHostToDevice));
    HIP_TRY(hipMemset(ctx->d_tetG[0], 0, sizeof(double) * 8 * nt));
    HIP_TRY(hipMemset(ctx->d_tetG[1], 0, sizeof(double) * 8 * nt));
    HIP_TRY(hipDeviceSynchronize());
    ctx->host = std::move(M);
    ctx->has_mesh = true;
    ctx->mesh_hash = etpic::ckpt::mesh_hash(n_vert, xyz_host, n_tet, tet_vert_host);
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

static int check_sort_pair(etpic_ctx *ctx, const etpic_particles *src, const etpic_particles *dst) {
    if (!ctx || !src || !dst) return fail(ETPIC_EINVAL, "null argument");
    if (!ctx->has_mesh) return fail(ETPIC_ESTATE, "no mesh uploaded");
    if (int r = check_particles(ctx, src)) return r;
    if (int r = check_particles(ctx, dst)) return r;
    if (src->n != dst->n) return fail(ETPIC_EINVAL, "source and destination sizes differ");
    if ((src->id == nullptr) != (dst->id == nullptr)) return fail(ETPIC_EINVAL, "id array given on one side only");
    for (int k = 0; k < 3; ++k)
        if (src->lam[k] == dst->lam[k] || src->vel[k] == dst->vel[k])
            return fail(ETPIC_EINVAL, "sort needs distinct source and destination buffers");
    if (src->tet == dst->tet || (src->id && src->id == dst->id))
        return fail(ETPIC_EINVAL, "sort needs distinct source and destination buffers");
    return ETPIC_OK;
}

int etpic_gather_push_deposit(etpic_ctx *ctx, const etpic_particles *p, int precision, const etpic_species *sp,
                              const etpic_fields *f, int64_t step, double dt, double omega, double *dG,
                              double *rho, uint32_t flags, void *stream) {
    if (int r = check_step_args(ctx, sp, f, dt, omega)) return r;
    if (!dG) return fail(ETPIC_EINVAL, "null current accumulator");
    if (int r = check_particles(ctx, p)) return r;
    if (int r = check_precision(precision, true)) return r;
    if (p->n == 0) return ETPIC_OK;
    if (int r = set_device(ctx)) return r;
    flags = step_flags(flags, precision);
    if (precision == ETPIC_FP64) return ctx->step<double>(p, sp, f, step, dt, omega, dG, rho, flags, stream);
    return ctx->step<float>(p, sp, f, step, dt, omega, dG, rho, flags, stream);
}

int etpic_coarse_step(etpic_ctx *ctx, const etpic_particles *p, int precision, const etpic_species *sp,
                      const etpic_fields snap[3], double t_coarse, double dt_coarse, int fine_steps, double omega,
                      double *dG, double *rho, uint32_t flags, void *stream) {
    if (!snap) return fail(ETPIC_EINVAL, "null snapshot array");
    for (int k = 0; k < 3; ++k)
        if (int r = check_step_args(ctx, sp, &snap[k], dt_coarse, omega)) return r;
    if (!dG) return fail(ETPIC_EINVAL, "null current accumulator");
    if (fine_steps < 1 || !(dt_coarse > 0.0) || !std::isfinite(t_coarse))
        return fail(ETPIC_EINVAL, "need fine_steps >= 1, dt_coarse > 0 and a finite t_coarse");
    if (int r = check_particles(ctx, p)) return r;
    if (int r = check_precision(precision, true)) return r;
    if (p->n == 0) return ETPIC_OK;
    if (int r = set_device(ctx)) return r;
    const double dt = dt_coarse / fine_steps;
    std::vector<StepPlan> plans((size_t)fine_steps);
    for (int j = 0; j < fine_steps; ++j) {
        // fine step j gathers at t = t_n + j dt; with u = j / M in [0, 1) the
        // quadratic Lagrange weights on the nodes u = -1, 0, 1 are
        // u(u - 1)/2, 1 - u^2, u(u + 1)/2
        const double u = (double)j / fine_steps;
        plans[j] = StepPlan{{&snap[0], &snap[1], &snap[2]},
                            {0.5 * u * (u - 1.0), 1.0 - u * u, 0.5 * u * (u + 1.0)},
                            t_coarse + j * dt};
    }
    flags = step_flags(flags, precision);
    if (precision == ETPIC_FP64)
        return ctx->run_steps<double>(p, sp, plans.data(), fine_steps, dt, omega, dG, rho, flags, stream);
    return ctx->run_steps<float>(p, sp, plans.data(), fine_steps, dt, omega, dG, rho, flags, stream);
}

int etpic_run_steps(etpic_ctx *ctx, const etpic_particles *p, int precision, const etpic_species *sp,
                    const etpic_fields *f, int64_t step0, int nsteps, double dt, double omega, double *dG,
                    double *rho, uint32_t flags, void *stream) {
    if (int r = check_step_args(ctx, sp, f, dt, omega)) return r;
    if (!dG) return fail(ETPIC_EINVAL, "null current accumulator");
    if (nsteps < 0) return fail(ETPIC_EINVAL, "negative step count");
    if (int r = check_particles(ctx, p)) return r;
    if (int r = check_precision(precision, true)) return r;
    if (p->n == 0 || nsteps == 0) return ETPIC_OK;
    if (int r = set_device(ctx)) return r;
    std::vector<StepPlan> plans((size_t)nsteps);
    for (int j = 0; j < nsteps; ++j) plans[j] = StepPlan{{f, nullptr, nullptr}, {1.0, 0.0, 0.0}, (double)(step0 + j) * dt};
    flags = step_flags(flags, precision);
    if (precision == ETPIC_FP64)
        return ctx->run_steps<double>(p, sp, plans.data(), nsteps, dt, omega, dG, rho, flags, stream);
    return ctx->run_steps<float>(p, sp, plans.data(), nsteps, dt, omega, dG, rho, flags, stream);
}

int etpic_sort_run_steps(etpic_ctx *ctx, const etpic_particles *src, const etpic_particles *dst, int precision,
                         const etpic_species *sp, const etpic_fields *f, int64_t step0, int nsteps, double dt,
                         double omega, double *dG, double *rho, uint32_t flags, void *stream) {
    if (int r = check_sort_pair(ctx, src, dst)) return r;
    if (int r = check_step_args(ctx, sp, f, dt, omega)) return r;
    if (!dG) return fail(ETPIC_EINVAL, "null current accumulator");
    if (nsteps < 1) return fail(ETPIC_EINVAL, "need at least one step");
    if (int r = check_precision(precision, true)) return r;
    if (src->n == 0) return ETPIC_OK;
    if (int r = set_device(ctx)) return r;
    std::vector<StepPlan> plans((size_t)nsteps);
    for (int j = 0; j < nsteps; ++j) plans[j] = StepPlan{{f, nullptr, nullptr}, {1.0, 0.0, 0.0}, (double)(step0 + j) * dt};
    flags = step_flags(flags, precision);
    if (precision == ETPIC_FP64)
        return ctx->run_steps<double>(dst, sp, plans.data(), nsteps, dt, omega, dG, rho, flags, stream, src);
    return ctx->run_steps<float>(dst, sp, plans.data(), nsteps, dt, omega, dG, rho, flags, stream, src);
}

static size_t ds_history_size(int64_t n, int precision) {
    return (precision == ETPIC_FP64 ? sizeof(double) : sizeof(float)) * (size_t)kDsArrays * (size_t)n;
}

int etpic_ds_rows_bytes(const etpic_ctx *ctx, size_t *bytes) {
    if (!ctx || !bytes) return fail(ETPIC_EINVAL, "null argument");
    if (!ctx->has_mesh) return fail(ETPIC_ESTATE, "no mesh uploaded");
    *bytes = sizeof(double) * (size_t)kEnvRow * (size_t)ctx->host.nt;
    return ETPIC_OK;
}

int etpic_ds_rows_bind(etpic_ctx *ctx, void *dev_buf, size_t bytes) {
    if (!ctx) return fail(ETPIC_EINVAL, "null context");
    size_t need = 0;
    if (int r = etpic_ds_rows_bytes(ctx, &need)) return r;
    if (int r = check_buffer(dev_buf, bytes, need, "downshifted rows")) return r;
    ctx->d_coef_env = static_cast<double *>(dev_buf);
    return ETPIC_OK;
}

int etpic_ds_history_bytes(int64_t n, int precision, size_t *bytes_out) {
    if (!bytes_out || n < 0) return fail(ETPIC_EINVAL, "bad arguments");
    if (int r = check_precision(precision, false)) return r;
    *bytes_out = ds_history_size(n, precision);
    return ETPIC_OK;
}

int etpic_ds_steps(etpic_ctx *ctx, const etpic_particles *p, int precision, void *hist, size_t hist_bytes,
                   const etpic_species *sp, const etpic_fields *f, int64_t step0, int nsteps, int hist0, double dt,
                   double omega, double *dG, double *rho, uint32_t flags, void *stream) {
    if (int r = check_step_args(ctx, sp, f, dt, omega)) return r;
    if (!dG) return fail(ETPIC_EINVAL, "null current accumulator");
    if (int r = check_particles(ctx, p)) return r;
    if (nsteps < 1 || hist0 < 0) return fail(ETPIC_EINVAL, "need nsteps >= 1 and hist0 >= 0");
    if (int r = check_precision(precision, false)) return r;
    if (!hist || hist_bytes < ds_history_size(p->n, precision))
        return fail(ETPIC_EINVAL, "history buffer missing or smaller than etpic_ds_history_bytes");
    if ((reinterpret_cast<uintptr_t>(hist) & 7) != 0) return fail(ETPIC_EINVAL, "history buffer not 8-byte aligned");
    if (p->n == 0) return ETPIC_OK;
    if (int r = set_device(ctx)) return r;
    if (precision == ETPIC_FP64)
        return ctx->ds_steps<double>(p, hist, sp, f, step0, nsteps, hist0, dt, omega, dG, rho, flags, stream);
    return ctx->ds_steps<float>(p, hist, sp, f, step0, nsteps, hist0, dt, omega, dG, rho, flags, stream);
}

int etpic_ds_sort(etpic_ctx *ctx, const etpic_particles *src, const etpic_particles *dst, int precision,
                  const void *hist_src, void *hist_dst, size_t hist_bytes, void *stream) {
    if (int r = check_sort_pair(ctx, src, dst)) return r;
    if (int r = check_precision(precision, false)) return r;
    const size_t need = ds_history_size(src->n, precision);
    if (!hist_src || !hist_dst || hist_bytes < need)
        return fail(ETPIC_EINVAL, "history buffers missing or smaller than etpic_ds_history_bytes");
    if (hist_src == hist_dst) return fail(ETPIC_EINVAL, "sort needs distinct history buffers");
    if (((reinterpret_cast<uintptr_t>(hist_src) | reinterpret_cast<uintptr_t>(hist_dst)) & 7) != 0)
        return fail(ETPIC_EINVAL, "history buffers not 8-byte aligned");
    if (src->n == 0) return ETPIC_OK;
    if (int r = set_device(ctx)) return r;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (precision == ETPIC_FP64)
        return ctx->sort<double>(src, dst, st, static_cast<const double *>(hist_src), static_cast<double *>(hist_dst),
                                 kDsArrays);
    return ctx->sort<float>(src, dst, st, static_cast<const float *>(hist_src), static_cast<float *>(hist_dst),
                            kDsArrays);
}

int etpic_adjoint_workspace(const etpic_ctx *ctx, int64_t n, int nsteps, int checkpoint_every, size_t *bytes_out) {
    if (!ctx || !bytes_out) return fail(ETPIC_EINVAL, "null argument");
    if (!ctx->has_mesh) return fail(ETPIC_ESTATE, "no mesh uploaded");
    if (n < 0 || nsteps < 0 || checkpoint_every < 1) return fail(ETPIC_EINVAL, "bad sizes");
    *bytes_out = adj_layout(n, ctx->host.ne, nsteps, checkpoint_every).total;
    return ETPIC_OK;
}

int etpic_forward_checkpointed(etpic_ctx *ctx, const etpic_particles *p, const etpic_species *sp,
                               const etpic_fields *f, int64_t step0, int nsteps, double dt, double omega,
                               int checkpoint_every, void *workspace, size_t workspace_bytes, double *dG,
                               void *stream) {
    if (int r = check_step_args(ctx, sp, f, dt, omega)) return r;
    if (int r = check_particles(ctx, p)) return r;
    if (nsteps < 0 || checkpoint_every < 1 || !workspace) return fail(ETPIC_EINVAL, "bad sizes or null workspace");
    const AdjLayout L = adj_layout(p->n, ctx->host.ne, nsteps, checkpoint_every);
    if (workspace_bytes < L.total) return fail(ETPIC_EINVAL, "workspace too small (%zu < %zu)", workspace_bytes, L.total);
    if (p->n == 0 || nsteps == 0) return ETPIC_OK;
    if (int r = set_device(ctx)) return r;
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *acc = dG ? dG : reinterpret_cast<double *>(static_cast<char *>(workspace) + L.dG_off);
    for (int k = 0; k < nsteps; ++k) {
        if (k % checkpoint_every == 0)
            if (int r = copy_state(*p, state_view(workspace, (size_t)(k / checkpoint_every) * L.state, L, p->n), p->n, st))
                return r;
        if (int r = ctx->step<double>(p, sp, f, step0 + k, dt, omega, acc, nullptr, ETPIC_STEP_XCD_REMAP, stream))
            return r;
    }
    return ETPIC_OK;
}

int etpic_backward(etpic_ctx *ctx, int64_t n, const etpic_species *sp, const etpic_fields *f, int64_t step0,
                   int nsteps, double dt, double omega, int checkpoint_every, void *workspace,
                   size_t workspace_bytes, double *const vbar[3], double *const xbar[3], double *grad_e,
                   void *stream) {
    if (int r = check_step_args(ctx, sp, f, dt, omega)) return r;
    if (n < 0 || nsteps < 0 || checkpoint_every < 1 || !workspace || !grad_e || !vbar || !xbar)
        return fail(ETPIC_EINVAL, "bad sizes or null pointer");
    for (int k = 0; k < 3; ++k)
        if (!vbar[k] || !xbar[k]) return fail(ETPIC_EINVAL, "null adjoint array");
    if (n > (int64_t)kWalkQueueCap * 64) return fail(ETPIC_EINVAL, "particle count above 2^29");
    const AdjLayout L = adj_layout(n, ctx->host.ne, nsteps, checkpoint_every);
    if (workspace_bytes < L.total) return fail(ETPIC_EINVAL, "workspace too small (%zu < %zu)", workspace_bytes, L.total);
    if (n == 0 || nsteps == 0) return ETPIC_OK;
    if (int r = set_device(ctx)) return r;
    hipStream_t st = static_cast<hipStream_t>(stream);
    double *scratch_dG = reinterpret_cast<double *>(static_cast<char *>(workspace) + L.dG_off);
    const int64_t nt = ctx->host.nt;
    for (int seg = L.ncp - 1; seg >= 0; --seg) {
        const int k0 = seg * checkpoint_every, k1 = std::min(nsteps, k0 + checkpoint_every);
        // recompute the states before steps k0 .. k1-1 into the slots
        const etpic_particles first = state_view(workspace, L.slots_off, L, n);
        if (int r = copy_state(state_view(workspace, (size_t)seg * L.state, L, n), first, n, st)) return r;
        for (int k = k0; k < k1 - 1; ++k) {
            const etpic_particles cur = state_view(workspace, L.slots_off + (size_t)(k - k0) * L.state, L, n);
            const etpic_particles nxt = state_view(workspace, L.slots_off + (size_t)(k - k0 + 1) * L.state, L, n);
            if (int r = copy_state(cur, nxt, n, st)) return r;
            if (int r = ctx->step<double>(&nxt, sp, f, step0 + k, dt, omega, scratch_dG, nullptr,
                                          ETPIC_STEP_XCD_REMAP, stream))
                return r;
        }
        for (int k = k1 - 1; k >= k0; --k) {
            const etpic_particles cur = state_view(workspace, L.slots_off + (size_t)(k - k0) * L.state, L, n);
            const double t = (double)(step0 + k) * dt;
            const double c = std::cos(omega * t), s = std::sin(omega * t);
            const etpic_fields *snap[3] = {f, nullptr, nullptr};
            const double w1[3] = {1.0, 0.0, 0.0};
            FieldPtrs F = field_ptrs(snap, w1, c, s);
            F.xcd = ctx->coef_xcd();
            k_tet_coef<double, 1><<<grid_for(2 * nt), kBlock, 0, st>>>(nt, ctx->d_gpush64, ctx->d_tetface, F,
                                                                       static_cast<double *>(ctx->d_coef));
            HIP_TRY(hipGetLastError());
            StepArgs<double> a = ctx->step_args<double>(&cur, sp, dt, scratch_dG, nullptr);
            AdjArgs b{};
            b.lam1 = cur.lam[0];
            b.lam2 = cur.lam[1];
            b.lam3 = cur.lam[2];
            b.v0 = static_cast<const double *>(cur.vel[0]);
            b.v1 = static_cast<const double *>(cur.vel[1]);
            b.v2 = static_cast<const double *>(cur.vel[2]);
            b.tet = cur.tet;
            b.vb0 = vbar[0];
            b.vb1 = vbar[1];
            b.vb2 = vbar[2];
            b.xb0 = xbar[0];
            b.xb1 = xbar[1];
            b.xb2 = xbar[2];
            b.grad_e = grad_e;
            b.c = c;
            b.s = s;
            b.dt = dt;
            k_adjoint<<<grid_for(n), kBlock, 0, st>>>(a, b);
            HIP_TRY(hipGetLastError());
        }
    }
    return ETPIC_OK;
}

int etpic_particles_locate(etpic_ctx *ctx, const etpic_particles *p, int precision, const double *const xyz[3],
                           const int32_t *hint, void *stream) {
    if (!ctx || !p || !xyz) return fail(ETPIC_EINVAL, "null argument");
    if (int r = check_precision(precision, true)) return r;
    if (!ctx->has_mesh) return fail(ETPIC_ESTATE, "no mesh uploaded");
    if (p->n < 0 || p->n > (int64_t)kWalkQueueCap * 64) return fail(ETPIC_EINVAL, "particle count outside [0, 2^29]");
    if (p->n == 0) return ETPIC_OK;
    if (!p->lam[0] || !p->lam[1] || !p->lam[2] || !p->tet || !xyz[0] || !xyz[1] || !xyz[2])
        return fail(ETPIC_EINVAL, "null particle or position array");
    if (int r = set_device(ctx)) return r;
    hipStream_t st = static_cast<hipStream_t>(stream);
    unsigned *fails = reinterpret_cast<unsigned *>(ctx->d_red);
    k_fill_u32<<<1, kBlock, 0, st>>>(fails, 1, 0u);
    k_locate<<<grid_for(p->n), kBlock, 0, st>>>(p->n, xyz[0], xyz[1], xyz[2], hint, ctx->host.nt, ctx->d_topo,
                                                ctx->d_grad64, ctx->d_xyz, ctx->grid, p->lam[0], p->lam[1],
                                                p->lam[2], p->tet, fails, precision == ETPIC_MIXED_FIXED ? 1 : 0);
    HIP_TRY(hipGetLastError());
    unsigned nfail = 0;
    HIP_TRY(hipMemcpyAsync(&nfail, fails, sizeof nfail, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (nfail)
        return fail(ETPIC_EPARTICLE, "%u of %lld points not located (outside the mesh, non-finite, or not reachable by "
                    "a straight walk from the start tet); their tet is set to -1", nfail, (long long)p->n);
    return ETPIC_OK;
}

int etpic_particles_positions(etpic_ctx *ctx, const etpic_particles *p, int precision, double *const xyz[3],
                              void *stream) {
    if (!ctx || !p || !xyz) return fail(ETPIC_EINVAL, "null argument");
    if (int r = check_precision(precision, true)) return r;
    if (!ctx->has_mesh) return fail(ETPIC_ESTATE, "no mesh uploaded");
    if (p->n < 0 || p->n > (int64_t)kWalkQueueCap * 64) return fail(ETPIC_EINVAL, "particle count outside [0, 2^29]");
    if (p->n == 0) return ETPIC_OK;
    if (!p->lam[0] || !p->lam[1] || !p->lam[2] || !p->tet || !xyz[0] || !xyz[1] || !xyz[2])
        return fail(ETPIC_EINVAL, "null particle or position array");
    if (int r = set_device(ctx)) return r;
    k_positions<<<grid_for(p->n), kBlock, 0, static_cast<hipStream_t>(stream)>>>(
        p->n, ctx->host.nt, p->lam[0], p->lam[1], p->lam[2], p->tet, ctx->d_topo, ctx->d_xyz, xyz[0], xyz[1], xyz[2],
        ctx->d_status, precision == ETPIC_MIXED_FIXED ? 1 : 0);
    HIP_TRY(hipGetLastError());
    return ETPIC_OK;
}

// ------------------------------------------------------------------ checkpoints
namespace {
// the particle arrays in the checkpoint file's order
void particle_arrays(const etpic_particles *p, void *arr[etpic::ckpt::kArrays]) {
    arr[0] = p->tet;
    for (int k = 0; k < 3; ++k) {
        arr[1 + k] = p->lam[k];
        arr[4 + k] = p->vel[k];
    }
    arr[7] = p->id;
}
}  // namespace

int etpic_checkpoint_write(etpic_ctx *ctx, const etpic_particles *p, int precision, int64_t step, const char *path,
                           void *stream) {
    if (!ctx || !p || !path) return fail(ETPIC_EINVAL, "null argument");
    if (int r = check_precision(precision, true)) return r;
    if (!ctx->has_mesh) return fail(ETPIC_ESTATE, "no mesh uploaded");
    if (int r = check_particles(ctx, p)) return r;
    if (int r = set_device_only(ctx)) return r;
    etpic::ckpt::Header h{};
    h.precision = (uint32_t)precision;
    h.n = p->n;
    h.step = step;
    h.n_tet = ctx->host.nt;
    h.n_vert = ctx->host.nv;
    h.mesh_hash = ctx->mesh_hash;
    h.has_id = p->id ? 1u : 0u;
    void *arr[etpic::ckpt::kArrays];
    particle_arrays(p, arr);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t herr = hipSuccess;
    auto fetch = [&](int k, size_t off, void *buf, size_t len) -> std::string {
        herr = hipMemcpyAsync(buf, static_cast<const char *>(arr[k]) + off, len, hipMemcpyDeviceToHost, st);
        if (herr == hipSuccess) herr = hipStreamSynchronize(st);
        return herr == hipSuccess ? std::string() : std::string("device to host copy: ") + hipGetErrorString(herr);
    };
    const std::string e = etpic::ckpt::write(path, h, fetch);
    if (!e.empty()) return fail(herr != hipSuccess ? ETPIC_EHIP : ETPIC_EIO, "checkpoint write: %s", e.c_str());
    return ETPIC_OK;
}

int etpic_checkpoint_info(const char *path, int64_t *n, int *precision, int64_t *step, int *has_id) {
    if (!path) return fail(ETPIC_EINVAL, "null path");
    etpic::ckpt::Header h{};
    const std::string e = etpic::ckpt::read_header(path, h);
    if (!e.empty()) return fail(ETPIC_EIO, "checkpoint: %s", e.c_str());
    if (n) *n = h.n;
    if (precision) *precision = (int)h.precision;
    if (step) *step = h.step;
    if (has_id) *has_id = (int)h.has_id;
    return ETPIC_OK;
}

int etpic_checkpoint_read(etpic_ctx *ctx, const etpic_particles *p, int precision, const char *path, int64_t *step,
                          void *stream) {
    if (!ctx || !p || !path) return fail(ETPIC_EINVAL, "null argument");
    if (int r = check_precision(precision, true)) return r;
    if (!ctx->has_mesh) return fail(ETPIC_ESTATE, "no mesh uploaded");
    if (int r = check_particles(ctx, p)) return r;
    etpic::ckpt::Header h{};
    {
        const std::string e = etpic::ckpt::read_header(path, h);
        if (!e.empty()) return fail(ETPIC_EIO, "checkpoint: %s", e.c_str());
    }
    if ((int)h.precision != precision)
        return fail(ETPIC_EINVAL, "checkpoint precision %u, particles given as %d", h.precision, precision);
    if (h.n != p->n)
        return fail(ETPIC_EINVAL, "checkpoint holds %lld particles, arrays hold %lld", (long long)h.n, (long long)p->n);
    if (h.n > 0 && (h.has_id != 0) != (p->id != nullptr))
        return fail(ETPIC_EINVAL, h.has_id ? "checkpoint has particle ids, no id array given"
                                           : "checkpoint has no particle ids, an id array was given");
    if (h.n_tet != ctx->host.nt || h.n_vert != ctx->host.nv || h.mesh_hash != ctx->mesh_hash)
        return fail(ETPIC_EMESH, "checkpoint taken on another mesh (%lld tets, %lld vertices)", (long long)h.n_tet,
                    (long long)h.n_vert);
    if (int r = set_device_only(ctx)) return r;
    void *arr[etpic::ckpt::kArrays];
    particle_arrays(p, arr);
    hipStream_t st = static_cast<hipStream_t>(stream);
    hipError_t herr = hipSuccess;
    auto store = [&](int k, size_t off, void *buf, size_t len) -> std::string {
        herr = hipMemcpyAsync(static_cast<char *>(arr[k]) + off, buf, len, hipMemcpyHostToDevice, st);
        if (herr == hipSuccess) herr = hipStreamSynchronize(st);
        return herr == hipSuccess ? std::string() : std::string("host to device copy: ") + hipGetErrorString(herr);
    };
    const std::string e = etpic::ckpt::read(path, h, store);
    if (!e.empty()) return fail(herr != hipSuccess ? ETPIC_EHIP : ETPIC_EIO, "checkpoint read: %s", e.c_str());
    if (step) *step = h.step;
    return ETPIC_OK;
}

int etpic_vertex_charge(etpic_ctx *ctx, const etpic_particles *p, int precision, const etpic_species *sp, double *rho,
                        void *stream) {
    if (!ctx || !sp || !rho) return fail(ETPIC_EINVAL, "null argument");
    if (int r = check_precision(precision, true)) return r;
    if (!ctx->has_mesh) return fail(ETPIC_ESTATE, "no mesh uploaded");
    if (int r = check_particles(ctx, p)) return r;
    if (p->n == 0) return ETPIC_OK;
    if (int r = set_device(ctx)) return r;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int fixed = precision == ETPIC_MIXED_FIXED ? 1 : 0;
    const int64_t n = p->n;
    // the charge's atomics go straight to the vertices: slices from shorter runs on
    switch (ctx->slices_from_runs(n, 96.0, 256.0)) {
    case 16:
        k_charge_slices<16><<<grid_for((n + 15) / 16), kBlock, 0, st>>>(n, ctx->host.nt, p->lam[0], p->lam[1],
                                                                        p->lam[2], p->tet, ctx->d_topo, sp->q * sp->w,
                                                                        rho, ctx->d_status, fixed);
        break;
    case 4:
        k_charge_slices<4><<<grid_for((n + 3) / 4), kBlock, 0, st>>>(n, ctx->host.nt, p->lam[0], p->lam[1], p->lam[2],
                                                                     p->tet, ctx->d_topo, sp->q * sp->w, rho,
                                                                     ctx->d_status, fixed);
        break;
    default:
        k_charge<<<grid_for(n), kBlock, 0, st>>>(n, ctx->host.nt, p->lam[0], p->lam[1], p->lam[2], p->tet, ctx->d_topo,
                                                 sp->q * sp->w, rho, ctx->d_status, fixed);
        break;
    }
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
    if (!std::isfinite(out_host[0]) || !std::isfinite(out_host[1]))
        return fail(ETPIC_ENAN, "continuity residual: non-finite current or charge (max|r| %g, max|rho_old| %g)",
                    out_host[0], out_host[1]);
    return ETPIC_OK;
}

int etpic_stream_probe(etpic_ctx *ctx, const etpic_particles *p, int precision, uint32_t flags, void *stream) {
    if (!ctx) return fail(ETPIC_EINVAL, "null context");
    if (int r = check_particles(ctx, p)) return r;
    if (int r = check_precision(precision, true)) return r;
    if (p->n == 0) return ETPIC_OK;
    if (int r = set_device(ctx)) return r;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int remap = (flags & ETPIC_STEP_XCD_REMAP) ? 1 : 0;
    if (precision == ETPIC_FP64)
        k_stream<double><<<grid_for(p->n), kBlock, 0, st>>>(
            p->n, p->lam[0], p->lam[1], p->lam[2], static_cast<double *>(p->vel[0]), static_cast<double *>(p->vel[1]),
            static_cast<double *>(p->vel[2]), p->tet, 0.0, remap, 0);
    else
        k_stream<float><<<grid_for(p->n), kBlock, 0, st>>>(
            p->n, p->lam[0], p->lam[1], p->lam[2], static_cast<float *>(p->vel[0]), static_cast<float *>(p->vel[1]),
            static_cast<float *>(p->vel[2]), p->tet, 0.0, remap, precision == ETPIC_MIXED_FIXED ? 1 : 0);
    HIP_TRY(hipGetLastError());
    return ETPIC_OK;
}

int etpic_gauss_residual_noalloc(etpic_ctx *ctx, const double *dG, const double *rho_new, const double *rho_old,
                                 double out_host[2], void *stream) {
    if (!ctx || !dG || !rho_new || !rho_old || !out_host) return fail(ETPIC_EINVAL, "null argument");
    if (!ctx->has_mesh) return fail(ETPIC_ESTATE, "no mesh uploaded");
    if (!ctx->d_scratch) return fail(ETPIC_ESTATE, "residual scratch address not taken");
    const int64_t nv = ctx->host.nv;
    if (nv > (int64_t)INT32_MAX) return fail(ETPIC_EINVAL, "%lld vertices beyond the 32-bit limit", (long long)nv);
    if (int r = set_device(ctx)) return r;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int nblk = (int)std::min<int64_t>(std::max<int64_t>(grid_for(nv), 1), kResBlocks);
    double *part = ctx->d_scratch, *res = ctx->d_scratch + 2 * kResBlocks;
    k_gauss_part<<<nblk, kBlock, 0, st>>>(nv, ctx->d_v2e_ptr, ctx->d_v2e_code, dG, rho_new, rho_old, part);
    k_gauss_final<<<1, kBlock, 0, st>>>(part, nblk, res);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipMemcpyAsync(out_host, res, 2 * sizeof(double), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (!std::isfinite(out_host[0]) || !std::isfinite(out_host[1]))
        return fail(ETPIC_ENAN, "continuity residual: non-finite current or charge (max|r| %g, max|rho_old| %g)",
                    out_host[0], out_host[1]);
    return ETPIC_OK;
}

int etpic_sort(etpic_ctx *ctx, const etpic_particles *src, const etpic_particles *dst, int precision,
               void *stream) {
    if (int r = check_sort_pair(ctx, src, dst)) return r;
    if (int r = check_precision(precision, true)) return r;
    if (src->n == 0) return ETPIC_OK;
    if (int r = set_device(ctx)) return r;
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (precision == ETPIC_FP64) return ctx->sort<double>(src, dst, st);
    return ctx->sort<float>(src, dst, st, nullptr, nullptr, 0, precision == ETPIC_MIXED_FIXED ? 1 : 0);
}

}  // extern "C"

namespace {

// Field solver arrays: CSR row pointers, columns, M and K values, Dirichlet
// mask, face -> edge table, Jacobi inverse diagonal, 9 complex work vectors,
// block partials and the 12 iteration scalars.
struct FieldPtrs2 {
    int32_t *rowptr, *col, *face_edge;
    double *M, *K, *partial, *sc;
    uint8_t *dir;
    double2 *dinv, *vec;
};
FieldPtrs2 field_layout(Carve &cv, int64_t ne, int64_t nf, int64_t nnz) {
    FieldPtrs2 f;
    const int64_t nb = std::max<int64_t>(grid_for(ne), kNsBlocks);
    f.rowptr = cv.take<int32_t>(ne + 1);
    f.col = cv.take<int32_t>(nnz);
    f.M = cv.take<double>(nnz);
    f.K = cv.take<double>(nnz);
    f.dir = cv.take<uint8_t>(ne);
    f.face_edge = cv.take<int32_t>(3 * nf);
    f.dinv = cv.take<double2>(ne);
    f.vec = cv.take<double2>(9 * ne);
    f.partial = cv.take<double>(4 * (nb + kNsBlocks));
    f.sc = cv.take<double>(12);
    return f;
}

// The host field system for (eps, mu): the one a size query built, else a new one.
int field_system(etpic_ctx *ctx, double eps, double mu) {
    if (ctx->field_pending && ctx->field_pending_eps == eps && ctx->field_pending_mu == mu) return ETPIC_OK;
    std::string err;
    auto S = std::make_unique<etpic::FieldSystem>();
    if (etpic::build_field_system(ctx->host, eps, mu, *S, err) != 0) return fail(ETPIC_EINVAL, "field: %s", err.c_str());
    ctx->field_pending = std::move(S);
    ctx->field_pending_eps = eps;
    ctx->field_pending_mu = mu;
    return ETPIC_OK;
}

}  // namespace

extern "C" {

int etpic_field_bytes(etpic_ctx *ctx, double eps, double mu, size_t *bytes) {
    if (!ctx || !bytes) return fail(ETPIC_EINVAL, "null argument");
    if (!ctx->has_mesh) return fail(ETPIC_ESTATE, "no mesh uploaded");
    if (!(eps > 0.0) || !(mu > 0.0)) return fail(ETPIC_EINVAL, "eps, mu must be positive");
    if (int r = field_system(ctx, eps, mu)) return r;
    const etpic::FieldSystem &S = *ctx->field_pending;
    Carve cv;
    (void)field_layout(cv, S.ne, S.nf, S.nnz);
    *bytes = cv.used;
    return ETPIC_OK;
}

int etpic_field_setup(etpic_ctx *ctx, double dt, double omega, double eps, double mu, void *dev_buf, size_t bytes) {
    if (!ctx) return fail(ETPIC_EINVAL, "null context");
    if (!ctx->has_mesh) return fail(ETPIC_ESTATE, "no mesh uploaded");
    if (!(dt > 0.0) || !std::isfinite(omega) || !(eps > 0.0) || !(mu > 0.0))
        return fail(ETPIC_EINVAL, "dt, eps, mu must be positive and omega finite");
    if (int r = field_system(ctx, eps, mu)) return r;
    const etpic::FieldSystem &S = *ctx->field_pending;
    size_t need = 0;
    {
        Carve cv;
        (void)field_layout(cv, S.ne, S.nf, S.nnz);
        need = cv.used;
    }
    if (int r = check_buffer(dev_buf, bytes, need, "field")) return r;
    const int64_t ne = S.ne;
    // Jacobi preconditioner: inverse diagonal of A = alpha M + beta K
    const double ar = 1.0 - 0.25 * omega * omega * dt * dt, ai = omega * dt, beta = 0.25 * dt * dt;
    std::vector<double2> dinv((size_t)ne);
    for (int64_t i = 0; i < ne; ++i) {
        double mii = 0.0, kii = 0.0;
        for (int32_t j = S.rowptr[i]; j < S.rowptr[i + 1]; ++j)
            if (S.col[j] == i) {
                mii = S.M[j];
                kii = S.K[j];
            }
        const double dr = ar * mii + beta * kii, di = ai * mii, den = dr * dr + di * di;
        if (!(den > 0.0)) return fail(ETPIC_EMESH, "field: zero diagonal at edge %lld", (long long)i);
        dinv[i] = make_double2(dr / den, -di / den);
    }
    if (int r = set_device_only(ctx)) return r;
    HIP_TRY(hipDeviceSynchronize());
    FieldState &F = ctx->field;
    F.release();
    F.dt = dt;
    F.omega = omega;
    F.eps = eps;
    F.mu = mu;
    F.ne = S.ne;
    F.nf = S.nf;
    F.nnz = S.nnz;
    F.nb = std::max<int64_t>(grid_for(ne), kNsBlocks);
    Carve cv;
    cv.base = static_cast<char *>(dev_buf);
    cv.cap = bytes;
    const FieldPtrs2 f = field_layout(cv, S.ne, S.nf, S.nnz);
    F.rowptr = f.rowptr;
    F.col = f.col;
    F.M = f.M;
    F.K = f.K;
    F.dir = f.dir;
    F.face_edge = f.face_edge;
    F.dinv = f.dinv;
    F.vec = f.vec;
    F.partial = f.partial;
    F.sc = f.sc;
    HIP_TRY(hipMemcpy(F.rowptr, S.rowptr.data(), sizeof(int32_t) * (ne + 1), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(F.col, S.col.data(), sizeof(int32_t) * S.nnz, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(F.M, S.M.data(), sizeof(double) * S.nnz, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(F.K, S.K.data(), sizeof(double) * S.nnz, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(F.dir, S.dirichlet.data(), sizeof(uint8_t) * ne, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(F.face_edge, S.face_edge.data(), sizeof(int32_t) * 3 * S.nf, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(F.dinv, dinv.data(), sizeof(double2) * ne, hipMemcpyHostToDevice));
    F.ready = true;
    ctx->field_pending.reset();
    return ETPIC_OK;
}

int etpic_field_nnz(const etpic_ctx *ctx, int64_t *nnz_out) {
    if (!ctx || !nnz_out) return fail(ETPIC_EINVAL, "null argument");
    if (!ctx->field.ready) return fail(ETPIC_ESTATE, "etpic_field_setup not called");
    *nnz_out = ctx->field.nnz;
    return ETPIC_OK;
}

int etpic_field_spmv(etpic_ctx *ctx, const double *x, double *y, double alpha_re, double alpha_im, double beta,
                     void *stream) {
    if (!ctx || !x || !y) return fail(ETPIC_EINVAL, "null argument");
    if (!ctx->field.ready) return fail(ETPIC_ESTATE, "etpic_field_setup not called");
    if (int r = set_device(ctx)) return r;
    const FieldState &F = ctx->field;
    k_field_spmv<<<grid_for(F.ne * kRowLanes), kBlock, 0, static_cast<hipStream_t>(stream)>>>(
        F.csr(), make_double2(alpha_re, alpha_im), beta, reinterpret_cast<const double2 *>(x),
        reinterpret_cast<double2 *>(y));
    HIP_TRY(hipGetLastError());
    return ETPIC_OK;
}

int etpic_field_step(etpic_ctx *ctx, double t_next, double *u, double *v, double *a, double *b, const double *gdd,
                     double tol, int max_iter, int *iters_out, double *resid_out, void *stream) {
    if (!ctx || !u || !v || !a || !b) return fail(ETPIC_EINVAL, "null argument");
    if (!ctx->field.ready) return fail(ETPIC_ESTATE, "etpic_field_setup not called");
    if (!(tol > 0.0) || max_iter < 1 || !std::isfinite(t_next)) return fail(ETPIC_EINVAL, "bad tol / max_iter / time");
    if (int r = set_device(ctx)) return r;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const FieldState &F = ctx->field;
    const int64_t ne = F.ne;
    const unsigned ge = grid_for(ne), gr = grid_for(ne * kRowLanes);
    const double dt = F.dt, w = F.omega;
    const double2 alpha = make_double2(1.0 - 0.25 * w * w * dt * dt, w * dt);
    const double beta = 0.25 * dt * dt;
    const double c = std::cos(w * t_next), s = std::sin(w * t_next);
    double2 *U = reinterpret_cast<double2 *>(u), *V = reinterpret_cast<double2 *>(v), *A = reinterpret_cast<double2 *>(a);
    double2 *us = F.v(0), *vs = F.v(1), *wv = F.v(2), *rhs = F.v(3), *x = F.v(4), *r = F.v(5), *z = F.v(6), *p = F.v(7),
            *q = F.v(8);
    k_nm_predict<<<ge, kBlock, 0, st>>>(ne, U, V, A, us, vs, wv, dt, w);
    k_nm_rhs<<<gr, kBlock, 0, st>>>(F.csr(), wv, us, gdd, c, s, rhs);
    // partial sets: the start and the update write the first, the product the second
    double *pa = F.partial, *pb = F.partial + 4 * F.nb;
    k_cocg_init<<<ge, kBlock, 0, st>>>(ne, rhs, F.dinv, x, r, z, p, q, pa, F.sc);
    HIP_TRY(hipGetLastError());
    const unsigned ga = (unsigned)std::min<int64_t>((ne * kRowLanes + kNsThreads - 1) / kNsThreads, kNsBlocks);
    const unsigned gu = (unsigned)std::min<int64_t>((ne + kNsVecThreads - 1) / kNsVecThreads, kNsBlocks);
    // iterations in batches of `check`; the host reads the scalars once per batch
    const int check = 5;
    const double tol2 = tol * tol;
    double hs[12];
    int k = 0;
    for (;;) {
        const int n = std::min(check, max_iter - k);
        for (int j = 0; j < n; ++j, ++k) {
            k_cocg_apply<<<ga, kNsThreads, 0, st>>>(F.csr(), alpha, beta, F.sc, z, p, q, pa, k == 0 ? (int64_t)ge : gu,
                                                    pb, k, tol2, 0);
            k_cocg_update<<<gu, kNsVecThreads, 0, st>>>(ne, F.sc, F.dinv, p, q, x, r, z, pb, ga, pa, k);
        }
        if (k >= max_iter)
            k_cocg_apply<<<ga, kNsThreads, 0, st>>>(F.csr(), alpha, beta, F.sc, z, p, q, pa, k == 0 ? (int64_t)ge : gu,
                                                    pb, k, tol2, 1);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(hs, F.sc, sizeof hs, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (hs[10] != 0.0 || k >= max_iter) break;
    }
    const double rel = hs[9] > 0.0 ? std::sqrt(hs[8] / hs[9]) : 0.0;
    const int it = (int)hs[11];
    if (iters_out) *iters_out = it;
    if (resid_out) *resid_out = rel;
    if (hs[10] == 0.0 || !std::isfinite(rel)) return fail(ETPIC_ENOCONV, "COCG: relative residual %.3e after %d iterations", rel, it);
    k_nm_faraday<<<grid_for(F.nf), kBlock, 0, st>>>(F.nf, F.face_edge, U, us, x, reinterpret_cast<double2 *>(b), dt, w);
    k_nm_correct<<<ge, kBlock, 0, st>>>(ne, us, vs, x, U, V, A, dt);
    HIP_TRY(hipGetLastError());
    return ETPIC_OK;
}

}  // extern "C"

namespace {

// Gauss-law solver arrays: CSR row pointers, columns, edge -> vertex table,
// values, Jacobi inverse diagonal, wall mask, 8 work vectors, block partials,
// the 12 iteration scalars, and zero face / edge envelopes.
struct NsPtrs {
    int32_t *rowptr, *col, *ev;
    double *S, *dinv, *vec, *partial, *sc, *bzero, *ezero;
    uint8_t *wall;
};
NsPtrs ns_layout(Carve &cv, int64_t nv, int64_t ne, int64_t nf, int64_t nnz) {
    NsPtrs n;
    n.rowptr = cv.take<int32_t>(nv + 1);
    n.col = cv.take<int32_t>(nnz);
    n.ev = cv.take<int32_t>(2 * ne);
    n.S = cv.take<double>(nnz);
    n.dinv = cv.take<double>(nv);
    n.wall = cv.take<uint8_t>(nv);
    n.vec = cv.take<double>(8 * nv);
    n.partial = cv.take<double>(8 * kNsBlocks);
    n.sc = cv.take<double>(12);
    n.bzero = cv.take<double>(2 * nf);
    n.ezero = cv.take<double>(2 * ne);
    return n;
}

int ns_system(etpic_ctx *ctx, double eps) {
    if (ctx->ns_pending && ctx->ns_pending_eps == eps) return ETPIC_OK;
    std::string err;
    auto S = std::make_unique<etpic::NsSystem>();
    if (etpic::build_ns_system(ctx->host, eps, *S, err) != 0) return fail(ETPIC_EINVAL, "ns: %s", err.c_str());
    ctx->ns_pending = std::move(S);
    ctx->ns_pending_eps = eps;
    return ETPIC_OK;
}

}  // namespace

extern "C" {

int etpic_ns_bytes(etpic_ctx *ctx, double eps, size_t *bytes) {
    if (!ctx || !bytes) return fail(ETPIC_EINVAL, "null argument");
    if (!ctx->has_mesh) return fail(ETPIC_ESTATE, "no mesh uploaded");
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(ETPIC_EINVAL, "eps must be positive");
    if (int r = ns_system(ctx, eps)) return r;
    Carve cv;
    (void)ns_layout(cv, ctx->ns_pending->nv, ctx->host.ne, ctx->host.nf, ctx->ns_pending->nnz);
    *bytes = cv.used;
    return ETPIC_OK;
}

int etpic_ns_setup(etpic_ctx *ctx, double eps, void *dev_buf, size_t bytes) {
    if (!ctx) return fail(ETPIC_EINVAL, "null context");
    if (!ctx->has_mesh) return fail(ETPIC_ESTATE, "no mesh uploaded");
    if (!(eps > 0.0) || !std::isfinite(eps)) return fail(ETPIC_EINVAL, "eps must be positive");
    if (int r = ns_system(ctx, eps)) return r;
    const etpic::NsSystem &S = *ctx->ns_pending;
    const int64_t nv = S.nv, ne = ctx->host.ne, nf = ctx->host.nf;
    size_t need = 0;
    {
        Carve cv;
        (void)ns_layout(cv, nv, ne, nf, S.nnz);
        need = cv.used;
    }
    if (int r = check_buffer(dev_buf, bytes, need, "ns")) return r;
    std::vector<double> dinv((size_t)nv, 0.0);
    for (int64_t i = 0; i < nv; ++i) {
        double d = 0.0;
        for (int32_t j = S.rowptr[i]; j < S.rowptr[i + 1]; ++j)
            if (S.col[j] == i) d = S.S[j];
        if (!(d > 0.0)) return fail(ETPIC_EMESH, "ns: non-positive diagonal at node %lld", (long long)i);
        dinv[i] = 1.0 / d;
    }
    if (int r = set_device_only(ctx)) return r;
    HIP_TRY(hipDeviceSynchronize());
    NsState &N = ctx->ns;
    N.release();
    N.eps = eps;
    N.nv = nv;
    N.ne = ne;
    N.nnz = S.nnz;
    for (uint8_t b : S.wall) N.n_wall += b;
    Carve cv;
    cv.base = static_cast<char *>(dev_buf);
    cv.cap = bytes;
    const NsPtrs n = ns_layout(cv, nv, ne, nf, S.nnz);
    N.rowptr = n.rowptr;
    N.col = n.col;
    N.ev = n.ev;
    N.S = n.S;
    N.dinv = n.dinv;
    N.wall = n.wall;
    N.vec = n.vec;
    N.partial = n.partial;
    N.sc = n.sc;
    N.bzero = n.bzero;
    N.ezero = n.ezero;
    HIP_TRY(hipMemset(N.sc, 0, sizeof(double) * 12));
    HIP_TRY(hipMemset(N.vec, 0, sizeof(double) * 8 * nv));
    HIP_TRY(hipMemset(N.bzero, 0, sizeof(double) * 2 * nf));
    HIP_TRY(hipMemset(N.ezero, 0, sizeof(double) * 2 * ne));
    HIP_TRY(hipMemcpy(N.rowptr, S.rowptr.data(), sizeof(int32_t) * (nv + 1), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(N.col, S.col.data(), sizeof(int32_t) * S.nnz, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(N.ev, ctx->host.edges.data(), sizeof(int32_t) * 2 * ne, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(N.S, S.S.data(), sizeof(double) * S.nnz, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(N.dinv, dinv.data(), sizeof(double) * nv, hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(N.wall, S.wall.data(), sizeof(uint8_t) * nv, hipMemcpyHostToDevice));
    HIP_TRY(hipDeviceSynchronize());
    N.ready = true;
    ctx->ns_pending.reset();
    return ETPIC_OK;
}

int etpic_ns_info(const etpic_ctx *ctx, int64_t *nnz_out, int64_t *wall_nodes_out) {
    if (!ctx || !nnz_out) return fail(ETPIC_EINVAL, "null argument");
    if (!ctx->ns.ready) return fail(ETPIC_ESTATE, "etpic_ns_setup not called");
    *nnz_out = ctx->ns.nnz;
    if (wall_nodes_out) *wall_nodes_out = ctx->ns.n_wall;
    return ETPIC_OK;
}

}  // extern "C"

namespace {

// The CG of eq. ns_equation on `st` (synchronises it), from x = 0 or, warm,
// from the x of the previous solve; outputs scaled by e^{-j w t} = c - j s.
int ns_solve_impl(etpic_ctx *ctx, const NsRhs &R, double *x, double c, double s, double2 *x_out, double2 *e_out,
                  double *edc_out, const double *edc_add, double tol, int max_iter, bool warm, int *iters_out,
                  double *resid_out, hipStream_t st) {
    const NsState &N = ctx->ns;
    const int64_t nv = N.nv;
    const unsigned gv = (unsigned)std::min<int64_t>((nv + kNsVecThreads - 1) / kNsVecThreads, kNsBlocks);
    const unsigned gr = (unsigned)std::min<int64_t>((nv * kRowLanes + kNsThreads - 1) / kNsThreads, kNsBlocks);
    double *r = N.v(1), *z = N.v(2), *p = N.v(3), *q = N.v(4);
    // partials: pa from the product (gr blocks), pb from the start and the update
    double *pa = N.partial, *pb = N.partial + 4 * kNsBlocks;
    int64_t nb = warm ? gr : gv;
    if (warm)
        k_ns_start_warm<<<gr, kNsThreads, 0, st>>>(N.csr(), ctx->d_v2e_ptr, ctx->d_v2e_code, R, N.wall, N.dinv, x, r,
                                                   z, p, q, pb, N.sc);
    else
        k_ns_start<<<gv, kNsVecThreads, 0, st>>>(nv, ctx->d_v2e_ptr, ctx->d_v2e_code, R, N.wall, N.dinv, x, r, z, p, q,
                                                 pb, N.sc);
    HIP_TRY(hipGetLastError());
    // Iterations are launched in batches; the device raises the done flag when
    // the residual is small enough and the rest of the batch returns at once.
    // The host reads the scalars once per batch.
    const int batch = 10;
    const double tol2 = tol * tol;
    double hs[12];
    int k = 0;
    for (;;) {
        const int n = std::min(batch, max_iter - k);
        for (int j = 0; j < n; ++j, ++k) {
            k_ns_apply<<<gr, kNsThreads, 0, st>>>(N.csr(), N.sc, z, p, q, pb, nb, pa, k, tol2, 0);
            k_ns_update<<<gv, kNsVecThreads, 0, st>>>(nv, N.sc, N.dinv, p, q, x, r, z, pa, gr, pb, k);
            nb = gv;
        }
        if (k >= max_iter) k_ns_apply<<<gr, kNsThreads, 0, st>>>(N.csr(), N.sc, z, p, q, pb, nb, pa, k, tol2, 1);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipMemcpyAsync(hs, N.sc, sizeof hs, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        if (hs[10] != 0.0 || k >= max_iter) break;
    }
    const double bnorm2 = hs[9];
    if (!(bnorm2 > 0.0) && warm) HIP_TRY(hipMemsetAsync(x, 0, sizeof(double) * nv, st));   // no source: x = 0
    const double rel = bnorm2 > 0.0 ? std::sqrt(hs[8] / bnorm2) : 0.0;
    const int it = (int)hs[11];
    if (iters_out) *iters_out = it;
    if (resid_out) *resid_out = rel;
    if (hs[10] == 0.0 || !std::isfinite(rel))
        return fail(ETPIC_ENOCONV, "ns CG: relative residual %.3e after %d iterations", rel, it);
    if (x_out || e_out || edc_out)
        k_ns_out<<<grid_for(std::max(N.ne, nv)), kBlock, 0, st>>>(N.ne, nv, N.ev, x, c, s, x_out, e_out, edc_out,
                                                                  edc_add);
    HIP_TRY(hipGetLastError());
    return ETPIC_OK;
}

// The field step's source with its gradient part removed in the [*eps]
// inner product: gs = gdd - [*eps] D (D^T [*eps] D)^-1 D^T gdd, the inverse
// taken at the inner nodes (wall grounded).  On boundary edges D y = 0 and
// the field step's mass row is the identity, so gs = gdd there.  Work
// vectors: the field step's F.v(3), F.v(4); warm start from N.v(7).
int sol_source_impl(etpic_ctx *ctx, const double *gdd, double *gs, double tol, int max_iter, bool warm,
                    int *iters_out, double *resid_out, hipStream_t st) {
    const FieldState &F = ctx->field;
    double2 *dy = F.v(3), *m = F.v(4);
    if (int r = ns_solve_impl(ctx, NsRhs{gdd, nullptr, 1.0, nullptr, 0}, ctx->ns.v(7), 1.0, 0.0, nullptr, dy, nullptr,
                              nullptr, tol, max_iter, warm, iters_out, resid_out, st))
        return r;
    k_field_spmv<<<grid_for(F.ne * kRowLanes), kBlock, 0, st>>>(F.csr(), make_double2(1.0, 0.0), 0.0, dy, m);
    k_sol_add<<<grid_for(F.ne), kBlock, 0, st>>>(F.ne, gdd, m, gs);
    HIP_TRY(hipGetLastError());
    return ETPIC_OK;
}

// Both solvers set up on this context with the same eps.
int check_split_setup(const etpic_ctx *ctx) {
    if (!ctx->ns.ready) return fail(ETPIC_ESTATE, "etpic_ns_setup not called");
    if (!ctx->field.ready) return fail(ETPIC_ESTATE, "etpic_field_setup not called");
    if (std::fabs(ctx->field.eps - ctx->ns.eps) > 1e-15 * ctx->ns.eps)
        return fail(ETPIC_EINVAL, "etpic_field_setup and etpic_ns_setup were given different eps");
    return ETPIC_OK;
}

}  // namespace

extern "C" {

int etpic_ns_solve(etpic_ctx *ctx, const double *G, const double *rho0, double t, double omega, double *x_out,
                   double *e_out, double tol, int max_iter, uint32_t flags, int *iters_out, double *resid_out,
                   void *stream) {
    if (!ctx) return fail(ETPIC_EINVAL, "null context");
    if (!x_out && !e_out) return fail(ETPIC_EINVAL, "no output: x_out and e_out are both NULL");
    if (!ctx->ns.ready) return fail(ETPIC_ESTATE, "etpic_ns_setup not called");
    if (!(tol > 0.0) || max_iter < 1 || !std::isfinite(t) || !std::isfinite(omega))
        return fail(ETPIC_EINVAL, "bad tol / max_iter / time / omega");
    if (flags & ~(uint32_t)ETPIC_NS_WARM) return fail(ETPIC_EINVAL, "unknown flags 0x%x", flags);
    if (int r = set_device(ctx)) return r;
    return ns_solve_impl(ctx, NsRhs{G, rho0, 1.0, nullptr, 0}, ctx->ns.v(0), std::cos(omega * t),
                         std::sin(omega * t), reinterpret_cast<double2 *>(x_out), reinterpret_cast<double2 *>(e_out),
                         nullptr, nullptr, tol, max_iter, (flags & ETPIC_NS_WARM) != 0, iters_out, resid_out,
                         static_cast<hipStream_t>(stream));
}

int etpic_ns_run_steps(etpic_ctx *ctx, const etpic_particles *p, int precision, const etpic_species *sp,
                       const etpic_fields *ext, int64_t step0, int nsteps, int steps_per_solve, double dt,
                       double omega, double *G, const double *rho0, double *e_work, double tol, int max_iter,
                       uint32_t flags, int *iters_out, void *stream) {
    if (!ctx) return fail(ETPIC_EINVAL, "null context");
    if (!ctx->ns.ready) return fail(ETPIC_ESTATE, "etpic_ns_setup not called");
    if (!G || !e_work) return fail(ETPIC_EINVAL, "null G or e_work");
    if (ext && (!ext->e_env || !ext->b_env)) return fail(ETPIC_EINVAL, "external fields without e_env / b_env");
    if (ext && (ext->e_dc == e_work || ext->e_env == e_work || ext->b_env == e_work || ext->b_dc == e_work))
        return fail(ETPIC_EINVAL, "e_work aliases an external field array");
    if (G == e_work || (rho0 && rho0 == e_work)) return fail(ETPIC_EINVAL, "e_work aliases G or rho0");
    if (nsteps < 0 || steps_per_solve < 1) return fail(ETPIC_EINVAL, "bad step counts");
    if (!(tol > 0.0) || max_iter < 1) return fail(ETPIC_EINVAL, "bad tol / max_iter");
    const etpic_fields f{ext ? ext->e_env : ctx->ns.ezero, e_work, ext ? ext->b_env : ctx->ns.bzero,
                         ext ? ext->b_dc : nullptr};
    if (int r = check_step_args(ctx, sp, &f, dt, omega)) return r;
    if (int r = check_particles(ctx, p)) return r;
    if (int r = check_precision(precision, false)) return r;
    if (nsteps == 0) return ETPIC_OK;
    if (int r = set_device(ctx)) return r;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const uint32_t sf = flags & ~((uint32_t)ETPIC_NS_WARM | kFlagFixed);
    std::vector<StepPlan> plans((size_t)std::min(steps_per_solve, nsteps));
    int total = 0;
    for (int j = 0; j < nsteps; j += steps_per_solve) {
        const int n = std::min(steps_per_solve, nsteps - j);
        int it = 0;
        const bool warm = j > 0 || (flags & ETPIC_NS_WARM);
        if (int r = ns_solve_impl(ctx, NsRhs{G, rho0, 1.0, nullptr, 0}, ctx->ns.v(0), 1.0, 0.0, nullptr, nullptr,
                                  e_work, ext ? ext->e_dc : nullptr, tol, max_iter, warm, &it, nullptr, st)) {
            if (iters_out) *iters_out = total + it;
            return r;
        }
        total += it;
        if (p->n == 0) continue;
        for (int i = 0; i < n; ++i) plans[i] = StepPlan{{&f, nullptr, nullptr}, {1.0, 0.0, 0.0}, (double)(step0 + j + i) * dt};
        const int r = precision == ETPIC_FP64 ? ctx->run_steps<double>(p, sp, plans.data(), n, dt, omega, G, nullptr, sf, stream)
                                              : ctx->run_steps<float>(p, sp, plans.data(), n, dt, omega, G, nullptr, sf, stream);
        if (r) return r;
    }
    if (iters_out) *iters_out = total;
    return ETPIC_OK;
}

int etpic_ns_correct(etpic_ctx *ctx, const double *G, const double *rho0, double t, double omega, const double *u,
                     double *e_out, double tol, int max_iter, uint32_t flags, int *iters_out, double *resid_out,
                     void *stream) {
    if (!ctx || !u || !e_out) return fail(ETPIC_EINVAL, "null argument");
    if (int r = check_split_setup(ctx)) return r;
    if (!(tol > 0.0) || max_iter < 1 || !std::isfinite(t) || !std::isfinite(omega))
        return fail(ETPIC_EINVAL, "bad tol / max_iter / time / omega");
    if (flags & ~(uint32_t)ETPIC_NS_WARM) return fail(ETPIC_EINVAL, "unknown flags 0x%x", flags);
    if (int r = set_device(ctx)) return r;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const FieldState &F = ctx->field;
    NsState &N = ctx->ns;
    double2 *mu = F.v(3);   // [*eps] u (the field step's right-hand-side vector, free between steps)
    k_field_spmv<<<grid_for(F.ne * kRowLanes), kBlock, 0, st>>>(F.csr(), make_double2(1.0, 0.0), 0.0,
                                                                reinterpret_cast<const double2 *>(u), mu);
    HIP_TRY(hipGetLastError());
    const double c = std::cos(omega * t), s = std::sin(omega * t);
    const bool warm = (flags & ETPIC_NS_WARM) != 0;
    int it_re = 0, it_im = 0;
    double res_re = 0.0, res_im = 0.0;
    // e^{-j w t} (D^T G + rho0) = (c - j s)(D^T G + rho0): real and imaginary parts solved apart
    if (int r = ns_solve_impl(ctx, NsRhs{G, rho0, c, mu, 0}, N.v(5), 1.0, 0.0, nullptr, nullptr, nullptr, nullptr, tol,
                              max_iter, warm, &it_re, &res_re, st)) {
        if (iters_out) *iters_out = it_re;
        if (resid_out) *resid_out = res_re;
        return r;
    }
    if (int r = ns_solve_impl(ctx, NsRhs{G, rho0, -s, mu, 1}, N.v(6), 1.0, 0.0, nullptr, nullptr, nullptr, nullptr, tol,
                              max_iter, warm, &it_im, &res_im, st)) {
        if (iters_out) *iters_out = it_re + it_im;
        if (resid_out) *resid_out = res_im;
        return r;
    }
    if (iters_out) *iters_out = it_re + it_im;
    if (resid_out) *resid_out = std::max(res_re, res_im);
    k_ns_combine<<<grid_for(N.ne), kBlock, 0, st>>>(N.ne, N.ev, N.v(5), N.v(6), reinterpret_cast<const double2 *>(u),
                                                    reinterpret_cast<double2 *>(e_out));
    HIP_TRY(hipGetLastError());
    return ETPIC_OK;
}

int etpic_sol_source(etpic_ctx *ctx, const double *gdd, double *gs_out, double tol, int max_iter, uint32_t flags,
                     int *iters_out, double *resid_out, void *stream) {
    if (!ctx || !gdd || !gs_out) return fail(ETPIC_EINVAL, "null argument");
    if (int r = check_split_setup(ctx)) return r;
    if (!(tol > 0.0) || max_iter < 1) return fail(ETPIC_EINVAL, "bad tol / max_iter");
    if (flags & ~(uint32_t)ETPIC_NS_WARM) return fail(ETPIC_EINVAL, "unknown flags 0x%x", flags);
    if (int r = set_device(ctx)) return r;
    return sol_source_impl(ctx, gdd, gs_out, tol, max_iter, (flags & ETPIC_NS_WARM) != 0, iters_out, resid_out,
                           static_cast<hipStream_t>(stream));
}

int etpic_em_steps(etpic_ctx *ctx, const etpic_particles *p, int precision, const etpic_species *sp, int64_t step0,
                   int nsteps, double *u, double *v, double *a, double *b, double *e, double *G, double *G_hist,
                   const double *rho0, double tol, int max_iter, uint32_t flags, int *iters_out, void *stream) {
    if (!ctx || !u || !v || !a || !b || !e || !G || !G_hist) return fail(ETPIC_EINVAL, "null argument");
    if (int r = check_split_setup(ctx)) return r;
    if (nsteps < 0) return fail(ETPIC_EINVAL, "negative step count");
    if (e == u || G == G_hist || G_hist == u || G_hist == e) return fail(ETPIC_EINVAL, "aliased state arrays");
    if (!(tol > 0.0) || max_iter < 1) return fail(ETPIC_EINVAL, "bad tol / max_iter");
    const double dt = ctx->field.dt, omega = ctx->field.omega;
    const etpic_fields f{e, nullptr, b, nullptr};
    if (int r = check_step_args(ctx, sp, &f, dt, omega)) return r;
    if (int r = check_particles(ctx, p)) return r;
    if (int r = check_precision(precision, false)) return r;
    if (nsteps == 0) return ETPIC_OK;
    if (int r = set_device(ctx)) return r;
    hipStream_t st = static_cast<hipStream_t>(stream);
    const int64_t ne = ctx->field.ne;
    double *h1 = G_hist, *h2 = G_hist + ne;
    const uint32_t sf = flags & ~((uint32_t)(ETPIC_NS_WARM | ETPIC_EM_SPLIT) | kFlagFixed);
    const bool split = (flags & ETPIC_EM_SPLIT) != 0;
    int total = 0;
    for (int j = 0; j < nsteps; ++j) {
        const double t = (double)(step0 + j) * dt, t_next = (double)(step0 + j + 1) * dt;
        if (p->n > 0) {
            const StepPlan plan{{&f, nullptr, nullptr}, {1.0, 0.0, 0.0}, t};
            const int r = precision == ETPIC_FP64 ? ctx->run_steps<double>(p, sp, &plan, 1, dt, omega, G, nullptr, sf, stream)
                                                  : ctx->run_steps<float>(p, sp, &plan, 1, dt, omega, G, nullptr, sf, stream);
            if (r) return r;
        }
        k_em_gdd<<<grid_for(ne), kBlock, 0, st>>>(ne, G, h1, h2, h2, 1.0 / (dt * dt));
        HIP_TRY(hipGetLastError());
        const bool warm = j > 0 || (flags & ETPIC_NS_WARM);
        int it = 0;
        if (split) {   // the solenoidal system's source
            if (int r = sol_source_impl(ctx, h2, h2, tol, max_iter, warm, &it, nullptr, st)) {
                if (iters_out) *iters_out = total + it;
                return r;
            }
            total += it;
        }
        if (int r = etpic_field_step(ctx, t_next, u, v, a, b, h2, tol, max_iter, &it, nullptr, stream)) {
            if (iters_out) *iters_out = total + it;
            return r;
        }
        total += it;
        k_em_shift<<<grid_for(ne), kBlock, 0, st>>>(ne, G, h1, h2);
        HIP_TRY(hipGetLastError());
        if (split) {   // e = u + e^{-j w t} D y, y from eq. ns_equation
            if (int r = ns_solve_impl(ctx, NsRhs{G, rho0, 1.0, nullptr, 0}, ctx->ns.v(0), std::cos(omega * t_next),
                                      std::sin(omega * t_next), nullptr, reinterpret_cast<double2 *>(e), nullptr,
                                      nullptr, tol, max_iter, warm, &it, nullptr, st)) {
                if (iters_out) *iters_out = total + it;
                return r;
            }
            k_em_add<<<grid_for(ne), kBlock, 0, st>>>(ne, reinterpret_cast<const double2 *>(u),
                                                      reinterpret_cast<double2 *>(e));
            HIP_TRY(hipGetLastError());
        } else {
            const uint32_t cf = warm ? (uint32_t)ETPIC_NS_WARM : 0u;
            if (int r = etpic_ns_correct(ctx, G, rho0, t_next, omega, u, e, tol, max_iter, cf, &it, nullptr, stream)) {
                if (iters_out) *iters_out = total + it;
                return r;
            }
        }
        total += it;
    }
    if (iters_out) *iters_out = total;
    return ETPIC_OK;
}

int etpic_kernel_time(etpic_ctx *ctx, double ms_out[4], int64_t launches_out[2], int reset) {
    if (!ctx || !ms_out) return fail(ETPIC_EINVAL, "null argument");
    if (int r = set_device(ctx)) return r;
    double tot[4] = {0.0, 0.0, 0.0, 0.0};
    int64_t cnt[2] = {0, 0};
    for (const auto &t : ctx->timing) {
        const int sorting = t.sorting ? 1 : 0;
        // intervals: coefficient pass, particle kernel, walk, edge gather
        float m[4] = {0.f, 0.f, 0.f, 0.f};
        for (int k = 0; k < 4; ++k)
            if (t.has & (1u << k)) {
                HIP_TRY(hipEventSynchronize(t.ev[2 * k + 1]));
                HIP_TRY(hipEventElapsedTime(&m[k], t.ev[2 * k], t.ev[2 * k + 1]));
            }
        tot[sorting ? 3 : 0] += m[1];
        tot[1] += m[0];
        tot[2] += m[2] + m[3];
        if (t.has & 2u) ++cnt[sorting];
    }
    for (int k = 0; k < 4; ++k) ms_out[k] = tot[k];
    if (launches_out) {
        launches_out[0] = cnt[0];
        launches_out[1] = cnt[1];
    }
    if (reset) {
        for (auto &e : ctx->timing) ctx->spare.push_back(e);
        ctx->timing.clear();
    }
    return ETPIC_OK;
}

int etpic_last_push_slices(const etpic_ctx *ctx, int *slices) {
    if (!ctx || !slices) return fail(ETPIC_EINVAL, "null argument");
    *slices = ctx->last_slices;
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
