// The two leaf sweeps of one primal-dual iteration (single objects and
// batches), the gradient-descent update sweep, and the energy reduction.
//
// Dual sweep (gradient + ascent + unit-ball projection):
//   g_d = sum_{k in N+_d(n)} c_nk (ubar_k - ubar_n)   ascending key, fma chain
//   q   = p + sigma g,  p = q / max(1, |q|)
//   ds  = C+_x p_x + C+_y p_y + C+_z p_z              C+_d = sum_k c_nk
// Primal sweep (divergence + generalised shrinkage + extrapolation + flags):
//   div = ds - sum_d sum_{m in N-_d(n)} c'_mn p_{m,d}
//   u'  = u + tau div
//   u+  = median of {F_(1..M)} and {u' - t S_k}, t = tau lambda / (sum W + gamma),
//         S_k = 2 P_k - W_tot: the smallest k with u' - t S_k <= F_(k+1) selects
//         max(u' - t S_k, F_(k)) (the median of the 2M+1 values)
//   ubar = 2 u+ - u,  u = u+
//   flags: split if |u+| < tau_s below max depth, joinable if |u+| > tau_j.
// Every floating-point operation is a single IEEE operation in a fixed order,
// and every sum is one sequential chain: over a + or - list in list order (x,
// y, z neighbours, each in ascending key), however long the list; over a
// leaf's observations in (F, view) order.
#include <mutex>

#include "otf_internal.h"

namespace otf {
namespace {

constexpr int kBlk = 256;
constexpr int kAhead = 8;   // leaves whose observations one wave loads ahead in k_primal
constexpr int kGather = 4;  // neighbour entries per thread in flight in the short-list sweeps

#ifdef OTF_DEBUG_BOUNDS
// Bounds-checked build: every adjacency entry (list range, neighbour index,
// level code) and every observation index the sweeps read is checked. A
// violation sets a bit of this flag, which the host reads and clears after
// each solver call, and the read goes to index 0 instead (no fault).
static __device__ uint32_t bounds_flag;
__device__ inline uint32_t chk(uint32_t i, int64_t n, uint32_t bit) {
    if ((int64_t)i >= n) {
        atomicOr(&bounds_flag, bit);
        return 0u;
    }
    return i;
}
#define OTF_NB(v, L) chk((v) & kIdxMask, (L), 1u)
#define OTF_LV(v) chk((v) >> (kIdxBits + 2), kMaxDepth + 1, 2u)
#define OTF_OBS(e, n) chk((e), (n), 4u)
#define OTF_SEG(e0, e1, n)                                                 \
    do {                                                                   \
        if ((int64_t)(e1) > (n) || (e0) > (e1)) {                          \
            atomicOr(&bounds_flag, 8u);                                    \
            (e0) = (e1) = 0u;                                              \
        }                                                                  \
    } while (0)
#else
#define OTF_NB(v, L) ((v) & kIdxMask)
#define OTF_LV(v) ((v) >> (kIdxBits + 2))
#define OTF_OBS(e, n) (e)
#define OTF_SEG(e0, e1, n) ((void)0)
#endif

__device__ inline float rdlane(float v, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
}
__device__ inline int rdlane_i(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

struct DualArgs {
    int64_t L, cap;
    const uint8_t *level;
    const float *ubar;  // the field differenced: ubar (primal-dual) or u (gradient descent)
    const uint32_t *off;
    const uint32_t *ent;
    int64_t n_ent;  // entries of the list (bounds-checked build)
    float *p;
    float *ds;
    float sigma;
    int gd;      // 1: gradient-descent flux q = g / sqrt(|g|^2 + eps^2) instead of the dual step
    float eps2;
};

// q = p + sigma g, projection onto the unit ball, and the leaf's own part of
// the divergence from the updated p.
__device__ inline void dual_finish(const DualArgs &a, int64_t i, float gx, float gy, float gz, float Cx, float Cy,
                                   float Cz) {
    float qx, qy, qz;
    if (a.gd) {
        const float r2 = __fmaf_rn(gx, gx, __fmaf_rn(gy, gy, gz * gz));
        const float den = sqrtf(r2 + a.eps2);
        qx = gx / den;
        qy = gy / den;
        qz = gz / den;
        a.p[i] = qx;
        a.p[a.cap + i] = qy;
        a.p[2 * a.cap + i] = qz;
        a.ds[i] = __fmaf_rn(Cz, qz, __fmaf_rn(Cy, qy, __fmaf_rn(Cx, qx, 0.0f)));
        return;
    }
    qx = __fmaf_rn(a.sigma, gx, a.p[i]);
    qy = __fmaf_rn(a.sigma, gy, a.p[a.cap + i]);
    qz = __fmaf_rn(a.sigma, gz, a.p[2 * a.cap + i]);
    const float r2 = __fmaf_rn(qx, qx, __fmaf_rn(qy, qy, qz * qz));
    if (r2 > 1.0f) {
        const float nrm = sqrtf(r2);
        qx = qx / nrm;
        qy = qy / nrm;
        qz = qz / nrm;
    }
    a.p[i] = qx;
    a.p[a.cap + i] = qy;
    a.p[2 * a.cap + i] = qz;
    a.ds[i] = __fmaf_rn(Cz, qz, __fmaf_rn(Cy, qy, __fmaf_rn(Cx, qx, 0.0f)));
}

// Dual update of leaf i (one thread); a leaf with a long + list is left to
// dual_long_wave.
__device__ inline void dual_leaf(const DualArgs &a, const Coef &cf, int64_t i) {
    uint32_t e0 = a.off[i], e1 = a.off[i + 1];
    OTF_SEG(e0, e1, a.n_ent);
    if (e1 - e0 > kLongList) return;
    const int ln = a.level[i];
    const float ub = a.ubar[i];
    float gx = 0.0f, gy = 0.0f, gz = 0.0f, Cx = 0.0f, Cy = 0.0f, Cz = 0.0f;
    // kGather entries at a time: their loads are issued before the first is used
    for (uint32_t e = e0; e < e1; e += kGather) {
        uint32_t v[kGather];
        float ubk[kGather];
#pragma unroll
        for (int r = 0; r < kGather; ++r) v[r] = e + r < e1 ? a.ent[e + r] : 0u;
#pragma unroll
        for (int r = 0; r < kGather; ++r) ubk[r] = e + r < e1 ? a.ubar[OTF_NB(v[r], a.L)] : 0.0f;
#pragma unroll
        for (int r = 0; r < kGather; ++r) {
            if (e + r >= e1) break;
            const int d = (v[r] >> kIdxBits) & 3;
            const float c = cf.c[ln][OTF_LV(v[r])];
            const float diff = ubk[r] - ub;
            if (d == 0) {
                gx = __fmaf_rn(c, diff, gx);
                Cx = Cx + c;
            } else if (d == 1) {
                gy = __fmaf_rn(c, diff, gy);
                Cy = Cy + c;
            } else {
                gz = __fmaf_rn(c, diff, gz);
                Cz = Cz + c;
            }
        }
    }
    dual_finish(a, i, gx, gy, gz, Cx, Cy, Cz);
}

// The coefficient tables copied into LDS (a kernel argument indexed by the
// levels of a leaf and its neighbour would be fetched from memory, one
// dependent load per list entry).
__device__ inline const Coef &stage_coef(const Coef &cf, Coef &sh) {
    const float *src = &cf.c[0][0];
    float *dst = &sh.c[0][0];
    for (int k = threadIdx.x; k < (int)(sizeof(Coef) / sizeof(float)); k += blockDim.x) dst[k] = src[k];
    __syncthreads();
    return sh;
}

// Dual update of kDualLeaves leaves per thread, the same arithmetic as
// dual_leaf: every leaf-local load (list bounds, level, ubar, p) is issued
// first, then the list entries of all the thread's leaves, then their
// neighbours' ubar, so that one thread has its leaves' dependent loads in
// flight together (the sweep is bound by these chains, not by bandwidth).
constexpr int kDualLeaves = 2;

__device__ inline void dual_leaves(const DualArgs &a, const Coef &cf, const int64_t (&idx)[kDualLeaves]) {
    constexpr int N = kDualLeaves;
    // loads are unconditional (out-of-range leaves read leaf 0, entries past
    // a list's end read its first slot, which lies inside the allocation) so
    // that they issue back to back without branches
    uint32_t e0[N], e1[N];
    int ln[N];
    float ub[N], pv[N][3];
    bool on[N];
#pragma unroll
    for (int n = 0; n < N; ++n) {
        on[n] = idx[n] < a.L;
        const int64_t i = on[n] ? idx[n] : 0;
        e0[n] = a.off[i];
        e1[n] = a.off[i + 1];
        OTF_SEG(e0[n], e1[n], a.n_ent);
        ln[n] = a.level[i];
        ub[n] = a.ubar[i];
#pragma unroll
        for (int d = 0; d < 3; ++d) pv[n][d] = a.p[d * a.cap + i];
    }
    uint32_t len = 0;
#pragma unroll
    for (int n = 0; n < N; ++n) {
        on[n] = on[n] && e1[n] - e0[n] <= kLongList;  // long lists: dual_long_wave
        if (!on[n]) e1[n] = e0[n];
        len = max(len, e1[n] - e0[n]);
    }
    float g[N][3], C[N][3];
#pragma unroll
    for (int n = 0; n < N; ++n)
#pragma unroll
        for (int d = 0; d < 3; ++d) g[n][d] = C[n][d] = 0.0f;
    for (uint32_t k = 0; k < len; k += kGather) {
        uint32_t v[N][kGather];
        float ubk[N][kGather];
#pragma unroll
        for (int n = 0; n < N; ++n)
#pragma unroll
            for (int r = 0; r < kGather; ++r) {
                const uint32_t e = e0[n] + k + r;
                v[n][r] = a.ent[e < e1[n] ? e : e0[n]];
            }
#pragma unroll
        for (int n = 0; n < N; ++n)
#pragma unroll
            for (int r = 0; r < kGather; ++r)
                ubk[n][r] = a.ubar[e0[n] + k + r < e1[n] ? OTF_NB(v[n][r], a.L) : 0u];
        // entries folded in list order; selects rather than branches, so that
        // no load is deferred into a conditional block
#pragma unroll
        for (int n = 0; n < N; ++n)
#pragma unroll
            for (int r = 0; r < kGather; ++r) {
                const bool ok = e0[n] + k + r < e1[n];
                const int d = ok ? (int)((v[n][r] >> kIdxBits) & 3) : 3;
                const float c = cf.c[ln[n]][OTF_LV(v[n][r])];
                const float diff = ubk[n][r] - ub[n];
#pragma unroll
                for (int x = 0; x < 3; ++x) {
                    const float gn = __fmaf_rn(c, diff, g[n][x]), Cn = C[n][x] + c;
                    g[n][x] = d == x ? gn : g[n][x];
                    C[n][x] = d == x ? Cn : C[n][x];
                }
            }
    }
#pragma unroll
    for (int n = 0; n < N; ++n) {
        if (!on[n]) continue;
        const int64_t i = idx[n];
        if (a.gd) {
            dual_finish(a, i, g[n][0], g[n][1], g[n][2], C[n][0], C[n][1], C[n][2]);
            continue;
        }
        float qx = __fmaf_rn(a.sigma, g[n][0], pv[n][0]);
        float qy = __fmaf_rn(a.sigma, g[n][1], pv[n][1]);
        float qz = __fmaf_rn(a.sigma, g[n][2], pv[n][2]);
        const float r2 = __fmaf_rn(qx, qx, __fmaf_rn(qy, qy, qz * qz));
        if (r2 > 1.0f) {
            const float nrm = sqrtf(r2);
            qx = qx / nrm;
            qy = qy / nrm;
            qz = qz / nrm;
        }
        a.p[i] = qx;
        a.p[a.cap + i] = qy;
        a.p[2 * a.cap + i] = qz;
        a.ds[i] = __fmaf_rn(C[n][2], qz, __fmaf_rn(C[n][1], qy, __fmaf_rn(C[n][0], qx, 0.0f)));
    }
}


// Leaves whose + list is longer than kLongList, one wave each. The wave loads
// the list in windows of kWin entries (coalesced, kLongUnroll entries per
// lane), stages each window in LDS as (coefficient, operand) pairs in list
// order and folds it into the sequential chains: every lane runs the same
// chain on the same LDS words (broadcast reads), so the result is on every
// lane. The next window's entries and operands are loaded while the current
// one is folded. The list is sorted by direction, so the entries of one
// direction in a window form one run; ballots count them.
constexpr int kLongUnroll = 4;
constexpr int kWin = 64 * kLongUnroll;  // list entries staged per window
constexpr int kWavesPerBlock = kBlk / 64;
constexpr int kWinWords = 2 * kWin;     // one wave's LDS for a staged window

// LDS of one wave in k_gd_update: a staged window, or kAhead rows of 64
// observation terms (row pitch 65 words, so that lane g reading row g
// touches distinct banks).
constexpr int kTermPitch = 65;
constexpr int kStageWords = kAhead * kTermPitch;
static_assert(kStageWords >= kWinWords, "a staged window must fit the stage");

// LDS writes of a wave's lanes before reads by other lanes of the same wave.
__device__ inline void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// g = fma(c, x, g), C = C + c over the staged pairs [k0, k1), in order; the
// LDS reads of the next 8 pairs are issued before the current 8 are folded.
__device__ inline void fold_grad(const float2 *st, int k0, int k1, float &g, float &C) {
    int k = k0;
    if (k1 - k >= 8) {
        float2 e[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) e[r] = st[k + r];
        for (k += 8; k + 8 <= k1; k += 8) {
            float2 nx[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) nx[r] = st[k + r];
#pragma unroll
            for (int r = 0; r < 8; ++r) {
                g = __fmaf_rn(e[r].x, e[r].y, g);
                C = C + e[r].x;
            }
#pragma unroll
            for (int r = 0; r < 8; ++r) e[r] = nx[r];
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            g = __fmaf_rn(e[r].x, e[r].y, g);
            C = C + e[r].x;
        }
    }
    for (; k < k1; ++k) {
        const float2 e = st[k];
        g = __fmaf_rn(e.x, e.y, g);
        C = C + e.x;
    }
}

// acc = fma(c, x, acc) over the staged pairs [k0, k1), in order (pipelined
// as fold_grad).
__device__ inline float fold_chain(const float2 *st, int k0, int k1, float acc) {
    int k = k0;
    if (k1 - k >= 8) {
        float2 e[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) e[r] = st[k + r];
        for (k += 8; k + 8 <= k1; k += 8) {
            float2 nx[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) nx[r] = st[k + r];
#pragma unroll
            for (int r = 0; r < 8; ++r) acc = __fmaf_rn(e[r].x, e[r].y, acc);
#pragma unroll
            for (int r = 0; r < 8; ++r) e[r] = nx[r];
        }
#pragma unroll
        for (int r = 0; r < 8; ++r) acc = __fmaf_rn(e[r].x, e[r].y, acc);
    }
    for (; k < k1; ++k) {
        const float2 e = st[k];
        acc = __fmaf_rn(e.x, e.y, acc);
    }
    return acc;
}

// Positions [lo, hi) of a staged window whose direction runs are [0, n0),
// [n0, n01) and [n01, ...): each part folded into its direction's chains.
__device__ inline void fold_runs(const float2 *st, int n0, int n01, int lo, int hi, float (&g)[3], float (&C)[3]) {
    fold_grad(st, lo, min(hi, n0), g[0], C[0]);
    fold_grad(st, max(lo, n0), min(hi, n01), g[1], C[1]);
    fold_grad(st, max(lo, n01), hi, g[2], C[2]);
}

__device__ void dual_long_wave(const DualArgs &a, const Coef &cf, int64_t i, int lane, float *lds) {
    float2 *st = reinterpret_cast<float2 *>(lds);
    uint32_t e0 = a.off[i], e1 = a.off[i + 1];
    OTF_SEG(e0, e1, a.n_ent);
    const uint32_t ne = e1 - e0;
    const int ln = a.level[i];
    const float ub = a.ubar[i];
    float g[3] = {0.0f, 0.0f, 0.0f}, C[3] = {0.0f, 0.0f, 0.0f};
    uint32_t v[kLongUnroll];
    float u[kLongUnroll];
#pragma unroll
    for (int r = 0; r < kLongUnroll; ++r) {
        const uint32_t q = 64 * r + lane;
        v[r] = a.ent[e0 + (q < ne ? q : 0u)];
    }
#pragma unroll
    for (int r = 0; r < kLongUnroll; ++r) u[r] = a.ubar[64 * r + lane < ne ? OTF_NB(v[r], a.L) : 0u];
    for (uint32_t q0 = 0; q0 < ne; q0 += kWin) {
        // stage the window in list order; count its x and y entries
        int n0 = 0, n1 = 0;
#pragma unroll
        for (int r = 0; r < kLongUnroll; ++r) {
            const int d = q0 + 64 * r + lane < ne ? (int)((v[r] >> kIdxBits) & 3) : 3;
            n0 += (int)__popcll(__ballot(d == 0));
            n1 += (int)__popcll(__ballot(d == 1));
            st[64 * r + lane] = make_float2(cf.c[ln][OTF_LV(v[r])], u[r] - ub);
        }
        const int nw = (int)min((uint32_t)kWin, ne - q0);
        const uint32_t q1 = q0 + kWin;
        if (q1 < ne) {  // the next window's entries (uniform)
#pragma unroll
            for (int r = 0; r < kLongUnroll; ++r) {
                const uint32_t q = q1 + 64 * r + lane;
                v[r] = a.ent[e0 + (q < ne ? q : 0u)];
            }
        }
        wave_lds_sync();
        fold_runs(st, n0, n0 + n1, 0, nw / 2, g, C);
        if (q1 < ne) {  // and their neighbours' ubar
#pragma unroll
            for (int r = 0; r < kLongUnroll; ++r) u[r] = a.ubar[q1 + 64 * r + lane < ne ? OTF_NB(v[r], a.L) : 0u];
        }
        fold_runs(st, n0, n0 + n1, nw / 2, nw, g, C);
        wave_lds_sync();
    }
    if (lane == 0) dual_finish(a, i, g[0], g[1], g[2], C[0], C[1], C[2]);
}

// Dual sweep in one launch: the first long_blocks blocks take the leaves with
// a long + list (dual_long_wave, one wave each), the others kDualLeaves leaves
// per thread: such a block covers kDualLeaves * kBlk consecutive leaves,
// thread t takes t, t + kBlk, ... (each group coalesced; long-list leaves are
// skipped). The two kinds of blocks touch disjoint leaves.
__global__ void __launch_bounds__(kBlk) __attribute__((amdgpu_waves_per_eu(6, 8)))
k_dual(DualArgs a, Coef cf, uint32_t n_long, const uint32_t *long_list, uint32_t long_blocks) {
    __shared__ Coef scf;
    const Coef &lcf = stage_coef(cf, scf);
    if (blockIdx.x < long_blocks) {
        __shared__ float lds[kWavesPerBlock][kWinWords];
        const uint32_t item = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
        if (item < n_long) dual_long_wave(a, lcf, long_list[item], threadIdx.x & 63, lds[threadIdx.x >> 6]);
        return;
    }
    const int64_t base = (int64_t)(blockIdx.x - long_blocks) * (kDualLeaves * kBlk) + threadIdx.x;
    int64_t idx[kDualLeaves];
#pragma unroll
    for (int n = 0; n < kDualLeaves; ++n) idx[n] = base + (int64_t)n * kBlk;
    dual_leaves(a, lcf, idx);
}

struct PrimalArgs {
    int64_t L, cap;
    const uint8_t *level;
    float *ds;  // own divergence term; replaced by u' for leaves with a long - list
    const float *p;
    const uint32_t *off;
    const uint32_t *ent;
    int64_t n_ent, n_obs;  // entries of the list and of the observation pool (bounds-checked build)
    const uint32_t *obs_off;
    const uint8_t *obs_m, *obs_unit;
    const float *inv, *wtot;
    const float *F, *P;
    const float *u_in;
    float *u, *ubar;
    uint8_t *flag;
    float *uprime, *uold;
    uint32_t *part;  // per-block counts of split flags [0, stride) and join flags [stride, 2 stride)
    int64_t part_stride;
    float tau, tl, split_tau, join_tau;
    int join_enabled, max_depth;
    // gradient descent: divergence kept in ds for long lists, step xi, TV weight lam
    int gd;
    float lam, xi, eps2;
    const float *W;
};

// Divergence of a leaf with a long - list, one wave: ds, then the incoming
// terms fma(-c', p_m, acc) in list order, one chain over LDS-staged windows
// as in dual_long_wave (the same value on every lane).
__device__ float long_divergence(const PrimalArgs &a, const Coef &cf, int64_t i, int lane, float *lds) {
    float2 *st = reinterpret_cast<float2 *>(lds);
    uint32_t e0 = a.off[i], e1 = a.off[i + 1];
    OTF_SEG(e0, e1, a.n_ent);
    const uint32_t ne = e1 - e0;
    const int ln = a.level[i];
    float acc = a.ds[i];
    uint32_t v[kLongUnroll];
    float pm[kLongUnroll];
#pragma unroll
    for (int r = 0; r < kLongUnroll; ++r) {
        const uint32_t q = 64 * r + lane;
        v[r] = a.ent[e0 + (q < ne ? q : 0u)];
    }
#pragma unroll
    for (int r = 0; r < kLongUnroll; ++r)
        pm[r] = a.p[64 * r + lane < ne ? (int64_t)((v[r] >> kIdxBits) & 3) * a.cap + OTF_NB(v[r], a.L) : 0];
    for (uint32_t q0 = 0; q0 < ne; q0 += kWin) {
#pragma unroll
        for (int r = 0; r < kLongUnroll; ++r) st[64 * r + lane] = make_float2(-cf.cp[OTF_LV(v[r])][ln], pm[r]);
        const int nw = (int)min((uint32_t)kWin, ne - q0);
        const uint32_t q1 = q0 + kWin;
        if (q1 < ne) {  // the next window's entries (uniform)
#pragma unroll
            for (int r = 0; r < kLongUnroll; ++r) {
                const uint32_t q = q1 + 64 * r + lane;
                v[r] = a.ent[e0 + (q < ne ? q : 0u)];
            }
        }
        wave_lds_sync();
        acc = fold_chain(st, 0, nw / 2, acc);
        if (q1 < ne) {  // and their p
#pragma unroll
            for (int r = 0; r < kLongUnroll; ++r)
                pm[r] = a.p[q1 + 64 * r + lane < ne ? (int64_t)((v[r] >> kIdxBits) & 3) * a.cap + OTF_NB(v[r], a.L)
                                                   : 0];
        }
        acc = fold_chain(st, nw / 2, nw, acc);
        wave_lds_sync();
    }
    return acc;
}

// u' for leaves with a long - list, one wave each (the batched sweeps, where
// a separate launch precedes the tiles: long units inside the persistent
// blocks would hold their tiles at the block's barriers); u' replaces ds for
// primal_wave<true>.
__device__ void primal_long_wave(const PrimalArgs &a, const Coef &cf, int64_t i, int lane, float *lds) {
    const float acc = long_divergence(a, cf, i, lane, lds);
    if (lane == 0) a.ds[i] = __fmaf_rn(a.tau, acc, a.u_in[i]);
}

// Own divergence term ds minus the incoming terms of the short - list
// [e0, e1), in list order; kGather entries in flight.
__device__ inline float divergence(const PrimalArgs &a, const Coef &cf, uint32_t e0, uint32_t e1, int ln,
                                   float acc) {
    // unconditional loads (entries past the end read the list's first slot,
    // inside the allocation; their neighbour reads leaf 0) and selects, so
    // that every load of a group issues before the first is used
    for (uint32_t e = e0; e < e1; e += kGather) {
        uint32_t v[kGather];
        float pm[kGather];
#pragma unroll
        for (int r = 0; r < kGather; ++r) v[r] = a.ent[e + r < e1 ? e + r : e0];
#pragma unroll
        for (int r = 0; r < kGather; ++r)
            pm[r] = a.p[e + r < e1 ? (int64_t)((v[r] >> kIdxBits) & 3) * a.cap + OTF_NB(v[r], a.L) : 0];
#pragma unroll
        for (int r = 0; r < kGather; ++r) {
            const float nx = __fmaf_rn(-cf.cp[OTF_LV(v[r])][ln], pm[r], acc);
            acc = e + r < e1 ? nx : acc;
        }
    }
    return acc;
}

// The generalised shrinkage of one leaf by a whole wave: lane k holds
// breakpoint k (F_k and the prefix weight P_k; lanes at or past M hold values
// never used); upl, tl, wtl and Ml are the leaf's, the same on every lane.
// p_k = u' - t S_k is tested against F_(k+1), a ballot's popcount is the
// index k* of the sequential search (the predicate holds on a prefix), and
// the median is max(p_k*, F_k*) (u' - t W_tot past the last breakpoint; u'
// itself without observations). Returns it on every lane.
__device__ inline float wave_prox(float Fk, float Pk, float upl, float tl_, float wtl, int Ml, int lane) {
    // S_k = 2 P_k - W_tot for every leaf (with unit weights P_k = k and
    // W_tot = M exactly); lanes at or past Ml compute a value never used
    const float S = __fmaf_rn(2.0f, Pk, -wtl);
    const float pk = __fmaf_rn(-tl_, S, upl);
    const bool pred = lane < Ml && pk > Fk;
    const int ks = __popcll(__ballot(pred));
    const float pend = __fmaf_rn(-tl_, wtl, upl);
    const float pks = (ks < Ml) ? rdlane(pk, min(ks, 63)) : pend;
    const float Fp = rdlane(Fk, max(ks - 1, 0));
    float v = (ks > 0) ? ((pks >= Fp) ? pks : Fp) : pks;
    v = (Ml > 0) ? v : upl;
    return v + 0.0f;
}

// Split and join flags of a leaf at level ln with new value v.
__device__ inline void primal_flags(const PrimalArgs &a, float v, int ln, bool &split, bool &join) {
    const float av = fabsf(v);
    split = av < a.split_tau && ln < a.max_depth;
    join = a.join_enabled && av > a.join_tau;
}

// Outputs of leaf i: u = v, ubar = 2 v - u_old, the flag byte, and for a leaf
// flagged to split its u' and u_old.
__device__ inline void primal_store(const PrimalArgs &a, int64_t i, float v, float un, float up, bool split,
                                    bool join) {
    a.ubar[i] = __fmaf_rn(2.0f, v, -un);
    a.u[i] = v;
    a.flag[i] = split ? 1 : (join ? (v > 0.0f ? 2 : 4) : 0);
    if (split) {
        a.uprime[i] = up;
        a.uold[i] = un;
    }
}

// Divergence per thread, then the prox cooperatively: the wave takes its 64
// leaves one after another; lane k tests breakpoint k of the current leaf
// (p_k = u' - t S_k against F_(k+1), coalesced loads of F and P), a ballot
// counts the true predicates (a prefix: p_k falls, F rises), which is the
// index k* of the sequential search; max(p_k*, F_(k*)) is the median.
// The wave's 64 consecutive leaves (this lane: leaf i, valid if i < L; valid
// lanes form a prefix of the wave). A leaf with a long - list takes u' from
// ds (kLongInDs, after primal_long_wave) or is left to its own wave
// (primal_long_full in the same launch): then it stays in the wave's prox
// loop, with a value that is not stored. Returns the wave's split and join
// flag counts (the same on every lane).
// wave_prox for two leaves at once, one per half-wave (segment s: lanes
// 32 s .. 32 s + 31, lane sl of the segment holding breakpoint sl), for
// leaves of at most 32 observations: per half the same operations and values.
__device__ inline float half_prox(float Fk, float Pk, float upl, float tl_, float wtl, int Ml, int sl, int seg) {
    const float S = __fmaf_rn(2.0f, Pk, -wtl);
    const float pk = __fmaf_rn(-tl_, S, upl);
    const bool pred = sl < Ml && pk > Fk;
    const int ks = __popc((uint32_t)(__ballot(pred) >> (32 * seg)));
    const float pend = __fmaf_rn(-tl_, wtl, upl);
    const float pkk = __shfl(pk, 32 * seg + min(ks, 31), 64);
    const float Fp = __shfl(Fk, 32 * seg + max(ks - 1, 0), 64);
    const float pks = (ks < Ml) ? pkk : pend;
    float v = (ks > 0) ? ((pks >= Fp) ? pks : Fp) : pks;
    v = (Ml > 0) ? v : upl;
    return v + 0.0f;
}

template <bool kLongInDs>
__device__ inline void primal_wave(const PrimalArgs &a, const Coef &cf, int64_t i, uint32_t &n_split,
                                   uint32_t &n_join) {
    const int lane = threadIdx.x & 63;
    const bool valid = i < a.L;
    bool own = valid;
    float up = 0.0f, un = 0.0f, t = 0.0f, wt = 0.0f;
    int M = 0, ln = 0;
    uint32_t oo = 0;
    if (valid) {
        // the leaf's own loads first, all in flight before the divergence's
        // dependent list loads
        ln = a.level[i];
        un = a.u_in[i];
        uint32_t e0 = a.off[i], e1 = a.off[i + 1];
        OTF_SEG(e0, e1, a.n_ent);
        const float dsi = a.ds[i];
        M = a.obs_m[i];
        oo = a.obs_off[i];
        const float inv = a.inv[i];
        wt = a.wtot[i];
        t = a.tl * inv;
        if (e1 - e0 > kLongList) {
            up = kLongInDs ? dsi : un;
            own = kLongInDs;
        } else {
            up = __fmaf_rn(a.tau, divergence(a, cf, e0, e1, ln, dsi), un);
        }
    }
    // valid lanes form a prefix of the wave; the F and P loads of kAhead
    // leaves are issued before the first of them is used, to keep enough
    // bytes in flight per wave.
    const int nact = __popcll(__ballot(valid));
    float myv = 0.0f;
    int mx = valid ? M : 0;  // the wave's largest observation count
    for (int o = 32; o > 0; o >>= 1) mx = max(mx, __shfl_xor(mx, o, 64));
    if (mx <= 32) {
        // two leaves per step, one per half-wave: leaves l0 + 2 g (lanes
        // 0-31) and l0 + 2 g + 1 (lanes 32-63)
        const int seg = lane >> 5, sl = lane & 31;
        constexpr int kSteps = kAhead / 2;  // kAhead leaves in flight, as below
        for (int l0 = 0; l0 < nact; l0 += 2 * kSteps) {
            float Fr[kSteps], Pr[kSteps];
            int Mg[kSteps];
#pragma unroll
            for (int g = 0; g < kSteps; ++g) {
                const int l = min(l0 + 2 * g + seg, 63);
                Mg[g] = __shfl(M, l, 64);
                const uint32_t ool = (uint32_t)__shfl((int)oo, l, 64);
                const uint32_t e = OTF_OBS(ool + (sl < Mg[g] ? (uint32_t)sl : 0u), a.n_obs);
                Fr[g] = a.F[e];
                Pr[g] = a.P[e];
            }
#pragma unroll
            for (int g = 0; g < kSteps; ++g) {
                const int lc = min(l0 + 2 * g + seg, 63);
                const float upl = __shfl(up, lc, 64), tl_ = __shfl(t, lc, 64), wtl = __shfl(wt, lc, 64);
                const float v = half_prox(Fr[g], Pr[g], upl, tl_, wtl, Mg[g], sl, seg);
                const float v0 = rdlane(v, 0), v1 = rdlane(v, 32);
                const int la = l0 + 2 * g;
                myv = (lane == la && la < nact) ? v0 : myv;
                myv = (lane == la + 1 && la + 1 < nact) ? v1 : myv;
            }
        }
    }
    for (int l0 = 0; mx > 32 && l0 < nact; l0 += kAhead) {
        float Fr[kAhead], Pr[kAhead];
        // unconditional loads (lanes past a segment's end, and leaves past
        // the wave's last, read its first entry, inside the pool's
        // allocation), so that leaf g's compute waits only for its own loads
#pragma unroll
        for (int g = 0; g < kAhead; ++g) {
            const int l = min(l0 + g, 63);
            const int Ml = rdlane_i(M, l);
            const uint32_t ool = (uint32_t)rdlane_i((int)oo, l);
            const uint32_t e = OTF_OBS(ool + (lane < Ml ? (uint32_t)lane : 0u), a.n_obs);
            Fr[g] = a.F[e];
            Pr[g] = a.P[e];
        }
        // every leaf of the group computed without branches (a leaf past the
        // wave's last reads lane 63 and is dropped), so that no load is
        // deferred into a conditional block
#pragma unroll
        for (int g = 0; g < kAhead; ++g) {
            const int l = l0 + g;
            const int lc = min(l, 63);
            const int Ml = rdlane_i(M, lc);
            const float upl = rdlane(up, lc), tl_ = rdlane(t, lc), wtl = rdlane(wt, lc);
            const float v = wave_prox(Fr[g], Pr[g], upl, tl_, wtl, Ml, lane);
            myv = (lane == l && l < nact) ? v : myv;
        }
    }
    bool split = false, join = false;
    if (own) {
        primal_flags(a, myv, ln, split, join);
        primal_store(a, i, myv, un, up, split, join);
    }
    n_split = (uint32_t)__popcll(__ballot(split));
    n_join = (uint32_t)__popcll(__ballot(join));
}

// Per-block flag counts: part[blk] (split) and part[stride + blk] (join).
template <int BLK>
__device__ inline void block_flag_counts(uint32_t n_split, uint32_t n_join, uint32_t *part, int64_t stride,
                                         int64_t blk) {
    __shared__ uint32_t cnt[2][BLK / 64];
    if ((threadIdx.x & 63) == 0) {
        cnt[0][threadIdx.x >> 6] = n_split;
        cnt[1][threadIdx.x >> 6] = n_join;
    }
    __syncthreads();
    if (threadIdx.x < 2) {
        uint32_t t = 0;
        for (int w = 0; w < BLK / 64; ++w) t += cnt[threadIdx.x][w];
        part[threadIdx.x * stride + blk] = t;
    }
    __syncthreads();
}

// The whole primal update of a leaf with a long - list, one wave: its own
// loads, u' = u + tau div (long_divergence), the prox of its observations
// (lane k: breakpoint k) and its outputs. The flags are returned on every lane.
__device__ void primal_long_full(const PrimalArgs &a, const Coef &cf, int64_t i, int lane, float *lds, bool &split,
                                 bool &join) {
    const int ln = a.level[i];
    const float un = a.u_in[i];
    const int M = a.obs_m[i];
    const uint32_t oo = a.obs_off[i];
    const float inv = a.inv[i], wt = a.wtot[i];
    const uint32_t e = OTF_OBS(oo + (lane < M ? (uint32_t)lane : 0u), a.n_obs);
    const float Fk = a.F[e], Pk = a.P[e];
    const float up = __fmaf_rn(a.tau, long_divergence(a, cf, i, lane, lds), un);
    const float v = wave_prox(Fk, Pk, up, a.tl * inv, wt, M, lane);
    primal_flags(a, v, ln, split, join);
    if (lane == 0) primal_store(a, i, v, un, up, split, join);
}

// Primal sweep in one launch: the first long_blocks blocks take the leaves
// with a long - list (primal_long_full, one wave each), the others 64
// consecutive leaves per wave (primal_wave, long-list leaves not stored).
// The two kinds of blocks write disjoint leaves; per-block flag counts go to
// part[block] and part[stride + block].
__global__ void __launch_bounds__(kBlk) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_primal(PrimalArgs a, Coef cf, uint32_t n_long, const uint32_t *long_list, uint32_t long_blocks) {
    __shared__ Coef scf;
    const Coef &lcf = stage_coef(cf, scf);
    uint32_t ns = 0, nj = 0;
    if (blockIdx.x < long_blocks) {
        __shared__ float lds[kWavesPerBlock][kWinWords];
        const uint32_t item = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
        if (item < n_long) {
            bool split, join;
            primal_long_full(a, lcf, long_list[item], threadIdx.x & 63, lds[threadIdx.x >> 6], split, join);
            ns = split ? 1u : 0u;
            nj = join ? 1u : 0u;
        }
    } else {
        primal_wave<false>(a, lcf, (int64_t)(blockIdx.x - long_blocks) * kBlk + threadIdx.x, ns, nj);
    }
    block_flag_counts<kBlk>(ns, nj, a.part, a.part_stride, blockIdx.x);
}

// Gradient descent (the paper's solver). Divergence per thread, then the
// data gradient cooperatively as in k_primal: the wave takes its 64 leaves in
// groups of kAhead, lane k loads observation k of each leaf (coalesced) and
// forms
//   t_k = W_k (r_k / sqrt(r_k^2 + eps^2)),  r_k = u - F_k  (0 for k >= M);
// the group's terms go to LDS, one row per leaf, and lane g adds row g in
// one sequential chain in observation order (the zero terms past M leave the
// sum unchanged: a chain started at +0 never holds -0). Then
//   u <- u + xi (lam div - d'),  d' = sum * inv.
// The divergence is kept (uprime) so that split children take the same step
// with their own data term.

// Data-gradient term of observation k on lane k (0 at or past M).
__device__ inline float gd_term(float u, float Fk, float Wk, float eps2, int Ml, int lane) {
    const float r = u - Fk;
    const float den = sqrtf(__fmaf_rn(r, r, eps2));  // > 0: eps > 0
    return lane < Ml ? Wk * (r / den) : 0.0f;
}

// Sequential sum of the n terms of LDS row `row` (every lane may call it; a
// lane reads its own row).
__device__ inline float row_sum(const float *lds, int row, int n) {
    const float *r = lds + row * kTermPitch;
    float acc = 0.0f;
    for (int k = 0; k < n; ++k) acc = acc + r[k];
    return acc;
}

// Update, flags and stores of a leaf from its divergence dv and data-gradient
// sum.
__device__ inline void gd_store(const PrimalArgs &a, int64_t i, float un, float dv, float sum, float inv, int ln,
                                bool &split, bool &join) {
    const float dg = sum * inv;
    const float v = __fmaf_rn(a.xi, __fmaf_rn(a.lam, dv, -dg), un);
    a.u[i] = v;
    a.ubar[i] = v;
    const float av = fabsf(v);
    split = av < a.split_tau && ln < a.max_depth;
    join = a.join_enabled && av > a.join_tau;
    a.flag[i] = split ? 1 : (join ? (v > 0.0f ? 2 : 4) : 0);
    if (split) {
        a.uprime[i] = dv;
        a.uold[i] = un;
    }
}

// The wave's 64 consecutive leaves, as primal_wave; a leaf with a long -
// list is left to its own wave in the same launch (kept in the loop, not
// stored).
__device__ inline void gd_wave(const PrimalArgs &a, const Coef &cf, int64_t i, float *lds, uint32_t &n_split,
                               uint32_t &n_join) {
    const int lane = threadIdx.x & 63;
    const bool valid = i < a.L;
    bool own = valid;
    float dv = 0.0f, un = 0.0f, inv = 0.0f;
    int M = 0, ln = 0;
    uint32_t oo = 0;
    if (valid) {
        // the leaf's own loads first, then the divergence's dependent ones
        ln = a.level[i];
        un = a.u_in[i];
        uint32_t e0 = a.off[i], e1 = a.off[i + 1];
        OTF_SEG(e0, e1, a.n_ent);
        const float dsi = a.ds[i];
        M = a.obs_m[i];
        oo = a.obs_off[i];
        inv = a.inv[i];
        if (e1 - e0 > kLongList) own = false;
        else dv = divergence(a, cf, e0, e1, ln, dsi);
    }
    const int nact = __popcll(__ballot(valid));
    float mysum = 0.0f;
    for (int l0 = 0; l0 < nact; l0 += kAhead) {
        float Fr[kAhead], Wr[kAhead];
        // unconditional loads and branch-free terms, as in primal_wave
#pragma unroll
        for (int g = 0; g < kAhead; ++g) {
            const int l = min(l0 + g, 63);
            const int Ml = rdlane_i(M, l);
            const uint32_t ool = (uint32_t)rdlane_i((int)oo, l);
            const uint32_t e = OTF_OBS(ool + (lane < Ml ? (uint32_t)lane : 0u), a.n_obs);
            Fr[g] = a.F[e];
            Wr[g] = a.W[e];
        }
        int nmax = 0;
#pragma unroll
        for (int g = 0; g < kAhead; ++g) {
            const int lc = min(l0 + g, 63);
            const int Ml = rdlane_i(M, lc);
            nmax = max(nmax, Ml);
            lds[g * kTermPitch + lane] = gd_term(rdlane(un, lc), Fr[g], Wr[g], a.eps2, Ml, lane);
        }
        wave_lds_sync();
        // lane g < kAhead sums leaf l0 + g; the sums reach their leaves' lanes
        const float sg = row_sum(lds, lane & (kAhead - 1), nmax);
        const float mine = __shfl(sg, (lane - l0) & (kAhead - 1), 64);
        mysum = (lane >= l0 && lane < l0 + kAhead) ? mine : mysum;
        wave_lds_sync();
    }
    bool split = false, join = false;
    if (own) gd_store(a, i, un, dv, mysum, inv, ln, split, join);
    n_split = (uint32_t)__popcll(__ballot(split));
    n_join = (uint32_t)__popcll(__ballot(join));
}

// The whole update of a leaf with a long - list, one wave: its divergence
// (long_divergence), the data gradient with lane k on observation k summed
// in one chain from LDS, and its stores. The flags are returned on every
// lane.
__device__ void gd_long_full(const PrimalArgs &a, const Coef &cf, int64_t i, int lane, float *lds, bool &split,
                             bool &join) {
    const int ln = a.level[i];
    const float un = a.u_in[i];
    const int M = a.obs_m[i];
    const uint32_t oo = a.obs_off[i];
    const float inv = a.inv[i];
    const uint32_t e = OTF_OBS(oo + (lane < M ? (uint32_t)lane : 0u), a.n_obs);
    const float Fk = a.F[e], Wk = a.W[e];
    const float dv = long_divergence(a, cf, i, lane, lds);
    lds[lane] = gd_term(un, Fk, Wk, a.eps2, M, lane);
    wave_lds_sync();
    const float sum = row_sum(lds, 0, M);
    wave_lds_sync();
    // the stores on lane 0, the flags (from the same values) on every lane
    const float v = __fmaf_rn(a.xi, __fmaf_rn(a.lam, dv, -(sum * inv)), un);
    const float av = fabsf(v);
    split = av < a.split_tau && ln < a.max_depth;
    join = a.join_enabled && av > a.join_tau;
    if (lane == 0) {
        bool s_, j_;
        gd_store(a, i, un, dv, sum, inv, ln, s_, j_);
    }
}

// Gradient-descent update in one launch: the first long_blocks blocks take
// the leaves with a long - list (gd_long_full, a wave each), the others 64
// consecutive leaves per wave (gd_wave); per-block flag counts as k_primal.
__global__ void __launch_bounds__(kBlk) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_gd_update(PrimalArgs a, Coef cf_arg, uint32_t n_long, const uint32_t *long_list, uint32_t long_blocks) {
    __shared__ Coef scf;
    __shared__ float lds[kWavesPerBlock][kStageWords];
    const Coef &cf = stage_coef(cf_arg, scf);
    float *wl = lds[threadIdx.x >> 6];
    uint32_t ns = 0, nj = 0;
    if (blockIdx.x < long_blocks) {
        const uint32_t item = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
        if (item < n_long) {
            bool split, join;
            gd_long_full(a, cf, long_list[item], threadIdx.x & 63, wl, split, join);
            ns = split ? 1u : 0u;
            nj = join ? 1u : 0u;
        }
    } else {
        gd_wave(a, cf, (int64_t)(blockIdx.x - long_blocks) * kBlk + threadIdx.x, wl, ns, nj);
    }
    block_flag_counts<kBlk>(ns, nj, a.part, a.part_stride, blockIdx.x);
}

// Energy: per-leaf terms in double, block partial sums in a fixed tree order.
// With eps2 > 0 the terms are the smoothed ones of the gradient-descent
// energy: sqrt(|Gu|^2 + eps^2) and sqrt((u - F)^2 + eps^2). The TV term per
// thread; the data term cooperatively, as the primal sweep reads the
// observations: the wave takes its 64 leaves in groups of kAhead, lane k
// loads observation k of each (coalesced, all of a group in flight), and a
// leaf's terms are added by a butterfly over the 64 lanes.
__global__ void __launch_bounds__(kBlk) k_energy(int64_t L, int D, const uint8_t *level, const float *u,
                                                 const uint32_t *off, const uint32_t *ent, const uint32_t *obs_off,
                                                 const uint8_t *obs_m, const float *inv, const float *F,
                                                 const float *W, Coef cf, double eps2, double *partial) {
    __shared__ double s_tv[kBlk], s_da[kBlk];
    const int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool valid = i < L;
    double tv = 0.0, vol = 0.0;
    float uf = 0.0f;
    int M = 0;
    uint32_t o = 0;
    if (valid) {
        const int ln = level[i];
        uf = u[i];
        M = obs_m[i];
        o = obs_off[i];
        const double un = uf;
        double g[3] = {0.0, 0.0, 0.0};
        for (uint32_t e = off[i]; e < off[i + 1]; ++e) {
            const uint32_t v = ent[e];
            const int d = (v >> kIdxBits) & 3;
            const int lk = v >> (kIdxBits + 2);
            const double c = cf.c[ln][lk];
            const double dif = (double)u[v & kIdxMask] - un;
            if (d == 0) g[0] += c * dif;
            else if (d == 1) g[1] += c * dif;
            else g[2] += c * dif;
        }
        const double s = ldexp(1.0, D - ln);
        vol = s * s * s;
        const double g2 = g[0] * g[0] + g[1] * g[1] + g[2] * g[2];
        tv = vol * (eps2 > 0.0 ? sqrt(g2 + eps2) : sqrt(g2));
    }
    const int nact = __popcll(__ballot(valid));
    double mine = 0.0;
    for (int l0 = 0; l0 < nact; l0 += kAhead) {
        float Fr[kAhead], Wr[kAhead];
#pragma unroll
        for (int g = 0; g < kAhead; ++g) {
            const int l = min(l0 + g, 63);
            const int Ml = rdlane_i(M, l);
            const uint32_t e = (uint32_t)rdlane_i((int)o, l) + (lane < Ml ? (uint32_t)lane : 0u);
            Fr[g] = F[e];
            Wr[g] = W[e];
        }
#pragma unroll
        for (int g = 0; g < kAhead; ++g) {
            const int l = l0 + g;
            const int lc = min(l, 63);
            const int Ml = rdlane_i(M, lc);
            const double r = (double)rdlane(uf, lc) - (double)Fr[g];
            double t = lane < Ml ? (double)Wr[g] * (eps2 > 0.0 ? sqrt(r * r + eps2) : fabs(r)) : 0.0;
#pragma unroll
            for (int sh = 1; sh < 64; sh <<= 1) t = t + __shfl_xor(t, sh, 64);
            mine = (lane == l && l < nact) ? t : mine;
        }
    }
    const double da = valid ? vol * (double)inv[i] * mine : 0.0;
    s_tv[threadIdx.x] = tv;
    s_da[threadIdx.x] = da;
    __syncthreads();
    for (int st = kBlk / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            s_tv[threadIdx.x] += s_tv[threadIdx.x + st];
            s_da[threadIdx.x] += s_da[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = s_tv[0];
        partial[2 * blockIdx.x + 1] = s_da[0];
    }
}

// ---------------------------------------------------------------- batches
// Many octrees swept by the same launches. Each object keeps its own store;
// a device table holds its sweep arguments. Tiles of BLK leaves never
// straddle two objects: tile t belongs to the object j with
// tile_begin[j] <= t < tile_begin[j+1] and covers its leaves from
// (t - tile_begin[j]) * BLK. Blocks stride over the tiles.
struct ObjDev {
    DualArgs d;
    PrimalArgs p;
    const uint32_t *heavy_p, *heavy_m;
    uint32_t *counters;
    int D;  // max depth: index of the coefficient table
};

// largest j < nobj with begin[j] <= t (begin[0] = 0)
__device__ inline int find_obj(const uint32_t *begin, int nobj, uint32_t t) {
    int lo = 0, hi = nobj;
    while (hi - lo > 1) {
        const int m = (lo + hi) >> 1;
        if (begin[m] <= t) lo = m;
        else hi = m;
    }
    return lo;
}

// tile_obj[t] is the member of tile t (one load instead of a binary search
// over the members' tile prefix at every tile's start). The dual runs BLK / 2
// threads per tile of BLK leaves, two leaves per thread as in k_dual.
template <int BLK>
__global__ void __launch_bounds__(BLK / 2) k_dual_b(const ObjDev *objs, const uint32_t *tile_obj,
                                                    const uint32_t *tile_begin, uint32_t ntiles, const Coef *coefs) {
    static_assert(kDualLeaves == 2, "two leaves per thread");
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int j = (int)tile_obj[t];
        const DualArgs a = objs[j].d;
        const int64_t base = (int64_t)(t - tile_begin[j]) * BLK + threadIdx.x;
        const int64_t idx[kDualLeaves] = {base, base + BLK / 2};
        dual_leaves(a, coefs[objs[j].D], idx);
    }
}

template <int BLK>
__global__ void __launch_bounds__(BLK) k_primal_b(const ObjDev *objs, const uint32_t *tile_obj,
                                                  const uint32_t *tile_begin, uint32_t ntiles, const Coef *coefs,
                                                  uint32_t *part) {
    for (uint32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const int j = (int)tile_obj[t];
        const PrimalArgs a = objs[j].p;
        uint32_t ns, nj;
        primal_wave<true>(a, coefs[objs[j].D], (int64_t)(t - tile_begin[j]) * BLK + threadIdx.x, ns, nj);
        block_flag_counts<BLK>(ns, nj, part, ntiles, t);
    }
}

// Long lists of all objects, one wave per item: item t < n is item
// t - begin[j] of object j's list.
__global__ void __launch_bounds__(kBlk) k_dual_long_b(const ObjDev *objs, int nobj, const uint32_t *begin,
                                                      uint32_t n, const Coef *coefs) {
    const uint32_t t = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (t >= n) return;
    const int j = find_obj(begin, nobj, t);
    __shared__ float lds[kWavesPerBlock][kWinWords];
    dual_long_wave(objs[j].d, coefs[objs[j].D], objs[j].heavy_p[t - begin[j]], threadIdx.x & 63,
                   lds[threadIdx.x >> 6]);
}

__global__ void __launch_bounds__(kBlk) k_primal_long_b(const ObjDev *objs, int nobj, const uint32_t *begin,
                                                        uint32_t n, const Coef *coefs) {
    const uint32_t t = blockIdx.x * kWavesPerBlock + (threadIdx.x >> 6);
    if (t >= n) return;
    const int j = find_obj(begin, nobj, t);
    __shared__ float lds[kWavesPerBlock][kWinWords];
    primal_long_wave(objs[j].p, coefs[objs[j].D], objs[j].heavy_m[t - begin[j]], threadIdx.x & 63,
                     lds[threadIdx.x >> 6]);
}

// Object j's split and join flag counts from its tiles' partials (block j),
// then the observation totals accumulated as by one iteration of a single
// context.
__global__ void __launch_bounds__(kBlk) k_batch_counts(const ObjDev *objs, const uint32_t *tile_begin,
                                                       uint32_t ntiles, const uint32_t *part) {
    __shared__ uint32_t red[2][kBlk / 64];
    const int j = blockIdx.x;
    const uint32_t t0 = tile_begin[j], t1 = tile_begin[j + 1];
    uint32_t s0 = 0, s1 = 0;
    for (uint32_t t = t0 + threadIdx.x; t < t1; t += kBlk) {
        s0 += part[t];
        s1 += part[ntiles + t];
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        s0 += (uint32_t)__shfl_xor((int)s0, off, 64);
        s1 += (uint32_t)__shfl_xor((int)s1, off, 64);
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = s0;
        red[1][threadIdx.x >> 6] = s1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t a = 0, b = 0;
        for (int w = 0; w < kBlk / 64; ++w) {
            a += red[0][w];
            b += red[1][w];
        }
        uint32_t *c = objs[j].counters;
        c[0] = a;
        c[1] = b;
        unsigned long long *o = reinterpret_cast<unsigned long long *>(c + 4);  // [16..17] += [4..5] + [6..7]
        o[6] += o[0] + o[1];
    }
}

DualArgs dual_args(Ctx &c, float sigma) {
    LeafStore &s = c.lv();
    return DualArgs{c.L, s.cap, s.level.p, s.ubar.p, s.nbp_off.p, s.nbp.p, s.n_nbp, s.p.p, s.ds.p, sigma, 0, 0.0f};
}

PrimalArgs primal_args(Ctx &c, float tau, float tl) {
    LeafStore &s = c.lv();
    PrimalArgs a;
    a.L = c.L;
    a.cap = s.cap;
    a.level = s.level.p;
    a.ds = s.ds.p;
    a.p = s.p.p;
    a.off = s.nbm_off.p;
    a.ent = s.nbm.p;
    a.n_ent = s.n_nbm;
    a.n_obs = (int64_t)c.op().F.n;  // the allocation: a leaf without observations reads its slot
    a.obs_off = s.obs_off.p;
    a.obs_m = s.obs_m.p;
    a.obs_unit = s.obs_unit.p;
    a.inv = s.inv.p;
    a.wtot = s.wtot.p;
    a.F = c.op().F.p;
    a.P = c.op().P.p;
    a.u_in = s.u.p;
    a.u = s.u.p;
    a.ubar = s.ubar.p;
    a.flag = s.flag.p;
    a.uprime = s.uprime.p;
    a.uold = s.uold.p;
    a.part = nullptr;
    a.part_stride = 0;
    a.tau = tau;
    a.tl = tl;
    a.split_tau = c.prm.split_tau;
    a.join_tau = c.prm.join_tau;
    a.join_enabled = !(c.prm.join_tau > 1.0f);
    a.max_depth = c.prm.max_depth;
    a.gd = 0;
    a.lam = a.xi = a.eps2 = 0.0f;
    a.W = c.op().W.p;
    return a;
}

template <int BLK>
void launch_batch(hipStream_t st, BatchState &b) {
    const ObjDev *objs = reinterpret_cast<const ObjDev *>(b.table.p);
    const int nobj = (int)b.objs.size();
    const unsigned grid = (unsigned)(b.cfg.grid > 0 ? std::min<uint32_t>(b.cfg.grid, b.ntiles) : b.ntiles);
    hipLaunchKernelGGL(k_dual_b<BLK>, dim3(grid), dim3(BLK / 2), 0, st, objs, (const uint32_t *)b.tile_obj.p,
                       (const uint32_t *)b.tile_begin.p, b.ntiles, (const Coef *)b.coefs.p);
    OTF_LAUNCH_CHECK("k_dual_b");
    if (b.n_hp > 0) {
        hipLaunchKernelGGL(k_dual_long_b, dim3((unsigned)cdiv(b.n_hp, kWavesPerBlock)), dim3(kBlk), 0, st, objs,
                           nobj, (const uint32_t *)b.hp_begin.p, (uint32_t)b.n_hp, (const Coef *)b.coefs.p);
        OTF_LAUNCH_CHECK("k_dual_long_b");
    }
    if (b.n_hm > 0) {
        hipLaunchKernelGGL(k_primal_long_b, dim3((unsigned)cdiv(b.n_hm, kWavesPerBlock)), dim3(kBlk), 0, st, objs,
                           nobj, (const uint32_t *)b.hm_begin.p, (uint32_t)b.n_hm, (const Coef *)b.coefs.p);
        OTF_LAUNCH_CHECK("k_primal_long_b");
    }
    hipLaunchKernelGGL(k_primal_b<BLK>, dim3(grid), dim3(BLK), 0, st, objs, (const uint32_t *)b.tile_obj.p,
                       (const uint32_t *)b.tile_begin.p, b.ntiles, (const Coef *)b.coefs.p, b.part.p);
    OTF_LAUNCH_CHECK("k_primal_b");
    hipLaunchKernelGGL(k_batch_counts, dim3((unsigned)nobj), dim3(kBlk), 0, st, objs,
                       (const uint32_t *)b.tile_begin.p, b.ntiles, (const uint32_t *)b.part.p);
    OTF_LAUNCH_CHECK("k_batch_counts");
}

}  // namespace

namespace {
// One k_dual launch: the long + lists' waves first, then the short-list leaves.
void dual_launch(Ctx &c, const DualArgs &a) {
    LeafStore &s = c.lv();
    const int64_t lb = cdiv(s.n_heavy_p, kWavesPerBlock);
    const int64_t nblk = lb + cdiv(c.L, kDualLeaves * kBlk);
    hipLaunchKernelGGL(k_dual, dim3((unsigned)nblk), dim3(kBlk), 0, c.stream, a, c.coef, (uint32_t)s.n_heavy_p,
                       (const uint32_t *)s.heavy_p.p, (uint32_t)lb);
    OTF_LAUNCH_CHECK("k_dual");
}
}  // namespace

void launch_dual(Ctx &c, float sigma) { dual_launch(c, dual_args(c, sigma)); }

void launch_primal(Ctx &c, float tau, float tl) {
    LeafStore &s = c.lv();
    PrimalArgs a = primal_args(c, tau, tl);
    const int64_t lb = cdiv(s.n_heavy_m, kWavesPerBlock);
    const int64_t nblk = lb + cdiv(c.L, kBlk);
    c.s.part.reserve(2 * nblk);
    a.part = c.s.part.p;
    a.part_stride = nblk;
    c.part_blocks = nblk;
    hipLaunchKernelGGL(k_primal, dim3((unsigned)nblk), dim3(kBlk), 0, c.stream, a, c.coef, (uint32_t)s.n_heavy_m,
                       (const uint32_t *)s.heavy_m.p, (uint32_t)lb);
    OTF_LAUNCH_CHECK("k_primal");
}

void launch_gd_flux(Ctx &c, float eps2) {
    LeafStore &s = c.lv();
    DualArgs d = dual_args(c, 0.0f);
    d.ubar = s.u.p;  // the flux differences u itself
    d.gd = 1;
    d.eps2 = eps2;
    dual_launch(c, d);
}

void launch_gd_update(Ctx &c, float lam, float xi, float eps2) {
    LeafStore &s = c.lv();
    PrimalArgs a = primal_args(c, 1.0f, 0.0f);
    const int64_t lb = cdiv(s.n_heavy_m, kWavesPerBlock);
    const int64_t nblk = lb + cdiv(c.L, kBlk);
    c.s.part.reserve(2 * nblk);
    a.part = c.s.part.p;
    a.part_stride = nblk;
    c.part_blocks = nblk;
    a.gd = 1;
    a.lam = lam;
    a.xi = xi;
    a.eps2 = eps2;
    hipLaunchKernelGGL(k_gd_update, dim3((unsigned)nblk), dim3(kBlk), 0, c.stream, a, c.coef, (uint32_t)s.n_heavy_m,
                       (const uint32_t *)s.heavy_m.p, (uint32_t)lb);
    OTF_LAUNCH_CHECK("k_gd_update");
}

void count_flags(Ctx &c) {
    const int64_t nblk = c.part_blocks;  // blocks of the last primal launch
    sum_parts(c, c.s.part.p, nblk, 2, nblk, c.counters.p);  // counters[0] split flags, [1] join flags
}

void energy(Ctx &c, double *tv, double *data, double eps) {
    LeafStore &s = c.lv();
    const int64_t blocks = cdiv(c.L, kBlk);
    c.s.dred.reserve(2 * blocks);
    hipLaunchKernelGGL(k_energy, dim3((unsigned)blocks), dim3(kBlk), 0, c.stream, c.L, c.prm.max_depth, s.level.p,
                       s.u.p, s.nbp_off.p, s.nbp.p, s.obs_off.p, s.obs_m.p, s.inv.p, c.op().F.p, c.op().W.p, c.coef,
                       eps * eps, c.s.dred.p);
    OTF_LAUNCH_CHECK("k_energy");
    std::vector<double> h(2 * blocks);
    OTF_HIP(hipMemcpyAsync(h.data(), c.s.dred.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    OTF_HIP(hipStreamSynchronize(c.stream));
    double t = 0.0, d = 0.0;
    for (int64_t b = 0; b < blocks; ++b) {
        t += h[2 * b];
        d += h[2 * b + 1];
    }
    *tv = t;
    *data = d;
}

// ------------------------------------------- energy without allocation
// For callers that cannot allocate device memory (graph capture, serving
// loops): the block partial sums and the two totals live in a static device
// array of the library instead of context scratch. Each device holds its own
// copy until the process ends; host code reaches it only through the address
// hipGetSymbolAddress returns on that device (the array's name on the host is
// a stand-in, not a device address). Calls on one device share the array:
// overlapping calls race.
constexpr int64_t kEnergyScratchBlocks = kLeafLimit / kBlk;  // 2^26 leaves at most
constexpr int kMaxDevices = 64;
static __device__ __align__(256) double energy_scratch[2 * kEnergyScratchBlocks + 2];

namespace {
// Totals of the partials in block order, the same order as the host sum of
// energy(), so the result is bit-identical.
__global__ void k_energy_total(const double *partial, int64_t blocks, double *out) {
    if (threadIdx.x != 0) return;
    double t = 0.0, d = 0.0;
    for (int64_t b = 0; b < blocks; ++b) {
        t += partial[2 * b];
        d += partial[2 * b + 1];
    }
    out[0] = t;
    out[1] = d;
}

std::mutex g_energy_scratch_mu;
double *g_energy_scratch[kMaxDevices] = {};

// The array's device address on the current device, looked up once per device.
double *energy_scratch_on(int device) {
    if (device < 0 || device >= kMaxDevices) fail(OTF_E_INVALID, "device index out of range");
    std::lock_guard<std::mutex> lock(g_energy_scratch_mu);
    if (!g_energy_scratch[device]) {
        void *p = nullptr;
        OTF_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(energy_scratch)));
        g_energy_scratch[device] = static_cast<double *>(p);
    }
    return g_energy_scratch[device];
}
}  // namespace

void energy_noalloc(Ctx &c, double *tv, double *data) {
    const int64_t blocks = cdiv(c.L, kBlk);
    if (blocks > kEnergyScratchBlocks) fail(OTF_E_CAPACITY, "more leaves than the static energy scratch holds (2^26)");
    double *scr = energy_scratch_on(c.device);
    double h[2] = {0.0, 0.0};
    if (blocks > 0) {
        LeafStore &s = c.lv();
        hipLaunchKernelGGL(k_energy, dim3((unsigned)blocks), dim3(kBlk), 0, c.stream, c.L, c.prm.max_depth,
                           s.level.p, s.u.p, s.nbp_off.p, s.nbp.p, s.obs_off.p, s.obs_m.p, s.inv.p, c.op().F.p,
                           c.op().W.p, c.coef, 0.0, scr);
        OTF_LAUNCH_CHECK("k_energy");
        hipLaunchKernelGGL(k_energy_total, dim3(1), dim3(64), 0, c.stream, (const double *)scr, blocks,
                           scr + 2 * kEnergyScratchBlocks);
        OTF_LAUNCH_CHECK("k_energy_total");
        OTF_HIP(hipMemcpyAsync(h, scr + 2 * kEnergyScratchBlocks, sizeof h, hipMemcpyDeviceToHost, c.stream));
        OTF_HIP(hipStreamSynchronize(c.stream));
    }
    *tv = h[0];
    *data = h[1];
}

uint32_t take_bounds_flag() {
#ifdef OTF_DEBUG_BOUNDS
    uint32_t h = 0, z = 0;
    OTF_HIP(hipMemcpyFromSymbol(&h, HIP_SYMBOL(bounds_flag), sizeof h));
    if (h) OTF_HIP(hipMemcpyToSymbol(HIP_SYMBOL(bounds_flag), &z, sizeof z));
    return h;
#else
    return 0;
#endif
}

BatchState::~BatchState() {
    if (h_stage) (void)hipHostFree(h_stage);
    if (staged) (void)hipEventDestroy(staged);
}

void batch_upload(hipStream_t st, BatchState &b, float sigma, float tau, float tl) {
    const int nobj = (int)b.objs.size();
    const int blk = b.cfg.blk;
    if (!b.coefs.p) {
        std::vector<Coef> cf(kMaxDepth + 1);
        for (int D = 1; D <= kMaxDepth; ++D) cf[D] = make_coef(D);
        b.coefs.reserve(kMaxDepth + 1);
        OTF_HIP(hipMemcpy(b.coefs.p, cf.data(), cf.size() * sizeof(Coef), hipMemcpyHostToDevice));
    }
    const size_t tbytes = (size_t)nobj * sizeof(ObjDev), ibytes = (size_t)(nobj + 1) * sizeof(uint32_t);
    size_t ntiles = 0;
    for (int j = 0; j < nobj; ++j) ntiles += (size_t)cdiv(b.objs[j]->L, blk);
    if (ntiles >= (size_t)UINT32_MAX) fail(OTF_E_CAPACITY, "too many batch tiles");
    const size_t obytes = std::max<size_t>(ntiles, 1) * sizeof(uint32_t);
    const size_t need = tbytes + 3 * ibytes + obytes;
    if (b.staged) OTF_HIP(hipEventSynchronize(b.staged));  // the previous upload has left the staging area
    else OTF_HIP(hipEventCreateWithFlags(&b.staged, hipEventDisableTiming));
    if (need > b.h_cap) {
        if (b.h_stage) OTF_HIP(hipHostFree(b.h_stage));
        b.h_stage = nullptr;
        OTF_HIP(hipHostMalloc((void **)&b.h_stage, 2 * need, hipHostMallocDefault));
        b.h_cap = 2 * need;
    }
    ObjDev *rec = reinterpret_cast<ObjDev *>(b.h_stage);
    uint32_t *tb = reinterpret_cast<uint32_t *>(b.h_stage + tbytes);
    uint32_t *hp = tb + (nobj + 1), *hm = hp + (nobj + 1);
    uint32_t *to = hm + (nobj + 1);  // member of each tile
    tb[0] = hp[0] = hm[0] = 0;
    for (int j = 0; j < nobj; ++j) {
        Ctx &c = *b.objs[j];
        LeafStore &s = c.lv();
        rec[j].d = dual_args(c, sigma);
        rec[j].p = primal_args(c, tau, tl);
        rec[j].heavy_p = s.heavy_p.p;
        rec[j].heavy_m = s.heavy_m.p;
        rec[j].counters = c.counters.p;
        rec[j].D = c.prm.max_depth;
        tb[j + 1] = tb[j] + (uint32_t)cdiv(c.L, blk);
        for (uint32_t t = tb[j]; t < tb[j + 1]; ++t) to[t] = (uint32_t)j;
        hp[j + 1] = hp[j] + (uint32_t)s.n_heavy_p;
        hm[j + 1] = hm[j] + (uint32_t)s.n_heavy_m;
    }
    b.ntiles = tb[nobj];
    b.n_hp = hp[nobj];
    b.n_hm = hm[nobj];
    b.table.reserve(tbytes);
    b.tile_begin.reserve(nobj + 1);
    b.hp_begin.reserve(nobj + 1);
    b.hm_begin.reserve(nobj + 1);
    b.part.reserve(2 * (size_t)b.ntiles);
    b.tile_obj.reserve(std::max<size_t>(b.ntiles, 1));
    OTF_HIP(hipMemcpyAsync(b.table.p, rec, tbytes, hipMemcpyHostToDevice, st));
    OTF_HIP(hipMemcpyAsync(b.tile_obj.p, to, (size_t)b.ntiles * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    OTF_HIP(hipMemcpyAsync(b.tile_begin.p, tb, ibytes, hipMemcpyHostToDevice, st));
    OTF_HIP(hipMemcpyAsync(b.hp_begin.p, hp, ibytes, hipMemcpyHostToDevice, st));
    OTF_HIP(hipMemcpyAsync(b.hm_begin.p, hm, ibytes, hipMemcpyHostToDevice, st));
    OTF_HIP(hipEventRecord(b.staged, st));
}

void batch_sweeps(hipStream_t st, BatchState &b) {
    switch (b.cfg.blk) {
        case 64: launch_batch<64>(st, b); break;
        case 128: launch_batch<128>(st, b); break;
        case 256: launch_batch<256>(st, b); break;
        case 512: launch_batch<512>(st, b); break;
        default: fail(OTF_E_INVALID, "unsupported batch block size");
    }
}

}  // namespace otf
