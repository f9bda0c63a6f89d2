// Construction (Sec. 3.1): per-view TSDF at every finest voxel (Eq. 1), the
// spread rule (Eq. 2) over a dense per-view pyramid, the per-view linear
// octrees, and the union structure that seeds the fused octree (Fig. 1).
//
// Dense pyramid of levels 0..D-1 in (level, Morton) order: level l holds 8^l
// nodes starting at (8^l - 1) / 7. The finest level D is never stored densely;
// its values are recomputed from the range maps where needed.
#include "otf_internal.h"

namespace otf {
namespace {

constexpr int kBlk = 256;

__host__ __device__ inline int64_t lvl_off(int l) { return ((int64_t(1) << (3 * l)) - 1) / 7; }

struct Pyr {
    float *S;
    uint32_t *cnt;
    float *mn, *mx;
    uint8_t *stored;
};

struct EvalArgs {
    CamDev cam;
    const float *depth;
    float h, delta, eta;
    int D;
};

__device__ inline bool splits(const Pyr &P, int64_t i, int l, int D, float spread_tau) {
    return l < D && P.cnt[i] > 0u && (P.mx[i] - P.mn[i]) > spread_tau;
}

// Level D-1 from its 8 finest voxels each (sums in child order 0..7).
__global__ void __launch_bounds__(kBlk) k_eval_reduce(EvalArgs a, Pyr P) {
    const int64_t n = int64_t(1) << (3 * (a.D - 1));
    const int64_t m = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    if (m >= n) return;
    uint32_t X, Y, Z;
    demorton3((uint32_t)m, X, Y, Z);
    float S = 0.0f, lo = INFINITY, hi = -INFINITY;
    uint32_t cnt = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        float f;
        if (tsdf_voxel(a.cam, a.depth, a.h, a.delta, a.eta, 2 * X + (c & 1), 2 * Y + ((c >> 1) & 1),
                       2 * Z + ((c >> 2) & 1), f)) {
            S = S + f;
            ++cnt;
            lo = fminf(lo, f);
            hi = fmaxf(hi, f);
        } else {
            S = S + 0.0f;
        }
    }
    const int64_t i = lvl_off(a.D - 1) + m;
    P.S[i] = S;
    P.cnt[i] = cnt;
    P.mn[i] = lo;
    P.mx[i] = hi;
}

__global__ void __launch_bounds__(kBlk) k_reduce_level(Pyr P, int l) {
    const int64_t n = int64_t(1) << (3 * l);
    const int64_t m = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    if (m >= n) return;
    const int64_t cb = lvl_off(l + 1) + 8 * m;
    float S = 0.0f, lo = INFINITY, hi = -INFINITY;
    uint32_t cnt = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        S = S + P.S[cb + c];
        cnt += P.cnt[cb + c];
        lo = fminf(lo, P.mn[cb + c]);
        hi = fmaxf(hi, P.mx[cb + c]);
    }
    const int64_t i = lvl_off(l) + m;
    P.S[i] = S;
    P.cnt[i] = cnt;
    P.mn[i] = lo;
    P.mx[i] = hi;
}

// stored(l, m) = l == 0 or (stored(parent) and parent splits)
__global__ void __launch_bounds__(kBlk) k_stored(Pyr P, int l, int D, float spread_tau) {
    const int64_t n = int64_t(1) << (3 * l);
    const int64_t m = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    if (m >= n) return;
    uint8_t s = 1;
    if (l > 0) {
        const int64_t p = lvl_off(l - 1) + (m >> 3);
        s = (P.stored[p] && splits(P, p, l - 1, D, spread_tau)) ? 1 : 0;
    }
    P.stored[lvl_off(l) + m] = s;
}

__global__ void __launch_bounds__(kBlk) k_last_split_flags(Pyr P, int D, float spread_tau, uint8_t *flag) {
    const int64_t n = int64_t(1) << (3 * (D - 1));
    const int64_t m = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    if (m >= n) return;
    const int64_t i = lvl_off(D - 1) + m;
    flag[m] = (P.stored[i] && splits(P, i, D - 1, D, spread_tau)) ? 1 : 0;
}

struct PoolDev {
    float *S;
    uint32_t *cnt, *child, *key;
    uint8_t *level;
};

// Stored nodes of levels 0..D-1 into the view's pool segment; marks union splits.
__global__ void __launch_bounds__(kBlk) k_emit_upper(Pyr P, int D, float spread_tau, const uint32_t *idx,
                                                     const uint32_t *rankS, uint32_t base, uint32_t upper_total,
                                                     PoolDev out, uint8_t *usplit) {
    const int64_t N = lvl_off(D);
    const int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    if (i >= N || !P.stored[i]) return;
    int l = 0;
    while (lvl_off(l + 1) <= i) ++l;
    const int64_t m = i - lvl_off(l);
    const uint32_t o = base + idx[i];
    const bool sp = splits(P, i, l, D, spread_tau);
    out.S[o] = P.S[i];
    out.cnt[o] = P.cnt[i];
    out.key[o] = (uint32_t)m << (3 * (D - l));
    out.level[o] = (uint8_t)l;
    uint32_t ch = kNone;
    if (sp) {
        ch = (l < D - 1) ? base + idx[lvl_off(l + 1) + 8 * m] : base + upper_total + 8u * rankS[m];
        usplit[i] = 1;
    }
    out.child[o] = ch;
}

// Finest stored nodes: the 8 voxels below every stored, split level D-1 node.
__global__ void __launch_bounds__(kBlk) k_emit_finest(EvalArgs a, const uint8_t *flag, const uint32_t *rankS,
                                                      uint32_t base, uint32_t upper_total, PoolDev out) {
    const int64_t n = int64_t(1) << (3 * (a.D - 1));
    const int64_t m = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    if (m >= n || !flag[m]) return;
    uint32_t X, Y, Z;
    demorton3((uint32_t)m, X, Y, Z);
    const uint32_t o0 = base + upper_total + 8u * rankS[m];
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        float f = 0.0f;
        bool ob = tsdf_voxel(a.cam, a.depth, a.h, a.delta, a.eta, 2 * X + (c & 1), 2 * Y + ((c >> 1) & 1),
                             2 * Z + ((c >> 2) & 1), f);
        const uint32_t o = o0 + c;
        out.S[o] = ob ? f : 0.0f;
        out.cnt[o] = ob ? 1u : 0u;
        out.key[o] = (uint32_t)(8 * m + c);
        out.level[o] = (uint8_t)a.D;
        out.child[o] = kNone;
    }
}

// Union structure: leaf counts bottom-up.
__global__ void __launch_bounds__(kBlk) k_union_count(const uint8_t *usplit, uint32_t *lc, int l, int D) {
    const int64_t n = int64_t(1) << (3 * l);
    const int64_t m = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    if (m >= n) return;
    const int64_t i = lvl_off(l) + m;
    uint32_t v = 1;
    if (usplit[i]) {
        if (l == D - 1) {
            v = 8;
        } else {
            v = 0;
            const int64_t cb = lvl_off(l + 1) + 8 * m;
            for (int c = 0; c < 8; ++c) v += lc[cb + c];
        }
    }
    lc[i] = v;
}

// Top-down offsets (Morton order of the leaves) and reachability.
__global__ void __launch_bounds__(kBlk) k_union_offsets(const uint8_t *usplit, const uint32_t *lc, uint32_t *off,
                                                        uint8_t *reach, int l) {
    const int64_t n = int64_t(1) << (3 * l);
    const int64_t m = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    if (m >= n) return;
    const int64_t i = lvl_off(l) + m;
    if (l == 0) {
        off[i] = 0;
        reach[i] = 1;
        return;
    }
    const int64_t p = lvl_off(l - 1) + (m >> 3);
    const uint8_t r = (reach[p] && usplit[p]) ? 1 : 0;
    reach[i] = r;
    uint32_t o = off[p];
    const int64_t sb = lvl_off(l) + (m & ~int64_t(7));
    for (int64_t c = 0; c < (m & 7); ++c) o += lc[sb + c];
    off[i] = o;
}

__global__ void __launch_bounds__(kBlk) k_union_emit(const uint8_t *usplit, const uint32_t *off,
                                                     const uint8_t *reach, int D, uint32_t *key, uint8_t *level) {
    const int64_t N = lvl_off(D);
    const int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    if (i >= N || !reach[i]) return;
    int l = 0;
    while (lvl_off(l + 1) <= i) ++l;
    const int64_t m = i - lvl_off(l);
    if (!usplit[i]) {
        key[off[i]] = (uint32_t)m << (3 * (D - l));
        level[off[i]] = (uint8_t)l;
    } else if (l == D - 1) {
        for (int c = 0; c < 8; ++c) {
            key[off[i] + c] = (uint32_t)(8 * m + c);
            level[off[i] + c] = (uint8_t)D;
        }
    }
}

__global__ void k_fill_u8(uint8_t *p, int64_t n, uint8_t v) {
    int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    if (i < n) p[i] = v;
}

template <class T>
void grow_keep(Ctx &c, DBuf<T> &b, size_t used, size_t need) {
    if (need <= b.n && b.p) return;
    size_t cap = b.n ? b.n : 1024;
    while (cap < need) cap *= 2;
    DBuf<T> nb;
    nb.reserve(cap);
    if (used && b.p) OTF_HIP(hipMemcpyAsync(nb.p, b.p, used * sizeof(T), hipMemcpyDeviceToDevice, c.stream));
    b.swap(nb);
    OTF_HIP(hipStreamSynchronize(c.stream));  // the old buffer is freed when nb leaves scope
}

unsigned grid(int64_t n) { return (unsigned)cdiv(n, kBlk); }

}  // namespace

void build_views_and_union(Ctx &c, const float *depth_dev, const std::vector<CamDev> &cams) {
    const int D = c.prm.max_depth;
    const int64_t N = lvl_off(D);                // pyramid nodes, levels 0..D-1
    const int64_t nlast = int64_t(1) << (3 * (D - 1));
    // pyramid scratch
    DBuf<float> S, mn, mx;
    DBuf<uint32_t> cnt, idx, rankS;
    DBuf<uint8_t> stored, lastflag, usplit;
    S.reserve(N);
    mn.reserve(N);
    mx.reserve(N);
    cnt.reserve(N);
    idx.reserve(N);
    stored.reserve(N);
    rankS.reserve(nlast);
    lastflag.reserve(nlast);
    usplit.reserve(N);
    hipLaunchKernelGGL(k_fill_u8, dim3(grid(N)), dim3(kBlk), 0, c.stream, usplit.p, N, (uint8_t)0);
    Pyr P{S.p, cnt.p, mn.p, mx.p, stored.p};

    ViewStore &vs = c.views;
    vs.count.assign(c.n_views, 0);
    vs.base.assign(c.n_views, 0);
    int64_t used = 0;
    const size_t H = (size_t)cams[0].height, W = (size_t)cams[0].width;
    EvalArgs ea;
    ea.h = ldexpf(1.0f, -D);
    ea.delta = c.prm.delta;
    ea.eta = c.prm.eta;
    ea.D = D;
    for (int v = 0; v < c.n_views; ++v) {
        ea.cam = cams[v];
        ea.depth = depth_dev + (size_t)v * H * W;
        hipLaunchKernelGGL(k_eval_reduce, dim3(grid(nlast)), dim3(kBlk), 0, c.stream, ea, P);
        OTF_LAUNCH_CHECK("k_eval_reduce");
        for (int l = D - 2; l >= 0; --l) {
            hipLaunchKernelGGL(k_reduce_level, dim3(grid(int64_t(1) << (3 * l))), dim3(kBlk), 0, c.stream, P, l);
            OTF_LAUNCH_CHECK("k_reduce_level");
        }
        for (int l = 0; l < D; ++l) {
            hipLaunchKernelGGL(k_stored, dim3(grid(int64_t(1) << (3 * l))), dim3(kBlk), 0, c.stream, P, l, D,
                               c.prm.spread_tau);
            OTF_LAUNCH_CHECK("k_stored");
        }
        hipLaunchKernelGGL(k_last_split_flags, dim3(grid(nlast)), dim3(kBlk), 0, c.stream, P, D, c.prm.spread_tau,
                           lastflag.p);
        const uint32_t upper = scan_exclusive_u8(c, stored.p, idx.p, N);
        const uint32_t nsplit_last = scan_exclusive_u8(c, lastflag.p, rankS.p, nlast);
        const int64_t nv = (int64_t)upper + 8 * (int64_t)nsplit_last;
        if (used + nv > (int64_t)0xFFFFFFF0) fail(OTF_E_CAPACITY, "view octrees exceed 2^32 nodes");
        grow_keep(c, vs.S, used, used + nv);
        grow_keep(c, vs.cnt, used, used + nv);
        grow_keep(c, vs.child, used, used + nv);
        grow_keep(c, vs.key, used, used + nv);
        grow_keep(c, vs.level, used, used + nv);
        PoolDev pd{vs.S.p, vs.cnt.p, vs.child.p, vs.key.p, vs.level.p};
        hipLaunchKernelGGL(k_emit_upper, dim3(grid(N)), dim3(kBlk), 0, c.stream, P, D, c.prm.spread_tau, idx.p,
                           rankS.p, (uint32_t)used, upper, pd, usplit.p);
        OTF_LAUNCH_CHECK("k_emit_upper");
        hipLaunchKernelGGL(k_emit_finest, dim3(grid(nlast)), dim3(kBlk), 0, c.stream, ea, lastflag.p, rankS.p,
                           (uint32_t)used, upper, pd);
        OTF_LAUNCH_CHECK("k_emit_finest");
        vs.base[v] = used;
        vs.count[v] = nv;
        used += nv;
    }
    vs.n_nodes = used;
    std::vector<uint32_t> roots(c.n_views);
    for (int v = 0; v < c.n_views; ++v) roots[v] = (uint32_t)vs.base[v];
    vs.root.reserve(c.n_views);
    OTF_HIP(hipMemcpyAsync(vs.root.p, roots.data(), roots.size() * sizeof(uint32_t), hipMemcpyHostToDevice,
                           c.stream));

    // union structure -> leaves in Morton order
    DBuf<uint32_t> lc, off;
    DBuf<uint8_t> reach;
    lc.reserve(N);
    off.reserve(N);
    reach.reserve(N);
    for (int l = D - 1; l >= 0; --l) {
        hipLaunchKernelGGL(k_union_count, dim3(grid(int64_t(1) << (3 * l))), dim3(kBlk), 0, c.stream, usplit.p,
                           lc.p, l, D);
        OTF_LAUNCH_CHECK("k_union_count");
    }
    for (int l = 0; l < D; ++l) {
        hipLaunchKernelGGL(k_union_offsets, dim3(grid(int64_t(1) << (3 * l))), dim3(kBlk), 0, c.stream, usplit.p,
                           lc.p, off.p, reach.p, l);
        OTF_LAUNCH_CHECK("k_union_offsets");
    }
    uint32_t L0 = 0;
    read_back(c, {{lc.p, 9}});
    L0 = c.h_counters[9];
    if (c.prm.max_leaves > 0 && (int64_t)L0 > c.prm.max_leaves) fail(OTF_E_CAPACITY, "initial leaves exceed max_leaves");
    if ((int64_t)L0 >= kLeafLimit) fail(OTF_E_CAPACITY, "initial leaves exceed 2^26");
    c.cur = 0;
    c.lv().reserve(L0);
    hipLaunchKernelGGL(k_union_emit, dim3(grid(N)), dim3(kBlk), 0, c.stream, usplit.p, off.p, reach.p, D,
                       c.lv().key.p, c.lv().level.p);
    OTF_LAUNCH_CHECK("k_union_emit");
    c.L = L0;
    OTF_HIP(hipStreamSynchronize(c.stream));  // scratch buffers are freed on return
}

}  // namespace otf
