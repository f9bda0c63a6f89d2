// Split and join of leaves after the primal update (Sec. 3.2, the two
// restructuring rules), keeping the leaf arrays in Morton order without a sort.
//
// Join: a leaf is joinable when |u+| > tau_j; an inner node collapses when
// every leaf below it is joinable with one sign, and only the largest such node
// is kept. Runs of consecutive same-sign joinable leaves are found with a
// max-scan of run heads; a leaf's collapse node is the largest aligned block
// containing it whose key range lies inside its run. The new leaf takes the
// hierarchical means (1/8 of the sum of its 8 children, recursively) of u,
// ubar and p.
// Split: a leaf with |u+| < tau_s above max depth becomes 8 children that
// inherit u', u_old and p; each child re-runs the prox on its own observations
// and splits again while still flagged (rounds of one level each).
// Emission: every old leaf contributes 0 (absorbed), 1 (kept or collapse
// head) or its cascade's leaf count; an exclusive scan of these counts gives
// the Morton-ordered positions in the new arrays.
#include "otf_internal.h"

namespace otf {
namespace {

constexpr int kBlk = 256;
unsigned grid(int64_t n) { return (unsigned)cdiv(n > 0 ? n : 1, kBlk); }
#define TID() ((int64_t)blockIdx.x * kBlk + threadIdx.x)

// ---------------------------------------------------------------- joins
__global__ void k_run_ends(int64_t L, const uint8_t *flag, const uint32_t *rs, uint32_t *runend) {
    const int64_t i = TID();
    if (i >= L) return;
    const uint8_t j = flag[i] & 6;
    if (!j) return;
    if (i == L - 1 || (flag[i + 1] & 6) != j) runend[rs[i]] = (uint32_t)i;
}

// The coarsest level whose node starts at key k (k aligned to its size).
__device__ inline int align_level(uint32_t k, int D) {
    if (k == 0u) return 0;
    const int l = D - (int)(__builtin_ctz(k) / 3);
    return l < 0 ? 0 : l;
}

// Per leaf: collapse target level jt (0xFF: none), head flag, and cand = 1
// if the leaf is the first leaf of some inner node inside its collapse block
// (a node at a level q with jt <= q < the leaf's level, starting at its key),
// i.e. it computes a hierarchical mean at some level. A thread takes two
// leaves (i and i + kBlk of its block's 2 kBlk), each step of their lookup
// chains (run start, run end, end key and level) issued for both together.
constexpr int kJoinLeaves = 2;

__global__ void __launch_bounds__(kBlk) k_join_target(int64_t L, int D, const uint8_t *flag, const uint32_t *key,
                                                      const uint8_t *level, const uint32_t *rs,
                                                      const uint32_t *runend, uint8_t *jt, uint8_t *jhead,
                                                      uint32_t *part, uint8_t *cand) {
    constexpr int N = kJoinLeaves;
    int64_t idx[N];
    bool on[N];
    uint32_t s[N], e[N], k[N];
    int ln[N];
#pragma unroll
    for (int n = 0; n < N; ++n) {
        idx[n] = ((int64_t)blockIdx.x * N + n) * kBlk + threadIdx.x;
        const bool in = idx[n] < L;
        on[n] = in && (flag[idx[n]] & 6);
        k[n] = in ? key[idx[n]] : 0u;
        ln[n] = in ? level[idx[n]] : 0;
        s[n] = on[n] ? rs[idx[n]] : 0u;
    }
#pragma unroll
    for (int n = 0; n < N; ++n) e[n] = on[n] ? runend[s[n]] : 0u;
    uint64_t K0[N], K1[N];
#pragma unroll
    for (int n = 0; n < N; ++n) {
        K0[n] = on[n] ? key[s[n]] : 0u;
        K1[n] = on[n] ? (uint64_t)key[e[n]] + (uint64_t(1) << (3 * (D - level[e[n]]))) : 0u;
    }
    uint32_t heads = 0;
#pragma unroll
    for (int n = 0; n < N; ++n) {
        uint8_t t = 0xFF, h = 0;
        if (on[n]) {
            for (int l = 0; l < ln[n]; ++l) {
                const uint64_t sz = uint64_t(1) << (3 * (D - l));
                const uint64_t B0 = (uint64_t)k[n] & ~(sz - 1);
                if (B0 >= K0[n] && B0 + sz <= K1[n]) {
                    t = (uint8_t)l;
                    h = ((uint64_t)k[n] == B0) ? 1 : 0;
                    break;
                }
            }
        }
        if (idx[n] < L) {
            jt[idx[n]] = t;
            jhead[idx[n]] = h;
            cand[idx[n]] = (t != 0xFF && max((int)t, align_level(k[n], D)) < ln[n]) ? 1 : 0;
        }
        heads += (uint32_t)__popcll(__ballot(h != 0));
    }
    // per-block count of collapse heads
    __shared__ uint32_t cnt[kBlk / 64];
    if ((threadIdx.x & 63) == 0) cnt[threadIdx.x >> 6] = heads;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t n = 0;
        for (int w = 0; w < kBlk / 64; ++w) n += cnt[w];
        part[blockIdx.x] = n;
    }
}

struct NewStore {
    uint32_t *key;
    uint8_t *level;
    float *u, *ubar, *p;
    int64_t cap;
    uint32_t *obs_off;
    uint8_t *obs_m, *obs_unit;
    float *inv, *wtot;
    uint8_t *isnew;
    uint32_t *src;
    uint8_t *need;
};

struct OldStore {
    const uint32_t *key;
    const uint8_t *level;
    const float *u, *ubar, *p;
    int64_t cap;
    const uint32_t *obs_off;
    const uint8_t *obs_m, *obs_unit;
    const float *inv, *wtot;
    const uint8_t *flag;
};

// Hierarchical means of the collapsed blocks, bottom-up in parallel, in place
// over the old leaf positions. val holds, at the position of a node's first
// leaf, the node's 5 values (u, ubar, px, py, pz); it starts as the leaves'
// own values. For q = D-1 .. 0, every inner node at level q inside a block
// (block level <= q, first leaf deeper than q) reads its 8 children at level
// q+1 (child c starts at the first leaf with key >= key + c * 8^(D-q-1)) and
// stores 1/8 of their sum in child order at its first leaf. Afterwards the
// block's first leaf holds the block's values.
__global__ void k_jval_init(int64_t L, const uint8_t *jt, OldStore o, float *val, int64_t cap) {
    const int64_t i = TID();
    if (i >= L || jt[i] == 0xFF) return;
    val[i] = o.u[i];
    val[cap + i] = o.ubar[i];
    val[2 * cap + i] = o.p[i];
    val[3 * cap + i] = o.p[o.cap + i];
    val[4 * cap + i] = o.p[2 * o.cap + i];
}

// Level q over the candidate list (its length at n_dev): a candidate that
// starts a level-q node inside its collapse block (block level <= q, leaf
// deeper than q) reads the node's 8 children at level q+1 and stores 1/8 of
// their sum in child order at its own position.
__global__ void __launch_bounds__(kBlk) k_jval_level(const uint32_t *list, const uint32_t *n_dev, int64_t L, int D,
                                                     int q, const uint8_t *jt, const uint32_t *key,
                                                     const uint8_t *level, float *val, int64_t cap) {
    const uint32_t n = *n_dev;
    for (uint32_t t = blockIdx.x * kBlk + threadIdx.x; t < n; t += gridDim.x * kBlk) {
        const int64_t i = list[t];
        if (jt[i] > q || level[i] <= q) continue;
        const uint64_t k0 = key[i];
        if (k0 & ((uint64_t(1) << (3 * (D - q))) - 1)) continue;  // not the first leaf of a level-q node
        const uint64_t step = uint64_t(1) << (3 * (D - q - 1));
        int64_t pos[8];
        pos[0] = i;
        const int64_t end = min(L, i + (int64_t)(uint64_t(1) << (3 * (D - q))));
        for (int c = 1; c < 8; ++c) {
            const int64_t lo = pos[c - 1] + 1;
            if (level[pos[c - 1]] == q + 1) {  // child c-1 is a single leaf: child c starts right after it
                pos[c] = lo;
                continue;
            }
            const uint64_t kc = k0 + c * step;
            int64_t a = lo, b = end;  // first index in [lo, end) with key >= kc
            while (a < b) {
                const int64_t m = (a + b) >> 1;
                if ((uint64_t)key[m] < kc) a = m + 1;
                else b = m;
            }
            pos[c] = a;
        }
        float v[5];
        for (int w = 0; w < 5; ++w) {
            float acc = 0.0f;
            for (int c = 0; c < 8; ++c) acc = acc + val[w * cap + pos[c]];
            v[w] = 0.125f * acc;
        }
        for (int w = 0; w < 5; ++w) val[w * cap + i] = v[w];
    }
}

// ---------------------------------------------------------------- splits
__global__ void k_make_parents0(int64_t L, const uint8_t *flag, const uint32_t *rank, uint32_t *porigin) {
    const int64_t i = TID();
    if (i >= L || !(flag[i] & 1)) return;
    porigin[rank[i]] = (uint32_t)i;
}

// children of round 0: parents are old leaves
__global__ void k_children0(int64_t np, int D, const uint32_t *porigin, const uint32_t *key, const uint8_t *level,
                            uint32_t *ckey, uint8_t *clevel, uint32_t *corigin) {
    const int64_t j = TID();
    if (j >= 8 * np) return;
    const int64_t q = j >> 3;
    const int c = (int)(j & 7);
    const uint32_t o = porigin[q];
    const int l = level[o] + 1;
    ckey[j] = key[o] | ((uint32_t)c << (3 * (D - l)));
    clevel[j] = (uint8_t)l;
    corigin[j] = o;
}

// children of a later round: parents are the split children of the previous one
__global__ void k_children_next(int64_t nc_prev, int D, const uint8_t *csplit, const uint32_t *crank,
                                const uint32_t *pkey, const uint8_t *plevel, const uint32_t *porig,
                                uint32_t *ckey, uint8_t *clevel, uint32_t *corigin) {
    const int64_t jp = TID();
    if (jp >= nc_prev || !csplit[jp]) return;
    const int64_t q = crank[jp];
    const int l = plevel[jp] + 1;
    for (int c = 0; c < 8; ++c) {
        ckey[8 * q + c] = pkey[jp] | ((uint32_t)c << (3 * (D - l)));
        clevel[8 * q + c] = (uint8_t)l;
        corigin[8 * q + c] = porig[jp];
    }
}

// Children's values: the prox of the parent's u' on the child's own
// observations (primal-dual), or the parent's descent step (divergence kept in
// uprime) with the child's own data term (gradient descent).
__global__ void k_cascade_prox(int64_t nc, int stride, const float *tF, const float *tW, const uint8_t *tM,
                               const uint8_t *tU, const float *tInv, const float *tWt, const uint32_t *corigin,
                               const uint8_t *clevel, const float *uprime, const float *uold, float tl,
                               float split_tau, int D, Solver sol, float *cu, float *cub, uint8_t *csplit) {
    const int64_t j = TID();
    if (j >= nc) return;
    const uint32_t o = corigin[j];
    const float up = uprime[o], uo = uold[o];
    const float *F = tF + j * (int64_t)stride, *W = tW + j * (int64_t)stride;
    float val;
    if (sol.gd) {
        // data gradient terms in one sequential chain in (F, view) order
        const int M = tM[j];
        float x = 0.0f;
        for (int k = 0; k < M; ++k) {
            const float r = uo - F[k];
            const float den = sqrtf(__fmaf_rn(r, r, sol.eps2));
            x = x + W[k] * (r / den);
        }
        val = __fmaf_rn(sol.xi, __fmaf_rn(sol.lam, up, -(x * tInv[j])), uo);
        cu[j] = val;
        cub[j] = val;
    } else {
        val = prox_select(up, tl * tInv[j], tM[j], tU[j] != 0, F, W, tWt[j]);
        cu[j] = val;
        cub[j] = __fmaf_rn(2.0f, val, -uo);
    }
    csplit[j] = (fabsf(val) < split_tau && clevel[j] < D) ? 1 : 0;
}

__global__ void k_leafcnt(int64_t nc, const uint8_t *csplit, const uint32_t *crank, const uint32_t *next_cnt,
                          uint32_t *cnt) {
    const int64_t j = TID();
    if (j >= nc) return;
    uint32_t s = 1;
    if (csplit[j]) {
        const int64_t q = crank[j];
        s = 0;
        for (int c = 0; c < 8; ++c) s += next_cnt[8 * q + c];
    }
    cnt[j] = s;
}

// ---------------------------------------------------------------- emission
// Per old leaf its number of new-store leaves; per block the number of those
// that are new (collapse heads and cascade leaves) into part[blockIdx].
__global__ void __launch_bounds__(kBlk) k_out_count(int64_t L, const uint8_t *flag, const uint8_t *jt,
                                                    const uint8_t *jhead, const uint32_t *rank0,
                                                    const uint32_t *cnt0, uint32_t *cnt, uint32_t *part) {
    const int64_t i = TID();
    uint32_t v = 1, fresh = 0;
    if (i < L) {
        if (jt && jt[i] != 0xFF) {
            v = jhead[i] ? 1u : 0u;
            fresh = v;
        } else if (rank0 && (flag[i] & 1)) {
            const int64_t q = rank0[i];
            v = 0;
            for (int c = 0; c < 8; ++c) v += cnt0[8 * q + c];
            fresh = v;
        }
        cnt[i] = v;
    }
    __shared__ uint32_t red[kBlk / 64];
    uint32_t w = fresh;
    for (int off = 32; off > 0; off >>= 1) w += (uint32_t)__shfl_xor((int)w, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t t = 0;
        for (int k = 0; k < kBlk / 64; ++k) t += red[k];
        part[blockIdx.x] = t;
    }
}

// Kept leaves are copied; the head of a collapse writes the collapsed leaf
// (its level and hierarchical means, computed in place at the head's old
// position: val[k * vcap + i] for u, ubar, p_x, p_y, p_z); absorbed and split
// leaves write nothing here.
__global__ void k_emit_keep(int64_t L, OldStore o, const uint8_t *jt, const uint8_t *jhead, const float *val,
                            int64_t vcap, int splits, const uint32_t *out_off, NewStore ns) {
    const int64_t i = TID();
    if (i >= L) return;
    if (jt && jt[i] != 0xFF) {
        if (!jhead[i]) return;
        const uint32_t w = out_off[i];
        ns.key[w] = o.key[i];
        ns.level[w] = jt[i];
        ns.u[w] = val[i];
        ns.ubar[w] = val[vcap + i];
        ns.p[w] = val[2 * vcap + i];
        ns.p[ns.cap + w] = val[3 * vcap + i];
        ns.p[2 * ns.cap + w] = val[4 * vcap + i];
        ns.isnew[w] = 1;
        ns.src[w] = kNone;
        ns.need[w] = 1;
        return;
    }
    if (splits && (o.flag[i] & 1)) return;
    const uint32_t w = out_off[i];
    ns.key[w] = o.key[i];
    ns.level[w] = o.level[i];
    ns.u[w] = o.u[i];
    ns.ubar[w] = o.ubar[i];
    for (int d = 0; d < 3; ++d) ns.p[d * ns.cap + w] = o.p[d * o.cap + i];
    ns.obs_off[w] = o.obs_off[i];
    ns.obs_m[w] = o.obs_m[i];
    ns.obs_unit[w] = o.obs_unit[i];
    ns.inv[w] = o.inv[i];
    ns.wtot[w] = o.wtot[i];
    ns.isnew[w] = 0;
    ns.src[w] = (uint32_t)i;
    ns.need[w] = 0;
}

// A kept leaf next to a changed (absorbed, collapsed or split) leaf must have
// its adjacency searched again.
__device__ inline bool changed(int64_t j, const uint8_t *flag, const uint8_t *jt, int splits) {
    return (jt && jt[j] != 0xFF) || (splits && (flag[j] & 1));
}

// Marked from the changed side (adjacency is symmetric): every kept neighbour
// of a changed leaf; concurrent stores all write 1. The + and - lists are
// walked together, kMarkBatch entries of each at a time, with every load
// unconditional at a valid address (entries past a list's end read entry 0
// and are dropped), so that each step of the lookup chain (entry, changed?,
// new position) is one round of loads in flight.
constexpr int kMarkBatch = 8;

__device__ inline void nbr_mark(int64_t i, int64_t L, const uint8_t *flag, const uint8_t *jt, int splits,
                                const uint32_t *off_p, const uint32_t *ent_p, const uint32_t *off_m,
                                const uint32_t *ent_m, const uint32_t *out_off, uint8_t *need) {
    if (i >= L || !changed(i, flag, jt, splits)) return;
    const uint32_t *ent[2] = {ent_p, ent_m};
    uint32_t b0[2] = {off_p[i], off_m[i]}, b1[2] = {off_p[i + 1], off_m[i + 1]};
#pragma unroll
    for (int sd = 0; sd < 2; ++sd)
        if (b1[sd] - b0[sd] > kLongList) b1[sd] = b0[sd];  // long lists: nbr_mark_long
    const uint32_t len = max(b1[0] - b0[0], b1[1] - b0[1]);
    for (uint32_t k = 0; k < len; k += kMarkBatch) {
        uint32_t n[2][kMarkBatch], o[2][kMarkBatch];
        bool keep[2][kMarkBatch];
#pragma unroll
        for (int sd = 0; sd < 2; ++sd)
#pragma unroll
            for (int r = 0; r < kMarkBatch; ++r) {
                const uint32_t e = b0[sd] + k + r;
                const bool ok = e < b1[sd];
                const uint32_t v = ent[sd][ok ? e : 0u];
                n[sd][r] = ok ? (v & kIdxMask) : 0u;
                keep[sd][r] = ok;
            }
#pragma unroll
        for (int sd = 0; sd < 2; ++sd)
#pragma unroll
            for (int r = 0; r < kMarkBatch; ++r) keep[sd][r] = keep[sd][r] && !changed(n[sd][r], flag, jt, splits);
#pragma unroll
        for (int sd = 0; sd < 2; ++sd)
#pragma unroll
            for (int r = 0; r < kMarkBatch; ++r) o[sd][r] = out_off[keep[sd][r] ? n[sd][r] : 0u];
#pragma unroll
        for (int sd = 0; sd < 2; ++sd)
#pragma unroll
            for (int r = 0; r < kMarkBatch; ++r)
                if (keep[sd][r]) need[o[sd][r]] = 1;
    }
}

// Long lists of changed leaves: one wave per leaf on the old long-list work
// lists (item: + lists, then - lists), lanes striding over the entries.
__device__ inline void nbr_mark_long(uint32_t item, const uint8_t *flag, const uint8_t *jt, int splits,
                                     const uint32_t *off_p, const uint32_t *ent_p, const uint32_t *off_m,
                                     const uint32_t *ent_m, const uint32_t *heavy_p, const uint32_t *heavy_m,
                                     uint32_t n_heavy_p, uint32_t n_heavy_m, const uint32_t *out_off, uint8_t *need) {
    const uint32_t lane = threadIdx.x & 63;
    if (item >= n_heavy_p + n_heavy_m) return;
    const bool plus = item < n_heavy_p;
    const uint32_t i = plus ? heavy_p[item] : heavy_m[item - n_heavy_p];
    if (!changed(i, flag, jt, splits)) return;
    const uint32_t *off = plus ? off_p : off_m;
    const uint32_t *ent = plus ? ent_p : ent_m;
    const uint32_t e1 = off[i + 1];
    for (uint32_t e = off[i] + lane; e < e1; e += 64) {
        const uint32_t n = ent[e] & kIdxMask;
        if (!changed(n, flag, jt, splits)) need[out_off[n]] = 1;
    }
}

// Both in one launch: the first long_blocks blocks take the long lists (a
// wave each), the others one leaf per thread; every store writes 1.
__global__ void __launch_bounds__(kBlk) k_nbr_mark(int64_t L, const uint8_t *flag, const uint8_t *jt, int splits,
                                                   const uint32_t *off_p, const uint32_t *ent_p,
                                                   const uint32_t *off_m, const uint32_t *ent_m,
                                                   const uint32_t *heavy_p, const uint32_t *heavy_m,
                                                   uint32_t n_heavy_p, uint32_t n_heavy_m, uint32_t long_blocks,
                                                   const uint32_t *out_off, uint8_t *need) {
    if (blockIdx.x < long_blocks)
        nbr_mark_long(((uint32_t)blockIdx.x * kBlk + threadIdx.x) >> 6, flag, jt, splits, off_p, ent_p, off_m, ent_m,
                      heavy_p, heavy_m, n_heavy_p, n_heavy_m, out_off, need);
    else
        nbr_mark((int64_t)(blockIdx.x - long_blocks) * kBlk + threadIdx.x, L, flag, jt, splits, off_p, ent_p, off_m,
                 ent_m, out_off, need);
}

__global__ void k_pos0(int64_t nc, const uint32_t *corigin, const uint32_t *out_off, const uint32_t *cnt,
                       uint32_t *pos) {
    const int64_t j = TID();
    if (j >= nc) return;
    const int64_t q = j >> 3;
    uint32_t b = out_off[corigin[j]];
    for (int64_t c = 0; c < (j & 7); ++c) b += cnt[8 * q + c];
    pos[j] = b;
}

// positions of round r+1 children from their parents (split children of round r)
__global__ void k_pos_next(int64_t nc_prev, const uint8_t *csplit, const uint32_t *crank, const uint32_t *ppos,
                           const uint32_t *cnt_next, uint32_t *pos_next) {
    const int64_t jp = TID();
    if (jp >= nc_prev || !csplit[jp]) return;
    const int64_t q = crank[jp];
    uint32_t b = ppos[jp];
    for (int c = 0; c < 8; ++c) {
        pos_next[8 * q + c] = b;
        b += cnt_next[8 * q + c];
    }
}

__global__ void k_emit_final(int64_t nc, const uint8_t *csplit, const uint32_t *pos, const uint32_t *ckey,
                             const uint8_t *clevel, const uint32_t *corigin, const float *cu, const float *cub,
                             const float *p_old, int64_t cap_old, NewStore ns) {
    const int64_t j = TID();
    if (j >= nc || csplit[j]) return;
    const uint32_t w = pos[j];
    const uint32_t o = corigin[j];
    ns.key[w] = ckey[j];
    ns.level[w] = clevel[j];
    ns.u[w] = cu[j];
    ns.ubar[w] = cub[j];
    for (int d = 0; d < 3; ++d) ns.p[d * ns.cap + w] = p_old[d * cap_old + o];
    ns.isnew[w] = 1;
    ns.src[w] = kNone;
    ns.need[w] = 1;
}

__global__ void k_zero_u32(int64_t n, uint32_t *a) {
    const int64_t i = TID();
    if (i < n) a[i] = 0u;
}

// New leaves' observations from their rows (target t: row t * stride, Mt[t]
// entries) to the pool at base + (off_t ? off_t[t] : off_leaf[tidx[t]]), one
// wave per target; the segment offset goes into the leaf header.
__global__ void k_place_obs(int64_t n, const uint32_t *tidx, const uint8_t *Mt, int stride, const float *F0,
                            const float *W0, const float *P0, const uint32_t *off_t, const uint32_t *off_leaf,
                            uint32_t base, float *F1, float *W1, float *P1, uint32_t *obs_off) {
    const int64_t t = ((int64_t)blockIdx.x * kBlk + threadIdx.x) >> 6;
    const int k = threadIdx.x & 63;
    if (t >= n) return;
    const uint32_t h = tidx[t];
    const uint32_t dst = base + (off_t ? off_t[t] : off_leaf[h]);
    if (k < Mt[t]) {
        const size_t src = (size_t)t * stride + k;
        F1[dst + k] = F0[src];
        W1[dst + k] = W0[src];
        P1[dst + k] = P0[src];
    }
    if (k == 0) obs_off[h] = dst;
}

// Pool compaction. A wave takes 64 consecutive leaves, their headers loaded
// one lane each, then copies their segments one leaf after another, lane k
// copying observation k (M <= 64). The loads of kSegAhead leaves are issued
// before the first store; every load is unconditional at a valid address
// (lanes past a segment's end read its first entry; new leaves, whose
// observations are placed afterwards, and leaves past the wave's last read
// entry 0), so that no load waits in a conditional block.
constexpr int kSegAhead = 8;

__global__ void __launch_bounds__(kBlk) k_copy_segments(int64_t L, const uint8_t *isnew, const uint8_t *M,
                                                        const uint32_t *new_off, uint32_t *obs_off, const float *F0,
                                                        const float *W0, const float *P0, float *F1, float *W1,
                                                        float *P1) {
    const int64_t i = TID();
    const int lane = threadIdx.x & 63;
    const bool valid = i < L;
    int m = 0;
    uint32_t src = 0, dst = 0;
    if (valid) {
        dst = new_off[i];
        src = obs_off[i];
        m = isnew[i] ? 0 : (int)M[i];
    }
    const int nact = __popcll(__ballot(valid));
    for (int l0 = 0; l0 < nact; l0 += kSegAhead) {
        float f[kSegAhead], w[kSegAhead], p[kSegAhead];
#pragma unroll
        for (int g = 0; g < kSegAhead; ++g) {
            const int l = min(l0 + g, 63);
            const int ml = __builtin_amdgcn_readlane(m, l);
            const uint32_t sl = (uint32_t)__builtin_amdgcn_readlane((int)src, l);
            const uint32_t e = ml > 0 ? sl + (lane < ml ? (uint32_t)lane : 0u) : 0u;
            f[g] = F0[e];
            w[g] = W0[e];
            p[g] = P0[e];
        }
#pragma unroll
        for (int g = 0; g < kSegAhead; ++g) {
            const int l = min(l0 + g, 63);
            const int ml = l0 + g < nact ? __builtin_amdgcn_readlane(m, l) : 0;
            const uint32_t d = (uint32_t)__builtin_amdgcn_readlane((int)dst, l) + (uint32_t)lane;
            if (lane < ml) {
                F1[d] = f[g];
                W1[d] = w[g];
                P1[d] = p[g];
            }
        }
    }
    if (valid) obs_off[i] = dst;
}

Round &round_at(Ctx &c, size_t r) {
    while (c.s.rounds.size() <= r) c.s.rounds.push_back(new Round());
    return *c.s.rounds[r];
}

}  // namespace

namespace {

// Join analysis: run heads, run ends, collapse target (jt) and head flag
// (jhead) per leaf, the number of collapse heads into counters[2].
void join_analysis(Ctx &c) {
    const int64_t L = c.L;
    const unsigned gL = grid(L);
    Scratch &s = c.s;
    LeafStore &os = c.lv();
    s.b.reserve(L);
    s.c.reserve(L);
    s.u8a.reserve(L);
    s.u8b.reserve(L);
    scan_run_starts(c, os.flag.p, s.b.p, L);
    hipLaunchKernelGGL(k_run_ends, dim3(gL), dim3(kBlk), 0, c.stream, L, os.flag.p, s.b.p, s.c.p);
    s.part.reserve(gL);
    s.r_jcand.reserve(L);
    const unsigned gJ = (unsigned)std::max<int64_t>(1, cdiv(L, kJoinLeaves * kBlk));
    hipLaunchKernelGGL(k_join_target, dim3(gJ), dim3(kBlk), 0, c.stream, L, c.prm.max_depth, os.flag.p, os.key.p,
                       os.level.p, s.b.p, s.c.p, s.u8a.p, s.u8b.p, s.part.p, s.r_jcand.p);
    sum_parts(c, s.part.p, gJ, 1, gJ, c.counters.p + 2);
    // the leaves that compute hierarchical means, listed by one compacting
    // scan (their number stays on the device, at r_jrank[0])
    s.r_jrank.reserve(1);
    s.r_jlist.reserve(L);
    scan_compact_u8(c, s.r_jcand.p, s.r_jlist.p, (uint32_t)L, s.r_jrank.p, L);
    OTF_LAUNCH_CHECK("join analysis");
}

// Rank of the split-flagged leaves (exclusive scan into s.d).
void split_rank(Ctx &c) {
    const int64_t L = c.L;
    Scratch &s = c.s;
    s.d.reserve(L + 1);
    scan_exclusive_flag_bits(c, c.lv().flag.p, 1u, s.d.p, L);
}

// Collapse values: hierarchical means level by level, in place over the old
// leaf positions (scratch r_jv). Queued in pieces (the initial copy, then one
// level each), so that they can fill several host waits: `next` is the first
// piece not yet queued, at most `count` are queued now.
void join_values(Ctx &c, const uint8_t *jt, int &next, int count) {
    const int64_t L = c.L;
    const int D = c.prm.max_depth;
    LeafStore &os = c.lv();
    DBuf<float> &val = c.s.r_jv;
    const OldStore osd{os.key.p, os.level.p, os.u.p, os.ubar.p, os.p.p, os.cap, os.obs_off.p, os.obs_m.p,
                       os.obs_unit.p, os.inv.p, os.wtot.p, os.flag.p};
    for (; count > 0 && next <= D; --count, ++next) {
        if (next == 0) {
            val.reserve(5 * (size_t)L);
            hipLaunchKernelGGL(k_jval_init, dim3(grid(L)), dim3(kBlk), 0, c.stream, L, jt, osd, val.p, L);
        } else {
            const int q = D - next;  // levels D-1 .. 0
            const unsigned gq = (unsigned)std::min<int64_t>(grid(L), 2048);
            hipLaunchKernelGGL(k_jval_level, dim3(gq), dim3(kBlk), 0, c.stream, (const uint32_t *)c.s.r_jlist.p,
                               (const uint32_t *)c.s.r_jrank.p, L, D, q, jt, os.key.p, os.level.p, val.p, L);
        }
    }
    OTF_LAUNCH_CHECK("join means");
}

}  // namespace

bool restructure(Ctx &c, float tl) {
    const int D = c.prm.max_depth;
    const int64_t L = c.L;
    LeafStore &os = c.lv();
    Scratch &s = c.s;
    const unsigned gL = grid(L);
    // While the host waits for the flag counts, the device analyses the joins
    // and ranks the splits when the previous restructure had them (results
    // that turn out unneeded are dropped).
    const uint32_t t_flags = read_back_begin(c, {{c.counters.p, 0}, {c.counters.p + 1, 1}});
    const bool spec_join = c.had_joins, spec_split = c.had_splits;
    if (spec_join) join_analysis(c);
    if (spec_split) split_rank(c);
    read_back_wait(c, t_flags);
    const uint32_t n_split = c.h_counters[0], n_join = c.h_counters[1];
    c.had_joins = n_join > 0;
    c.had_splits = n_split > 0;
    c.last_splits = c.last_joins = 0;
    if (n_split == 0 && n_join == 0) return false;
    if (n_join > 0 && !spec_join) join_analysis(c);
    if (n_split > 0 && !spec_split) split_rank(c);
    const uint8_t *jt = n_join > 0 ? s.u8a.p : nullptr;
    const uint8_t *jhead = n_join > 0 ? s.u8b.p : nullptr;
    int jv_next = 0;  // pieces of the collapse values queued so far
    auto queue_join_values = [&](int count) {
        if (jt) join_values(c, jt, jv_next, count);
    };

    // ---- split cascade
    int64_t nrounds = 0, total_splits = 0, cascade_leaves = 0;
    uint32_t *rank0 = nullptr;
    if (n_split > 0) {
        rank0 = s.d.p;
        const uint32_t np0 = n_split;
        Round &r0 = round_at(c, 0);
        r0.np = np0;
        r0.porigin.reserve(np0);
        hipLaunchKernelGGL(k_make_parents0, dim3(gL), dim3(kBlk), 0, c.stream, L, os.flag.p, rank0, r0.porigin.p);
        int64_t np = np0;
        size_t r = 0;
        const int stride = c.n_views;
        while (np > 0) {
            Round &R = round_at(c, r);
            R.np = np;
            R.nc = 8 * np;
            const int64_t nc = R.nc;
            R.ckey.reserve(nc);
            R.corigin.reserve(nc);
            R.crank.reserve(nc + 1);
            R.cnt.reserve(nc);
            R.pos.reserve(nc);
            R.clevel.reserve(nc);
            R.csplit.reserve(nc);
            R.cu.reserve(nc);
            R.cub.reserve(nc);
            if (r == 0) {
                hipLaunchKernelGGL(k_children0, dim3(grid(nc)), dim3(kBlk), 0, c.stream, np, D, R.porigin.p, os.key.p,
                                   os.level.p, R.ckey.p, R.clevel.p, R.corigin.p);
            } else {
                Round &P = *s.rounds[r - 1];
                hipLaunchKernelGGL(k_children_next, dim3(grid(P.nc)), dim3(kBlk), 0, c.stream, P.nc, D, P.csplit.p,
                                   P.crank.p, P.ckey.p, P.clevel.p, P.corigin.p, R.ckey.p, R.clevel.p, R.corigin.p);
            }
            OTF_LAUNCH_CHECK("cascade children");
            // observations of the children (stride n_views), then their prox
            s.fa.reserve(nc * stride);
            s.fb.reserve(nc * stride);
            s.fc.reserve(nc);
            s.fd.reserve(nc);
            DBuf<uint8_t> &tM = s.r_tM, &tU = s.r_tU;
            tM.reserve(nc);
            tU.reserve(nc);
            gather_fill(c, nc, R.ckey.p, R.clevel.p, nullptr, nullptr, 0, stride, s.fa.p, s.fb.p, nullptr, tM.p, tU.p,
                        s.fc.p, s.fd.p, nullptr, nullptr);
            hipLaunchKernelGGL(k_cascade_prox, dim3(grid(nc)), dim3(kBlk), 0, c.stream, nc, stride, s.fa.p, s.fb.p,
                               tM.p, tU.p, s.fc.p, s.fd.p, R.corigin.p, R.clevel.p, os.uprime.p, os.uold.p, tl,
                               c.prm.split_tau, D, c.sol, R.cu.p, R.cub.p, R.csplit.p);
            OTF_LAUNCH_CHECK("k_cascade_prox");
            scan_exclusive_u32_dev_u8(c, R.csplit.p, R.crank.p, nc);
            const uint32_t t_next = read_back_begin(c, {{R.crank.p + nc, 8}});
            queue_join_values(5);  // independent of the cascade: keeps the device busy meanwhile
            read_back_wait(c, t_next);
            const uint32_t next = c.h_counters[8];
            if (next > nc) fail(OTF_E_DEVICE, "split cascade count out of range");
            total_splits += np;
            cascade_leaves += nc - next;
            np = next;
            ++r;
        }
        nrounds = (int64_t)r;
        // leaf counts bottom-up
        for (int64_t q = nrounds - 1; q >= 0; --q) {
            Round &R = *s.rounds[q];
            const uint32_t *next_cnt = (q + 1 < nrounds) ? s.rounds[q + 1]->cnt.p : nullptr;
            hipLaunchKernelGGL(k_leafcnt, dim3(grid(R.nc)), dim3(kBlk), 0, c.stream, R.nc, R.csplit.p, R.crank.p,
                               next_cnt, R.cnt.p);
            OTF_LAUNCH_CHECK("k_leafcnt");
        }
    }
    queue_join_values(D + 1);

    // ---- emission
    s.e.reserve(L + 1);
    s.f.reserve(L + 1);
    s.part.reserve(gL);
    hipLaunchKernelGGL(k_out_count, dim3(gL), dim3(kBlk), 0, c.stream, L, os.flag.p, jt, jhead, rank0,
                       nrounds ? s.rounds[0]->cnt.p : (const uint32_t *)nullptr, s.e.p, s.part.p);
    OTF_LAUNCH_CHECK("k_out_count");
    sum_parts(c, s.part.p, gL, 1, gL, c.counters.p + 18);
    scan_exclusive_u32_dev(c, s.e.p, s.f.p, L);
    const uint32_t *out_off = s.f.p;
    const uint32_t t_out =
        read_back_begin(c, {{s.f.p + L, 12}, {c.counters.p + 2, 13}, {c.counters.p + 18, 18}});
    // Collapses only remove leaves, so kept leaves plus the cascade's leaves
    // bound the new count: the new store is sized by that bound and filled
    // while the host waits for the exact count (an out-of-range bound waits
    // for the exact count first).
    const int64_t Lub = L - (int64_t)n_split + cascade_leaves;
    int64_t Lnew = -1;
    uint32_t n_new = 0;
    auto take_counts = [&] {
        read_back_wait(c, t_out);
        Lnew = c.h_counters[12];
        n_new = c.h_counters[18];
        if (Lnew >= kLeafLimit) fail(OTF_E_CAPACITY, "leaf count exceeds 2^26");
        if (c.prm.max_leaves > 0 && Lnew > c.prm.max_leaves) fail(OTF_E_CAPACITY, "leaf count exceeds max_leaves");
        if (Lnew > Lub || (int64_t)n_new > Lnew) fail(OTF_E_DEVICE, "restructure counts out of range");
    };
    if (Lub >= kLeafLimit || (c.prm.max_leaves > 0 && Lub > c.prm.max_leaves)) take_counts();
    const int64_t Lsize = Lnew >= 0 ? Lnew : Lub;
    LeafStore &ns = c.leaves[c.cur ^ 1];
    DBuf<uint8_t> &isnew = s.r_isnew;
    ns.reserve(Lsize);
    isnew.reserve(Lsize);
    const NewStore nsd{ns.key.p, ns.level.p, ns.u.p,     ns.ubar.p, ns.p.p, ns.cap, ns.obs_off.p, ns.obs_m.p,
                       ns.obs_unit.p, ns.inv.p, ns.wtot.p,  isnew.p, ns.src.p, ns.need.p};
    const OldStore osd{os.key.p, os.level.p, os.u.p, os.ubar.p, os.p.p, os.cap, os.obs_off.p, os.obs_m.p,
                       os.obs_unit.p, os.inv.p, os.wtot.p, os.flag.p};
    hipLaunchKernelGGL(k_emit_keep, dim3(gL), dim3(kBlk), 0, c.stream, L, osd, jt, jhead,
                       jt ? (const float *)s.r_jv.p : (const float *)nullptr, L, n_split > 0 ? 1 : 0, out_off, nsd);
    OTF_LAUNCH_CHECK("k_emit_keep");
    for (int64_t q = 0; q < nrounds; ++q) {
        Round &R = *s.rounds[q];
        if (q == 0) {
            hipLaunchKernelGGL(k_pos0, dim3(grid(R.nc)), dim3(kBlk), 0, c.stream, R.nc, R.corigin.p, out_off,
                               R.cnt.p, R.pos.p);
        }
        hipLaunchKernelGGL(k_emit_final, dim3(grid(R.nc)), dim3(kBlk), 0, c.stream, R.nc, R.csplit.p, R.pos.p,
                           R.ckey.p, R.clevel.p, R.corigin.p, R.cu.p, R.cub.p, os.p.p, os.cap, nsd);
        if (q + 1 < nrounds) {
            Round &Nx = *s.rounds[q + 1];
            hipLaunchKernelGGL(k_pos_next, dim3(grid(R.nc)), dim3(kBlk), 0, c.stream, R.nc, R.csplit.p, R.crank.p,
                               R.pos.p, Nx.cnt.p, Nx.pos.p);
        }
        OTF_LAUNCH_CHECK("cascade emission");
    }
    // adjacency: a kept leaf next to a change is searched again
    const int64_t n_long = (int64_t)os.n_heavy_p + os.n_heavy_m;
    const int64_t mlb = cdiv(64 * n_long, kBlk);
    hipLaunchKernelGGL(k_nbr_mark, dim3((unsigned)(mlb + gL)), dim3(kBlk), 0, c.stream, L, os.flag.p, jt,
                       n_split > 0 ? 1 : 0, os.nbp_off.p, os.nbp.p, os.nbm_off.p, os.nbm.p, os.heavy_p.p, os.heavy_m.p,
                       (uint32_t)os.n_heavy_p, (uint32_t)os.n_heavy_m, (uint32_t)mlb, out_off, ns.need.p);
    OTF_LAUNCH_CHECK("k_nbr_mark");
    if (Lnew < 0) take_counts();
    if (jt) c.last_joins = c.h_counters[13];
    c.last_splits = total_splits;

    // ---- observations of the new leaves (append to the pool, or compact)
    DBuf<uint32_t> &nrank = s.r_nrank, &tidx = s.r_tidx, &moff = s.r_moff;
    // the new leaves (tidx, their number at nrank[0]) and the leaves whose
    // adjacency is searched again (the adjacency pass's list, its length at
    // e[0]), listed by one compacting scan of the two flag arrays
    nrank.reserve(1);
    s.e.reserve(1);
    s.dirty.reserve(Lnew);
    tidx.reserve(n_new);
    // cleared first, so that every entry is a valid leaf index even if the
    // two counts of new leaves were to disagree (checked below)
    hipLaunchKernelGGL(k_zero_u32, dim3(grid(n_new)), dim3(kBlk), 0, c.stream, (int64_t)n_new, tidx.p);
    scan_compact_pair_u8(c, isnew.p, tidx.p, n_new, nrank.p, ns.need.p, s.dirty.p, (uint32_t)Lnew, s.e.p, Lnew);
    // one fetch pass: sorted observations into rows of n_views (headers
    // written into the new store), placed into the pool once its offsets are
    // known. It runs on the second stream, beside the new store's adjacency
    // search on this one: the search reads keys, levels and marks, the fetch
    // writes observation headers, rows, their offsets and the observation
    // totals, and neither runs a scan while the other does (they share the
    // scan state). Joined before the pool is written.
    DBuf<uint8_t> &Mt = s.r_Mt;
    Mt.reserve(n_new);
    const int stride = c.n_views;
    s.fa.reserve((size_t)n_new * stride);
    s.fb.reserve((size_t)n_new * stride);
    s.fe.reserve((size_t)n_new * stride);
    moff.reserve(n_new + 1);
    ObsPool &pool = c.op();
    // the new store becomes current; its observation totals (the live
    // observations among them) are counted with the fetch
    c.cur ^= 1;
    c.L = Lnew;
    OTF_HIP(hipEventRecord(c.ev_fork, c.stream));
    OTF_HIP(hipStreamWaitEvent(c.side, c.ev_fork, 0));
    uint32_t t_obs;
    {
        OnSideStream on_side(c);
        gather_rows(c, n_new, ns.key.p, ns.level.p, tidx.p, stride, s.fa.p, s.fb.p, s.fe.p, Mt.p, ns.obs_m.p,
                    ns.obs_unit.p, ns.inv.p, ns.wtot.p);
        scan_exclusive_u32_dev_u8(c, Mt.p, moff.p, n_new);
        count_obs(c);
        t_obs = read_back_begin_side(c, {{moff.p + n_new, 19}, {c.counters.p + 4, 20}, {nrank.p, 21}});
        OTF_HIP(hipEventRecord(c.ev_join, c.side));
    }
    NbrPending nbr = build_neighbours_begin(c, os, out_off, true);
    read_back_wait_side(c, t_obs);
    OTF_HIP(hipStreamWaitEvent(c.stream, c.ev_join, 0));
    const uint32_t new_obs = c.h_counters[19], live = c.h_counters[20];
    if (c.h_counters[21] != n_new) fail(OTF_E_DEVICE, "new-leaf counts disagree");
    const bool compact = (pool.used + (int64_t)new_obs > pool.cap) || (pool.used > 2 * (int64_t)live + 4096);
    if (!compact) {
        hipLaunchKernelGGL(k_place_obs, dim3(grid(64 * (int64_t)n_new)), dim3(kBlk), 0, c.stream, (int64_t)n_new,
                           tidx.p, Mt.p, stride, s.fa.p, s.fb.p, s.fe.p, moff.p, (const uint32_t *)nullptr,
                           (uint32_t)pool.used, pool.F.p, pool.W.p, pool.P.p, ns.obs_off.p);
        OTF_LAUNCH_CHECK("k_place_obs");
        pool.used += new_obs;
    } else {
        ObsPool &np = c.obs[c.ocur ^ 1];
        np.reserve((int64_t)live + live / 4 + 1024);
        DBuf<uint32_t> &loff = s.r_loff;  // segment offsets in the compacted pool
        loff.reserve(Lnew + 1);
        scan_exclusive_u32_dev_u8(c, ns.obs_m.p, loff.p, Lnew);
        hipLaunchKernelGGL(k_copy_segments, dim3(grid(Lnew)), dim3(kBlk), 0, c.stream, Lnew, isnew.p,
                           ns.obs_m.p, loff.p, ns.obs_off.p, pool.F.p, pool.W.p, pool.P.p, np.F.p, np.W.p, np.P.p);
        OTF_LAUNCH_CHECK("k_copy_segments");
        hipLaunchKernelGGL(k_place_obs, dim3(grid(64 * (int64_t)n_new)), dim3(kBlk), 0, c.stream, (int64_t)n_new,
                           tidx.p, Mt.p, stride, s.fa.p, s.fb.p, s.fe.p, (const uint32_t *)nullptr, loff.p, 0u,
                           np.F.p, np.W.p, np.P.p, ns.obs_off.p);
        OTF_LAUNCH_CHECK("k_place_obs");
        np.used = live;
        c.ocur ^= 1;
        ++c.pool_compactions;
        OTF_HIP(hipStreamSynchronize(c.stream));
    }
    build_neighbours_end(c, nbr, nullptr);
    return true;
}

}  // namespace otf
