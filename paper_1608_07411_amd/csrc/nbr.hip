// Face adjacency of the fused octree (the neighbourhood of the forward and
// backward differences, Sec. 3.2 and Fig. 5) on the Morton-sorted leaf array.
// Entries: neighbour index | direction << 26 | neighbour level << 28.
// + list (faces +x,+y,+z) feeds the gradient, - list (-x,-y,-z) the divergence;
// within a face the neighbours are in ascending key (= index) order.
//
// For a leaf n and a face, the same-size cell across the face is located by a
// binary search for the leaf containing its minimum corner. If that leaf is at
// least as large as n it is the only neighbour. Otherwise the cell is a union
// of smaller leaves, contiguous in the array from that leaf up to the first key
// past the cell; the neighbours are those of them lying on the shared face.
// A short range is scanned by the leaf's own thread; a long one (a large leaf
// next to a finely split region) is cut into chunks, each scanned by one wave
// 64 leaves at a time, the hits placed with a ballot and prefix popcounts.
//
// After a restructure only leaves that are new or touch a changed leaf are
// searched: a kept leaf whose neighbours were all kept has the same neighbours
// as before (the space next to its faces is covered by the same leaves), so
// its lists are copied with indices mapped to the new positions; the mapping
// is monotone, so the order is preserved.
#include <algorithm>

#include "otf_internal.h"

namespace otf {
namespace {

constexpr int kBlk = 256;
constexpr uint32_t kLight = 32;  // longest range scanned by a single thread

// (zero, when given: a counter cleared for the count pass that follows)
__global__ void k_key_table(const uint32_t *key, int64_t L, int shift, uint32_t nb, uint32_t *table,
                            uint32_t *zero) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (zero && b == 0) *zero = 0u;
    if (b < nb) table[b] = (uint32_t)find_leaf(key, L, b << shift);
}

// The same table from a coarser one (tc: buckets of kKeyCoarse fine buckets,
// nbc entries): each fine bucket searches only between two coarse entries.
constexpr int kKeyCoarseShift = 6;
constexpr uint32_t kKeyCoarse = 1u << kKeyCoarseShift;

__global__ void k_key_table_fine(const uint32_t *key, int64_t L, int shift, uint32_t nb, const uint32_t *tc,
                                 uint32_t nbc, uint32_t *table) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const uint32_t bc = b / kKeyCoarse;
    const uint32_t k = b << shift;
    int64_t lo = tc[bc];
    int64_t hi = (bc + 1 < nbc) ? (int64_t)tc[bc + 1] + 1 : L;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (key[mid] <= k) lo = mid;
        else hi = mid;
    }
    table[b] = (uint32_t)lo;
}

// The table of a restructured store from the previous store's table (in
// place): bucket b's old containing leaf j was emitted at remap[j] (its first
// child if split, the collapsed leaf if it headed a collapse) or removed (an
// absorbed leaf: the collapsed leaf is the last one emitted before it), and
// the old leaf after j starts beyond the bucket's first key, so the new
// containing leaf lies in [remap[j] - 1, remap[j + 1]) (remap[L_old] = L):
// a search of one or two steps for an unchanged leaf.
__global__ void k_key_table_remap(const uint32_t *key, int shift, uint32_t nb, const uint32_t *remap,
                                  uint32_t *table, uint32_t *zero) {
    const uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (zero && b == 0) *zero = 0u;
    if (b >= nb) return;
    const uint32_t j = table[b], k = b << shift;
    const uint32_t r = remap[j];
    int64_t lo = r > 0 ? (int64_t)r - 1 : 0;
    int64_t hi = remap[j + 1];
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (key[mid] <= k) lo = mid;
        else hi = mid;
    }
    table[b] = (uint32_t)lo;
}

// first i with key[i] >= k (k may be the end of the domain)
__device__ inline int64_t lower_bound(const KeyIndex &ki, uint64_t k, uint64_t domain) {
    if (k >= domain) return ki.L;
    return find_leaf(ki, (uint32_t)(k - 1)) + 1;
}

struct Face {
    bool inside;     // the face is not on the domain boundary
    bool single;     // one neighbour, at least as large: index j
    int64_t j, hi;   // otherwise the cell's leaves are [j, hi)
    uint32_t plane;  // coordinate of the shared face along d
};

__device__ inline Face locate(const KeyIndex &ki, const uint8_t *__restrict__ level, int D, const uint32_t xyz[3],
                              int ln, int face) {
    Face f{false, false, 0, 0, 0};
    const uint32_t G = 1u << D, s = 1u << (D - ln);
    const int d = face % 3;
    uint32_t q[3] = {xyz[0], xyz[1], xyz[2]};
    if (face < 3) {
        if (q[d] + s >= G) return f;
        q[d] += s;
        f.plane = q[d];
    } else {
        if (q[d] == 0) return f;
        q[d] -= s;
        f.plane = xyz[d];
    }
    f.inside = true;
    const uint32_t kq = morton3(q[0], q[1], q[2]);
    f.j = find_leaf(ki, kq);
    if (level[f.j] <= ln) {
        f.single = true;
        return f;
    }
    f.hi = lower_bound(ki, (uint64_t)kq + (uint64_t(1) << (3 * (D - ln))), uint64_t(1) << (3 * D));
    return f;
}

// Leaf m (inside the cell across `face`) lies on the shared face.
__device__ inline bool on_face(uint32_t km, int lm, int D, int face, uint32_t plane) {
    const int d = face % 3;
    const uint32_t c = compact1by2(km >> d);
    return face < 3 ? (c == plane) : (c + (1u << (D - lm)) == plane);
}

__device__ inline uint32_t entry(int64_t j, int face, int lj) {
    return (uint32_t)j | ((uint32_t)(face % 3) << kIdxBits) | ((uint32_t)lj << (kIdxBits + 2));
}

struct Heavy {
    uint32_t *leaf;
    uint8_t *face;
    uint32_t *lo, *hi;
    uint32_t *count;  // device counter
    uint32_t cap;
};

// Unchanged leaves take their counts from the previous store; the others are
// listed, in index order, at their rank dpos[i] among the leaves to search.
// Two leaves per thread (i and i + kBlk of the block's 2 kBlk): the need
// marks and sources of both are loaded, then the four old offsets of both.
constexpr int kCleanLeaves = 2;

__global__ void __launch_bounds__(kBlk) k_nbr_count_clean(int64_t L, uint32_t *cnt_p, uint32_t *cnt_m, NbrOld old) {
    constexpr int N = kCleanLeaves;
    int64_t idx[N];
    bool clean[N];
    uint32_t j[N];
#pragma unroll
    for (int n = 0; n < N; ++n) {
        idx[n] = ((int64_t)blockIdx.x * N + n) * kBlk + threadIdx.x;
        const bool in = idx[n] < L;
        const bool need = in && old.need[idx[n]];
        clean[n] = in && !need;
        j[n] = clean[n] ? old.src[idx[n]] : 0u;
    }
    uint32_t p0[N], p1[N], m0[N], m1[N];
#pragma unroll
    for (int n = 0; n < N; ++n) {
        p0[n] = old.off_p[j[n]];
        p1[n] = old.off_p[j[n] + 1];
        m0[n] = old.off_m[j[n]];
        m1[n] = old.off_m[j[n] + 1];
    }
#pragma unroll
    for (int n = 0; n < N; ++n)
        if (clean[n]) {
            cnt_p[idx[n]] = p1[n] - p0[n];
            cnt_m[idx[n]] = m1[n] - m0[n];
        }
}

// Searched leaves, 8 lanes per leaf (lane f < 6 takes face f), grid-stride
// over the n leaves of the list (all leaves when dirty is null; n is read from
// n_dev when given).
// The located face of list item q is kept for the fill pass: cj[6q + face] =
// the first leaf, cm[6q + face] = 0 for a single neighbour, else the mask of
// the range's leaves that touch the face (ranges of at most kLight leaves);
// cj = kNone for a face without such a neighbour set (none, or a long range,
// whose count the chunk kernels fill in later).
__global__ void __launch_bounds__(kBlk) k_nbr_count(KeyIndex ki, const uint8_t *__restrict__ level, int D,
                                                    uint32_t *cnt_p, uint32_t *cnt_m, uint32_t *fc,
                                                    const uint32_t *dirty, const uint32_t *n_dev, int64_t n_host,
                                                    Heavy hv, uint32_t *cj, uint32_t *cm, uint32_t *zero2) {
    if (blockIdx.x == 0 && threadIdx.x < 2) zero2[threadIdx.x] = 0u;  // k_heavy_lists' counters
    const uint32_t *__restrict__ key = ki.key;
    const int64_t n = n_dev ? (int64_t)*n_dev : n_host;
    const int face = threadIdx.x & 7;
    const int64_t stride = ((int64_t)gridDim.x * kBlk) >> 3;
    for (int64_t q = ((int64_t)blockIdx.x * kBlk + threadIdx.x) >> 3; q < n; q += stride) {
        const int64_t i = dirty ? (int64_t)dirty[q] : q;
        uint32_t nf = 0;
        if (face < 6) {
            const int ln = level[i];
            uint32_t xyz[3];
            demorton3(key[i], xyz[0], xyz[1], xyz[2]);
            const Face f = locate(ki, level, D, xyz, ln, face);
            uint32_t jo = kNone, mo = 0u;
            if (f.inside) {
                if (f.single) {
                    nf = 1;
                    jo = (uint32_t)f.j;
                } else if ((uint64_t)(f.hi - f.j) <= kLight) {
                    uint32_t mask = 0;
                    for (int64_t m = f.j; m < f.hi; ++m)
                        if (on_face(key[m], level[m], D, face, f.plane)) mask |= 1u << (uint32_t)(m - f.j);
                    nf = (uint32_t)__popc(mask);
                    jo = mask ? (uint32_t)f.j : kNone;  // (a cell's face is always covered: mask != 0)
                    mo = mask;
                } else {
                    const uint32_t slot = atomicAdd(hv.count, 1u);  // rare: a large leaf by a fine region
                    if (slot < hv.cap) {
                        hv.leaf[slot] = (uint32_t)i;
                        hv.face[slot] = (uint8_t)face;
                        hv.lo[slot] = (uint32_t)f.j;
                        hv.hi[slot] = (uint32_t)f.hi;
                    }
                }
            }
            fc[6 * i + face] = nf;  // long ranges are counted by the chunk kernels
            cj[6 * q + face] = jo;
            cm[6 * q + face] = mo;
        }
        uint32_t sp = face < 3 ? nf : 0u, sm = face < 3 ? 0u : nf;
#pragma unroll
        for (int o = 1; o < 8; o <<= 1) {
            sp += (uint32_t)__shfl_xor((int)sp, o, 64);
            sm += (uint32_t)__shfl_xor((int)sm, o, 64);
        }
        if (face == 0) {
            cnt_p[i] = sp;
            cnt_m[i] = sm;
        }
    }
}

// Long ranges are cut into chunks of kChunk leaves, one wave per chunk.
// count pass: hits per chunk. fill pass: hits written after the leaf's earlier
// faces and the item's earlier chunks, in ascending index order (ballot and
// prefix popcounts within the chunk).
constexpr uint32_t kChunk = 2048;

struct Chunks {
    const uint32_t *item;  // chunk -> heavy item
    const uint32_t *base;  // heavy item -> first chunk (n_items + 1)
    uint32_t *count;       // hits per chunk
    const uint32_t *pos;   // exclusive scan of count
};

__global__ void k_chunk_count(uint32_t n_items, Heavy hv, uint32_t *nch) {
    const uint32_t t = blockIdx.x * kBlk + threadIdx.x;
    if (t < n_items) nch[t] = (hv.hi[t] - hv.lo[t] + kChunk - 1) / kChunk;
}

// chunk -> item: one thread per chunk, the last item whose first chunk is at
// or before it (every item has at least one chunk, so base rises strictly)
__global__ void k_chunk_expand(uint32_t n_items, uint32_t n_chunks, const uint32_t *base, uint32_t *item) {
    const uint32_t c = blockIdx.x * kBlk + threadIdx.x;
    if (c >= n_chunks) return;
    uint32_t lo = 0, hi = n_items;  // base[lo] <= c < base[hi]
    while (hi - lo > 1) {
        const uint32_t m = (lo + hi) >> 1;
        if (base[m] <= c) lo = m;
        else hi = m;
    }
    item[c] = lo;
}

// One wave per chunk of a long range (block b of the chunk blocks): counts
// its hits (FILL false) or writes them after the leaf's earlier faces.
template <bool FILL>
__device__ inline void nbr_chunk(uint32_t b, uint32_t n_chunks, const Heavy &hv, const Chunks &ch,
                                 const uint32_t *__restrict__ key, const uint8_t *__restrict__ level, int D,
                                 const uint32_t *__restrict__ fc, const uint32_t *off_p, const uint32_t *off_m,
                                 uint32_t *ent_p, uint32_t *ent_m) {
    const uint32_t chunk = (b * kBlk + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (chunk >= n_chunks) return;
    const uint32_t item = ch.item[chunk];
    const uint32_t i = hv.leaf[item];
    const int face = hv.face[item];
    const int64_t lo = (int64_t)hv.lo[item] + (int64_t)(chunk - ch.base[item]) * kChunk;
    const int64_t hi = min((int64_t)hv.hi[item], lo + (int64_t)kChunk);
    const int ln = level[i];
    uint32_t xyz[3];
    demorton3(key[i], xyz[0], xyz[1], xyz[2]);
    const int d = face % 3;
    const uint32_t plane = face < 3 ? xyz[d] + (1u << (D - ln)) : xyz[d];
    uint32_t w = 0;
    if (FILL) {
        w = face < 3 ? off_p[i] : off_m[i];
        for (int f = (face < 3 ? 0 : 3); f < face; ++f) w += fc[6 * (int64_t)i + f];
        w += ch.pos[chunk] - ch.pos[ch.base[item]];
    }
    uint32_t total = 0;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int64_t b0 = lo; b0 < hi; b0 += 64) {
        const int64_t m = b0 + lane;
        bool hit = false;
        int lm = 0;
        if (m < hi) {
            lm = level[m];
            hit = on_face(key[m], lm, D, face, plane);
        }
        const uint64_t b = __ballot(hit);
        if (FILL && hit) {
            const uint32_t pos = w + total + (uint32_t)__popcll(b & below);
            if (face < 3) ent_p[pos] = entry(m, face, lm);
            else ent_m[pos] = entry(m, face, lm);
        }
        total += (uint32_t)__popcll(b);
    }
    if (!FILL && lane == 0) ch.count[chunk] = total;
}

__global__ void __launch_bounds__(kBlk) k_nbr_chunk_count(uint32_t n_chunks, Heavy hv, Chunks ch,
                                                          const uint32_t *__restrict__ key,
                                                          const uint8_t *__restrict__ level, int D) {
    nbr_chunk<false>(blockIdx.x, n_chunks, hv, ch, key, level, D, nullptr, nullptr, nullptr, nullptr, nullptr);
}

// Per heavy item: face count from its chunks, added to the leaf's list count.
__global__ void k_chunk_totals(uint32_t n_items, Heavy hv, Chunks ch, uint32_t *fc, uint32_t *cnt_p,
                               uint32_t *cnt_m) {
    const uint32_t t = blockIdx.x * kBlk + threadIdx.x;
    if (t >= n_items) return;
    const uint32_t total = ch.pos[ch.base[t + 1]] - ch.pos[ch.base[t]];
    const uint32_t i = hv.leaf[t];
    const int face = hv.face[t];
    fc[6 * (int64_t)i + face] = total;
    atomicAdd(face < 3 ? &cnt_p[i] : &cnt_m[i], total);
}

// One wave copies entries [e0, e1) of an old list to dst + (e - e0), indices
// mapped to the new positions; kCopyUnroll loads per lane in flight.
constexpr int kCopyUnroll = 8;

__device__ inline void wave_copy(const uint32_t *__restrict__ src, uint32_t e0, uint32_t e1, uint32_t *dst,
                                 const uint32_t *__restrict__ remap, int lane) {
    for (uint32_t base = e0; base < e1; base += 64 * kCopyUnroll) {
        uint32_t v[kCopyUnroll], m[kCopyUnroll];
#pragma unroll
        for (int r = 0; r < kCopyUnroll; ++r) {
            const uint32_t e = base + 64 * r + lane;
            v[r] = e < e1 ? src[e] : 0u;
        }
#pragma unroll
        for (int r = 0; r < kCopyUnroll; ++r) {
            const uint32_t e = base + 64 * r + lane;
            m[r] = e < e1 ? remap[v[r] & kIdxMask] : 0u;
        }
#pragma unroll
        for (int r = 0; r < kCopyUnroll; ++r) {
            const uint32_t e = base + 64 * r + lane;
            if (e < e1) dst[e - e0] = (v[r] & ~kIdxMask) | m[r];
        }
    }
}

// One thread copies entries [e0, e1) like wave_copy, kCopyUnroll at a time.
__device__ inline void thread_copy(const uint32_t *__restrict__ src, uint32_t e0, uint32_t e1, uint32_t *dst,
                                   const uint32_t *__restrict__ remap) {
    for (uint32_t base = e0; base < e1; base += kCopyUnroll) {
        uint32_t v[kCopyUnroll], m[kCopyUnroll];
#pragma unroll
        for (int r = 0; r < kCopyUnroll; ++r) v[r] = base + r < e1 ? src[base + r] : 0u;
#pragma unroll
        for (int r = 0; r < kCopyUnroll; ++r) m[r] = base + r < e1 ? remap[v[r] & kIdxMask] : 0u;
#pragma unroll
        for (int r = 0; r < kCopyUnroll; ++r)
            if (base + r < e1) dst[base + r - e0] = (v[r] & ~kIdxMask) | m[r];
    }
}

// Lists of unchanged leaves (block b of the short-list blocks): a wave of 64
// unchanged leaves with consecutive sources copies one contiguous block of
// entries; otherwise each unchanged leaf copies its own short lists (long
// ones are copied by nbr_copy_long).
__device__ inline void nbr_fill_clean(uint32_t b, int64_t L, const uint32_t *__restrict__ off_p,
                                      const uint32_t *__restrict__ off_m, uint32_t *ent_p, uint32_t *ent_m,
                                      const NbrOld &old) {
    const int64_t i = (int64_t)b * kBlk + threadIdx.x;
    const int lane = threadIdx.x & 63;
    const bool clean = i < L && !old.need[i];
    const uint32_t j = clean ? old.src[i] : 0u;
    const uint32_t j0 = (uint32_t)__builtin_amdgcn_readlane((int)j, 0);
    if (__ballot(clean && j == j0 + (uint32_t)lane) == ~0ull) {
        const uint32_t wp = (uint32_t)__builtin_amdgcn_readlane((int)off_p[i], 0);
        const uint32_t wm = (uint32_t)__builtin_amdgcn_readlane((int)off_m[i], 0);
        wave_copy(old.ent_p, old.off_p[j0], old.off_p[j0 + 64], ent_p + wp, old.remap, lane);
        wave_copy(old.ent_m, old.off_m[j0], old.off_m[j0 + 64], ent_m + wm, old.remap, lane);
        return;
    }
    if (!clean) return;
    const uint32_t p0 = old.off_p[j], p1 = old.off_p[j + 1];
    if (p1 - p0 <= kLongList) thread_copy(old.ent_p, p0, p1, ent_p + off_p[i], old.remap);
    const uint32_t m0 = old.off_m[j], m1 = old.off_m[j + 1];
    if (m1 - m0 <= kLongList) thread_copy(old.ent_m, m0, m1, ent_m + off_m[i], old.remap);
}

// Searched leaves, 8 lanes per leaf as in k_nbr_count (block b of nb
// striding blocks): lane f writes face f's short range after the leaf's
// earlier faces; long ranges are written by the chunk fill.
// (the faces located by k_nbr_count are read back from cj / cm)
__device__ inline void nbr_fill(uint32_t b, uint32_t nb, const uint8_t *__restrict__ level,
                                const uint32_t *__restrict__ fc, const uint32_t *__restrict__ off_p,
                                const uint32_t *__restrict__ off_m, uint32_t *ent_p, uint32_t *ent_m,
                                const uint32_t *dirty, const uint32_t *n_dev, int64_t n_host,
                                const uint32_t *__restrict__ cj, const uint32_t *__restrict__ cm) {
    const int64_t n = n_dev ? (int64_t)*n_dev : n_host;
    const int face = threadIdx.x & 7;
    if (face >= 6) return;
    const int64_t stride = ((int64_t)nb * kBlk) >> 3;
    for (int64_t q = ((int64_t)b * kBlk + threadIdx.x) >> 3; q < n; q += stride) {
        const int64_t i = dirty ? (int64_t)dirty[q] : q;
        const uint32_t j = cj[6 * q + face];
        if (j == kNone) continue;  // no neighbour, or a long range (written by the chunk fill)
        uint32_t w = face < 3 ? off_p[i] : off_m[i];
        for (int f = (face < 3 ? 0 : 3); f < face; ++f) w += fc[6 * i + f];
        uint32_t *ent = face < 3 ? ent_p : ent_m;
        uint32_t mask = cm[6 * q + face];
        if (mask == 0u) {
            ent[w] = entry(j, face, level[j]);
        } else {
            while (mask) {  // ascending index order
                const uint32_t b = (uint32_t)__ffs((int)mask) - 1u;
                mask &= mask - 1u;
                ent[w++] = entry(j + b, face, level[j + b]);
            }
        }
    }
}

// Long lists of unchanged leaves, one wave per leaf of the old long-list work
// lists (items 0..n_p-1: + lists, then - lists; block b of the long-list
// blocks); an old leaf whose new position holds another leaf, or a searched
// one, is skipped.
__device__ inline void nbr_copy_long(uint32_t b, int64_t L, const NbrOld &old, const uint32_t *off_p,
                                     const uint32_t *off_m, uint32_t *ent_p, uint32_t *ent_m) {
    const uint32_t item = (b * kBlk + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (item >= old.n_heavy_p + old.n_heavy_m) return;
    const bool plus = item < old.n_heavy_p;
    const uint32_t j = plus ? old.heavy_p[item] : old.heavy_m[item - old.n_heavy_p];
    const uint32_t i = old.remap[j];
    if ((int64_t)i >= L || old.need[i] || old.src[i] != j) return;
    if (plus) wave_copy(old.ent_p, old.off_p[j], old.off_p[j + 1], ent_p + off_p[i], old.remap, lane);
    else wave_copy(old.ent_m, old.off_m[j], old.off_m[j + 1], ent_m + off_m[i], old.remap, lane);
}

// The lists of unchanged leaves in one launch: the first long_blocks blocks
// copy the long lists (a wave each, latency-bound), the others stream the
// short ones; the two write disjoint entries.
__global__ void __launch_bounds__(kBlk) k_nbr_fill_clean(int64_t L, const uint32_t *__restrict__ off_p,
                                                         const uint32_t *__restrict__ off_m, uint32_t *ent_p,
                                                         uint32_t *ent_m, NbrOld old, uint32_t long_blocks) {
    if (blockIdx.x < long_blocks) nbr_copy_long(blockIdx.x, L, old, off_p, off_m, ent_p, ent_m);
    else nbr_fill_clean(blockIdx.x - long_blocks, L, off_p, off_m, ent_p, ent_m, old);
}

// The searched leaves' lists in one launch: the first chunk_blocks blocks
// write the long ranges (a wave per chunk), the others stride over the
// searched leaves' short ranges; the two write disjoint entries.
__global__ void __launch_bounds__(kBlk) k_nbr_fill(uint32_t chunk_blocks, uint32_t n_chunks, Heavy hv, Chunks ch,
                                                   const uint32_t *__restrict__ key, int D,
                                                   const uint8_t *__restrict__ level,
                                                   const uint32_t *__restrict__ fc, const uint32_t *__restrict__ off_p,
                                                   const uint32_t *__restrict__ off_m, uint32_t *ent_p,
                                                   uint32_t *ent_m, const uint32_t *dirty, const uint32_t *n_dev,
                                                   int64_t n_host, const uint32_t *__restrict__ cj,
                                                   const uint32_t *__restrict__ cm) {
    if (blockIdx.x < chunk_blocks)
        nbr_chunk<true>(blockIdx.x, n_chunks, hv, ch, key, level, D, fc, off_p, off_m, ent_p, ent_m);
    else
        nbr_fill(blockIdx.x - chunk_blocks, gridDim.x - chunk_blocks, level, fc, off_p, off_m, ent_p, ent_m, dirty,
                 n_dev, n_host, cj, cm);
}

__global__ void k_zero_n(uint32_t *p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

// Work lists of the leaves whose + or - list is long (order irrelevant).
__global__ void __launch_bounds__(kBlk) k_heavy_lists(int64_t L, const uint32_t *off_p, const uint32_t *off_m,
                                                      uint32_t *hp, uint32_t *hm, uint32_t *counters) {
    const int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    if (i >= L) return;
    if (off_p[i + 1] - off_p[i] > kLongList) hp[atomicAdd(&counters[0], 1u)] = (uint32_t)i;
    if (off_m[i + 1] - off_m[i] > kLongList) hm[atomicAdd(&counters[1], 1u)] = (uint32_t)i;
}


KeyIndex key_index(Ctx &c) {
    const int D = c.prm.max_depth;
    const int shift = std::max(0, 3 * D - 20);
    const uint32_t nb = 1u << (3 * D - shift);
    return KeyIndex{c.lv().key.p, c.L, c.s.key_table.p, shift, nb};
}

unsigned grid8(int64_t L) { return (unsigned)std::min<int64_t>(cdiv(8 * L, kBlk), 8192); }

// the count pass (8 lanes per searched leaf, a bounded grid strides over the
// list), with room for p.cap long ranges; starts the read-back of their number.
// The long-range counter is cleared here when `clear` (else by the key table
// launch just before); the pass clears the long-list counters of k_heavy_lists.
#ifdef OTF_DEBUG_BOUNDS
// Bounds-checked build: the lists are filled with kUnwritten before the fill
// kernels, and afterwards every slot must hold an entry of a leaf at a level
// up to D. bad[0] counts the bad slots, bad[1] keeps the smallest, bad[2] the
// value of a bad slot (of the smallest unless two race).
constexpr uint32_t kUnwritten = 0xFFFFFFFFu;
__global__ void k_adj_mark(int64_t n, uint32_t *ent, uint32_t *bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) ent[i] = kUnwritten;
    if (i == 0) {
        bad[0] = 0;
        bad[1] = 0xFFFFFFFFu;
        bad[2] = 0;
    }
}
__global__ void k_adj_check(int64_t n, const uint32_t *ent, int64_t L, int D, uint32_t *bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint32_t v = ent[i];
    if (v == kUnwritten || (int64_t)(v & kIdxMask) >= L || (int)(v >> (kIdxBits + 2)) > D) {
        atomicAdd(bad, 1u);
        if (atomicMin(bad + 1, (uint32_t)i) > (uint32_t)i) atomicExch(bad + 2, v);
    }
}
void adj_mark(Ctx &c, int64_t n, uint32_t *ent, uint32_t *bad) {
    hipLaunchKernelGGL(k_adj_mark, dim3((unsigned)cdiv(std::max<int64_t>(n, 1), kBlk)), dim3(kBlk), 0, c.stream, n,
                       ent, bad);
    OTF_LAUNCH_CHECK("k_adj_mark");
}
void adj_check(Ctx &c, const char *side, int64_t n, const uint32_t *ent, uint32_t *bad) {
    if (n > 0)
        hipLaunchKernelGGL(k_adj_check, dim3((unsigned)cdiv(n, kBlk)), dim3(kBlk), 0, c.stream, n, ent, c.L,
                           c.prm.max_depth, bad);
    OTF_LAUNCH_CHECK("k_adj_check");
    uint32_t h[3];
    OTF_HIP(hipMemcpyAsync(h, bad, sizeof h, hipMemcpyDeviceToHost, c.stream));
    OTF_HIP(hipStreamSynchronize(c.stream));
    if (h[0])
        fail(OTF_E_DEVICE, std::string("adjacency check (bounds-checked build): ") + std::to_string(h[0]) + " of " +
                               std::to_string(n) + " " + side + " slots bad, the first " + std::to_string(h[1]) +
                               (h[2] == kUnwritten ? ", written by no search" : ", one holds " + std::to_string(h[2])));
}
#endif

uint32_t count_pass(Ctx &c, NbrPending &p, bool clear) {
    LeafStore &s = c.lv();
    c.s.hv_leaf.reserve(p.cap);
    c.s.hv_lo.reserve(p.cap);
    c.s.hv_hi.reserve(p.cap);
    c.s.hv_face.reserve(p.cap);
    Heavy hv{c.s.hv_leaf.p, c.s.hv_face.p, c.s.hv_lo.p, c.s.hv_hi.p, c.counters.p + 3, p.cap};
    if (clear) hipLaunchKernelGGL(k_zero_n, dim3(1), dim3(64), 0, c.stream, c.counters.p + 3, 1);
    hipLaunchKernelGGL(k_nbr_count, dim3(grid8(c.L)), dim3(kBlk), 0, c.stream, key_index(c), s.level.p,
                       c.prm.max_depth, c.s.a.p, c.s.b.p, c.s.g.p, p.dirty, p.n_dirty_dev, c.L, hv, c.s.nb_j.p,
                       c.s.nb_m.p, c.counters.p + 14);
    OTF_LAUNCH_CHECK("k_nbr_count");
    return read_back_begin(c, {{c.counters.p + 3, 3}});
}

NbrPending search_begin(Ctx &c, const NbrOld &old, bool need_scanned) {
    LeafStore &s = c.lv();
    const int64_t L = c.L;
    const int D = c.prm.max_depth;
    const unsigned g = (unsigned)cdiv(L, kBlk);
    c.s.a.reserve(L + 1);
    c.s.b.reserve(L + 1);
    c.s.g.reserve(6 * L);
    c.s.nb_j.reserve(6 * L);
    c.s.nb_m.reserve(6 * L);
    const int shift = std::max(0, 3 * D - 20);
    const uint32_t nb = 1u << (3 * D - shift);
    if (old.remap) {  // after a restructure: the previous store's table, remapped
        hipLaunchKernelGGL(k_key_table_remap, dim3((unsigned)cdiv(nb, kBlk)), dim3(kBlk), 0, c.stream, s.key.p,
                           shift, nb, old.remap, c.s.key_table.p, c.counters.p + 3);
    } else if (nb >= 4 * kKeyCoarse) {  // coarse table first (its entries after the fine ones), then the fine one
        const uint32_t nbc = nb / kKeyCoarse;
        c.s.key_table.reserve((size_t)nb + nbc);
        uint32_t *tc = c.s.key_table.p + nb;
        hipLaunchKernelGGL(k_key_table, dim3((unsigned)cdiv(nbc, kBlk)), dim3(kBlk), 0, c.stream, s.key.p, L,
                           shift + kKeyCoarseShift, nbc, tc, c.counters.p + 3);
        hipLaunchKernelGGL(k_key_table_fine, dim3((unsigned)cdiv(nb, kBlk)), dim3(kBlk), 0, c.stream, s.key.p, L,
                           shift, nb, (const uint32_t *)tc, nbc, c.s.key_table.p);
    } else {
        c.s.key_table.reserve(nb);
        hipLaunchKernelGGL(k_key_table, dim3((unsigned)cdiv(nb, kBlk)), dim3(kBlk), 0, c.stream, s.key.p, L, shift,
                           nb, c.s.key_table.p, c.counters.p + 3);
    }
    OTF_LAUNCH_CHECK("k_key_table");
    NbrPending p{};
    p.old = old;
    p.cap = (uint32_t)std::min<int64_t>(6 * L, std::max<int64_t>(4096, L / 8));
    // leaves to search: all of them, or (after a restructure) those marked in
    // need, listed in dirty by a compacting scan; their number e[0] stays on
    // the device
    if (old.need) {
        if (!need_scanned) {
            c.s.e.reserve(1);
            c.s.dirty.reserve(L);
            scan_compact_u8(c, old.need, c.s.dirty.p, (uint32_t)L, c.s.e.p, L);
        }
        const unsigned gc = (unsigned)std::max<int64_t>(1, cdiv(L, kCleanLeaves * kBlk));
        hipLaunchKernelGGL(k_nbr_count_clean, dim3(gc), dim3(kBlk), 0, c.stream, L, c.s.a.p, c.s.b.p, old);
        OTF_LAUNCH_CHECK("k_nbr_count_clean");
        p.dirty = c.s.dirty.p;
        p.n_dirty_dev = c.s.e.p;
    }
    p.ticket = count_pass(c, p, false);
    return p;
}

// `overlap` is queued at the first wait for a count (the chunk total, else
// the list totals).
void search_end(Ctx &c, NbrPending &p, void (*overlap)(Ctx &)) {
    LeafStore &s = c.lv();
    const int64_t L = c.L;
    const int D = c.prm.max_depth;
    const unsigned g = (unsigned)cdiv(L, kBlk);
    const NbrOld &old = p.old;
    read_back_wait(c, p.ticket);
    uint32_t n_heavy = c.h_counters[3];
    if (n_heavy > p.cap) {  // rare: more long ranges than room; count again with room for all
        p.cap = n_heavy;
        read_back_wait(c, count_pass(c, p, true));
        n_heavy = c.h_counters[3];
        if (n_heavy > p.cap) fail(OTF_E_DEVICE, "long-range count changed between passes");
    }
    Heavy hv{c.s.hv_leaf.p, c.s.hv_face.p, c.s.hv_lo.p, c.s.hv_hi.p, c.counters.p + 3, p.cap};
    Chunks ch{nullptr, nullptr, nullptr, nullptr};
    uint32_t n_chunks = 0;
    if (n_heavy > 0) {
        const unsigned gi = (unsigned)cdiv(n_heavy, kBlk);
        c.s.ch_base.reserve(n_heavy + 1);
        hipLaunchKernelGGL(k_chunk_count, dim3(gi), dim3(kBlk), 0, c.stream, n_heavy, hv, c.s.ch_base.p);
        scan_exclusive_u32_dev(c, c.s.ch_base.p, c.s.ch_base.p, n_heavy);
        const uint32_t t_ch = read_back_begin(c, {{c.s.ch_base.p + n_heavy, 3}});
        if (overlap) overlap(c);
        overlap = nullptr;
        read_back_wait(c, t_ch);
        n_chunks = c.h_counters[3];
        c.s.ch_item.reserve(n_chunks);
        c.s.ch_count.reserve(n_chunks + 1);
        c.s.ch_pos.reserve(n_chunks + 1);
        ch = Chunks{c.s.ch_item.p, c.s.ch_base.p, c.s.ch_count.p, c.s.ch_pos.p};
        hipLaunchKernelGGL(k_chunk_expand, dim3((unsigned)cdiv(n_chunks, kBlk)), dim3(kBlk), 0, c.stream, n_heavy,
                           n_chunks, c.s.ch_base.p, c.s.ch_item.p);
        hipLaunchKernelGGL(k_nbr_chunk_count, dim3((unsigned)cdiv((int64_t)n_chunks * 64, kBlk)), dim3(kBlk), 0,
                           c.stream, n_chunks, hv, ch, s.key.p, s.level.p, D);
        OTF_LAUNCH_CHECK("k_nbr_chunk_count");
        scan_exclusive_u32_dev(c, c.s.ch_count.p, c.s.ch_pos.p, n_chunks);
        hipLaunchKernelGGL(k_chunk_totals, dim3(gi), dim3(kBlk), 0, c.stream, n_heavy, hv, ch, c.s.g.p, c.s.a.p,
                           c.s.b.p);
        OTF_LAUNCH_CHECK("k_chunk_totals");
    }
    scan_exclusive_pair_u32(c, c.s.a.p, s.nbp_off.p, c.s.b.p, s.nbm_off.p, L);
    // work lists of the leaves with long lists need only the offsets
    s.heavy_p.reserve(L);
    s.heavy_m.reserve(L);
    hipLaunchKernelGGL(k_heavy_lists, dim3(g), dim3(kBlk), 0, c.stream, L, (const uint32_t *)s.nbp_off.p,
                       (const uint32_t *)s.nbm_off.p, s.heavy_p.p, s.heavy_m.p, c.counters.p + 14);
    OTF_LAUNCH_CHECK("k_heavy_lists");
    const uint32_t t_tot = read_back_begin(
        c, {{s.nbp_off.p + L, 10}, {s.nbm_off.p + L, 11}, {c.counters.p + 14, 14}, {c.counters.p + 15, 15}});
    if (overlap) overlap(c);
    read_back_wait(c, t_tot);
    s.n_nbp = c.h_counters[10];
    s.n_nbm = c.h_counters[11];
    s.n_heavy_p = c.h_counters[14];
    s.n_heavy_m = c.h_counters[15];
    s.nbp.reserve(s.n_nbp);
    s.nbm.reserve(s.n_nbm);
#ifdef OTF_DEBUG_BOUNDS
    c.s.adj_bad.reserve(6);
    adj_mark(c, s.n_nbp, s.nbp.p, c.s.adj_bad.p);
    adj_mark(c, s.n_nbm, s.nbm.p, c.s.adj_bad.p + 3);
#endif
    if (old.need) {
        const int64_t n_long = (int64_t)old.n_heavy_p + old.n_heavy_m;
        const int64_t lb = cdiv(n_long * 64, kBlk);
        hipLaunchKernelGGL(k_nbr_fill_clean, dim3((unsigned)(lb + g)), dim3(kBlk), 0, c.stream, L,
                           (const uint32_t *)s.nbp_off.p, (const uint32_t *)s.nbm_off.p, s.nbp.p, s.nbm.p, old,
                           (uint32_t)lb);
        OTF_LAUNCH_CHECK("k_nbr_fill_clean");
    }
    const int64_t cb = n_heavy > 0 ? cdiv((int64_t)n_chunks * 64, kBlk) : 0;
    hipLaunchKernelGGL(k_nbr_fill, dim3((unsigned)(cb + grid8(L))), dim3(kBlk), 0, c.stream, (uint32_t)cb, n_chunks,
                       hv, ch, s.key.p, D, s.level.p, (const uint32_t *)c.s.g.p, (const uint32_t *)s.nbp_off.p,
                       (const uint32_t *)s.nbm_off.p, s.nbp.p, s.nbm.p, p.dirty, p.n_dirty_dev, L,
                       (const uint32_t *)c.s.nb_j.p, (const uint32_t *)c.s.nb_m.p);
    OTF_LAUNCH_CHECK("k_nbr_fill");
#ifdef OTF_DEBUG_BOUNDS
    if (c.debug_unwritten_slot && s.n_nbp > 0) {  // test hook: as if no search had written + slot 0
        c.debug_unwritten_slot = false;
        const uint32_t m = kUnwritten;
        OTF_HIP(hipMemcpyAsync(s.nbp.p, &m, sizeof m, hipMemcpyHostToDevice, c.stream));
        OTF_HIP(hipStreamSynchronize(c.stream));
    }
    adj_check(c, "+", s.n_nbp, s.nbp.p, c.s.adj_bad.p);
    adj_check(c, "-", s.n_nbm, s.nbm.p, c.s.adj_bad.p + 3);
#endif
}

}  // namespace

void build_neighbours(Ctx &c) {
    NbrPending p = search_begin(
        c, NbrOld{nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, 0u, 0u}, false);
    search_end(c, p, nullptr);
}

NbrPending build_neighbours_begin(Ctx &c, const LeafStore &old, const uint32_t *remap, bool need_scanned) {
    const LeafStore &s = c.lv();
    // an unchanged leaf with a long list had that list in the previous store,
    // so it is on one of the old long-list work lists
    return search_begin(c,
                        NbrOld{s.need.p, s.src.p, old.nbp_off.p, old.nbm_off.p, old.nbp.p, old.nbm.p, remap,
                               old.heavy_p.p, old.heavy_m.p, (uint32_t)old.n_heavy_p, (uint32_t)old.n_heavy_m},
                        need_scanned);
}

void build_neighbours_end(Ctx &c, NbrPending &p, void (*overlap)(Ctx &)) { search_end(c, p, overlap); }

}  // namespace otf
