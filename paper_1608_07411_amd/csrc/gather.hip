// Data fetch of Fig. 4: for a fused-octree node at level L and every view,
// the view's stored node at level L, else the deepest view leaf containing it;
// F = sum/count, W = count/volume, W = 0 dropped. The observations of a node
// are sorted by (F, view) with the prefix weights and the normaliser
// 1/(sum W + gamma) of Eq. 5.
//
// One segment of SEG lanes (a power of two >= n_views) per target node: lane j
// descends view j's octree; the segment sorts by rank (each lane counts the
// lanes ordered before it) and the sequential sums are formed in rank order.
#include <algorithm>

#include "otf_internal.h"

namespace otf {
namespace {

constexpr int kBlk = 256;

struct GatherOut {
    const uint32_t *tidx;  // target t is leaf tidx[t] (key, level, header), or null: leaf t
    const uint32_t *off;   // per-target segment offset (+ base), or null: t * stride
    uint32_t base;
    int stride;
    float *F, *W, *P;  // P may be null
    uint8_t *Mcount;     // count mode: M per target t
    uint8_t *M, *unit;
    float *inv, *wtot, *u0;
    uint32_t *off_out;  // fill mode: segment offset written into the header, or null
};

template <int SEG>
__global__ void __launch_bounds__(kBlk) k_gather(ViewDev vd, int64_t n, const uint32_t *__restrict__ tkey,
                                                 const uint8_t *__restrict__ tlevel, GatherOut o, float gamma,
                                                 int count_only) {
    __shared__ float sF[kBlk], sW[kBlk];
    const int tid = threadIdx.x;
    const int64_t t = ((int64_t)blockIdx.x * kBlk + tid) / SEG;
    const int j = tid % SEG;
    const int lane = tid & 63;
    const int seg_lane0 = lane - j;
    const int seg_tid0 = tid - j;
    bool valid = false;
    float f = 0.0f, w = 0.0f;
    const int64_t h = (t < n && o.tidx) ? (int64_t)o.tidx[t] : t;
    if (t < n && j < vd.n_views) {
        const int D = vd.max_depth;
        const uint32_t key = tkey[h];
        const int L = tlevel[h];
        uint32_t node, l;
        const bool fine = vd.table && L >= vd.table_level;
        if (fine || (vd.table_c && L >= vd.table_c_level)) {  // start at a dense index
            const uint32_t *tab = fine ? vd.table : vd.table_c;
            const int T = fine ? vd.table_level : vd.table_c_level;
            const uint32_t e = tab[(size_t)(key >> (3 * (D - T))) * (uint32_t)vd.n_views + (uint32_t)j];
            node = e & ((1u << kTableIdxBits) - 1u);
            l = e >> kTableIdxBits;
        } else {
            node = vd.root[j];
            l = 0;
        }
        while ((int)l < L) {
            const uint32_t ch = vd.child[node];
            if (ch == kNone) break;
            node = ch + ((key >> (3 * (D - l - 1))) & 7u);
            ++l;
        }
        const uint32_t cn = vd.cnt[node];
        if (cn > 0u) {
            valid = true;
            f = vd.S[node] / (float)cn;
            w = ldexpf((float)cn, -3 * (D - l));
        }
    }
    const uint64_t ballot = __ballot(valid);
    const uint64_t segmask = (SEG == 64) ? ~0ull : (((1ull << SEG) - 1ull) << seg_lane0);
    const int m = __popcll(ballot & segmask);
    if (o.Mcount && t < n && j == 0) o.Mcount[t] = (uint8_t)m;
    if (count_only) return;
    int rank = 0;
#pragma unroll
    for (int i = 0; i < SEG; ++i) {
        const float fi = __shfl(f, seg_lane0 + i, 64);
        const bool vi = (ballot >> (seg_lane0 + i)) & 1ull;
        if (vi && (fi < f || (fi == f && i < j))) ++rank;
    }
    if (valid) {
        sF[seg_tid0 + rank] = f;
        sW[seg_tid0 + rank] = w;
    }
    __syncthreads();
    if (t >= n) return;
    const uint32_t off = o.base + (o.off ? o.off[t] : (uint32_t)(t * o.stride));
    if (valid) {
        o.F[off + rank] = f;
        o.W[off + rank] = w;
    }
    float P = 0.0f, acc = 0.0f;
    bool all1 = true;
    if constexpr (SEG == 64) {
        // the segment is the wave: every lane forms the same serial sums from
        // the sorted entries broadcast one at a time, and lane k keeps the
        // prefix before entry k (one coalesced store instead of m one-lane
        // stores); the order of operations is that of the serial loop below
        const float wj = sW[seg_tid0 + j], fj = sF[seg_tid0 + j];  // entry j (unused for j >= m)
        float Pj = 0.0f;
        for (int k = 0; k < m; ++k) {
            const float wk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(wj), k));
            const float fk = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(fj), k));
            Pj = (j == k) ? P : Pj;
            P = P + wk;
            acc = __fmaf_rn(wk, fk, acc);
            all1 = all1 && (wk == 1.0f);
        }
        if (o.P && j < m) o.P[off + j] = Pj;
    } else if (j == 0) {
        for (int k = 0; k < m; ++k) {
            const float wk = sW[seg_tid0 + k];
            if (o.P) o.P[off + k] = P;
            P = P + wk;
            acc = __fmaf_rn(wk, sF[seg_tid0 + k], acc);
            all1 = all1 && (wk == 1.0f);
        }
    }
    if (j == 0) {
        const float inv = 1.0f / (P + gamma);
        o.M[h] = (uint8_t)m;
        o.unit[h] = all1 ? 1 : 0;
        o.inv[h] = inv;
        o.wtot[h] = P;
        if (o.u0) o.u0[h] = acc * inv;
        if (o.off_out) o.off_out[h] = off;
    }
}

template <int SEG>
void launch_seg(Ctx &c, int64_t n, const uint32_t *tkey, const uint8_t *tlevel, const GatherOut &o, bool count_only) {
    const int64_t threads = n * SEG;
    hipLaunchKernelGGL((k_gather<SEG>), dim3((unsigned)cdiv(threads, kBlk)), dim3(kBlk), 0, c.stream, c.view_dev(), n,
                       tkey, tlevel, o, c.prm.gamma, count_only ? 1 : 0);
    OTF_LAUNCH_CHECK("k_gather");
}

void gather_launch(Ctx &c, int64_t n, const uint32_t *tkey, const uint8_t *tlevel, const GatherOut &o,
                   bool count_only);

}  // namespace

void gather_count(Ctx &c, int64_t n, const uint32_t *tkey, const uint8_t *tlevel, const uint32_t *tidx,
                  uint8_t *Mcount) {
    if (n <= 0) return;
    GatherOut o{tidx,    nullptr, 0,       0,       nullptr, nullptr, nullptr,
                Mcount,  nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    gather_launch(c, n, tkey, tlevel, o, true);
}

void gather_fill(Ctx &c, int64_t n, const uint32_t *tkey, const uint8_t *tlevel, const uint32_t *tidx,
                 const uint32_t *out_off, uint32_t base, int stride, float *F, float *W, float *P, uint8_t *M,
                 uint8_t *unit, float *inv, float *wtot, float *u0, uint32_t *off_out) {
    if (n <= 0) return;
    GatherOut o{tidx, out_off, base, stride, F, W, P, nullptr, M, unit, inv, wtot, u0, off_out};
    gather_launch(c, n, tkey, tlevel, o, false);
}

void gather_rows(Ctx &c, int64_t n, const uint32_t *tkey, const uint8_t *tlevel, const uint32_t *tidx, int stride,
                 float *F, float *W, float *P, uint8_t *Mt, uint8_t *M, uint8_t *unit, float *inv, float *wtot) {
    if (n <= 0) return;
    GatherOut o{tidx, nullptr, 0, stride, F, W, P, Mt, M, unit, inv, wtot, nullptr, nullptr};
    gather_launch(c, n, tkey, tlevel, o, false);
}

namespace {
void gather_launch(Ctx &c, int64_t n, const uint32_t *tkey, const uint8_t *tlevel, const GatherOut &o,
                   bool count_only) {
    const int nv = c.n_views;
    if (nv <= 1) launch_seg<1>(c, n, tkey, tlevel, o, count_only);
    else if (nv <= 2) launch_seg<2>(c, n, tkey, tlevel, o, count_only);
    else if (nv <= 4) launch_seg<4>(c, n, tkey, tlevel, o, count_only);
    else if (nv <= 8) launch_seg<8>(c, n, tkey, tlevel, o, count_only);
    else if (nv <= 16) launch_seg<16>(c, n, tkey, tlevel, o, count_only);
    else if (nv <= 32) launch_seg<32>(c, n, tkey, tlevel, o, count_only);
    else launch_seg<64>(c, n, tkey, tlevel, o, count_only);
}
}  // namespace

namespace {
constexpr int kObsBlocks = 1024;

// Per-block observation totals (all leaves, leaves with fractional weights);
// each thread reads 16 bytes of counts and flags at a time.
__global__ void __launch_bounds__(kBlk) k_obs_sizes(int64_t L, const uint8_t *M, const uint8_t *unit,
                                                    uint32_t *part) {
    __shared__ uint32_t st[kBlk], sn[kBlk];
    uint32_t m = 0, nu = 0;
    const int64_t nvec = L / 16;  // whole 16-byte groups (the arrays are 256-byte aligned)
    for (int64_t g = (int64_t)blockIdx.x * kBlk + threadIdx.x; g < nvec; g += (int64_t)gridDim.x * kBlk) {
        const uint4 mv = reinterpret_cast<const uint4 *>(M)[g];
        const uint4 uv = reinterpret_cast<const uint4 *>(unit)[g];
        const uint32_t mw[4] = {mv.x, mv.y, mv.z, mv.w}, uw[4] = {uv.x, uv.y, uv.z, uv.w};
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            const uint32_t mi = (mw[k >> 2] >> (8 * (k & 3))) & 0xFFu;
            m += mi;
            nu += ((uw[k >> 2] >> (8 * (k & 3))) & 0xFFu) ? 0u : mi;
        }
    }
    for (int64_t i = 16 * nvec + (int64_t)blockIdx.x * kBlk + threadIdx.x; i < L; i += (int64_t)gridDim.x * kBlk) {
        const uint32_t mi = M[i];
        m += mi;
        nu += unit[i] ? 0u : mi;
    }
    st[threadIdx.x] = m;
    sn[threadIdx.x] = nu;
    __syncthreads();
    for (int s = kBlk / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) {
            st[threadIdx.x] += st[threadIdx.x + s];
            sn[threadIdx.x] += sn[threadIdx.x + s];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[blockIdx.x] = st[0];
        part[kObsBlocks + blockIdx.x] = sn[0];
    }
}

// The two totals as u64 (one block of kObsBlocks threads).
__global__ void __launch_bounds__(kObsBlocks) k_obs_total(const uint32_t *part, int nblocks,
                                                          unsigned long long *out) {
    __shared__ unsigned long long red[2][kObsBlocks / 64];
    const int t = threadIdx.x, lane = t & 63, wid = t >> 6;
    unsigned long long a = t < nblocks ? part[t] : 0ull, b = t < nblocks ? part[kObsBlocks + t] : 0ull;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, 64);
        b += __shfl_xor(b, off, 64);
    }
    if (lane == 0) {
        red[0][wid] = a;
        red[1][wid] = b;
    }
    __syncthreads();
    if (t < 2) {
        unsigned long long s = 0;
        for (int w = 0; w < kObsBlocks / 64; ++w) s += red[t][w];
        out[t] = s;
    }
}
}  // namespace

// Totals of observations (all leaves, and leaves with fractional weights),
// left in the device counters.
void count_obs(Ctx &c) {
    unsigned long long *d = reinterpret_cast<unsigned long long *>(c.counters.p + 4);
    const int64_t blocks = std::min<int64_t>(kObsBlocks, cdiv(c.L > 0 ? c.L : 1, kBlk));
    c.s.part.reserve(2 * kObsBlocks);
    hipLaunchKernelGGL(k_obs_sizes, dim3((unsigned)blocks), dim3(kBlk), 0, c.stream, c.L, c.lv().obs_m.p,
                       c.lv().obs_unit.p, c.s.part.p);
    hipLaunchKernelGGL(k_obs_total, dim3(1), dim3(kObsBlocks), 0, c.stream, c.s.part.p, (int)blocks, d);
    OTF_LAUNCH_CHECK("k_obs_sizes");
}

namespace {
// counters [16..17] += [4..5] + [6..7] (observations read, plus the prefix
// weights of leaves with fractional weights), or + 2 [4..5] when every
// observation's weight is read (gradient descent)
__global__ void k_accum_obs(unsigned long long *c, int all_weights) {
    if (threadIdx.x == 0) c[6] += c[0] + (all_weights ? c[0] : c[1]);
}
}  // namespace

void accumulate_obs(Ctx &c, bool all_weights) {
    hipLaunchKernelGGL(k_accum_obs, dim3(1), dim3(64), 0, c.stream,
                       reinterpret_cast<unsigned long long *>(c.counters.p + 4), all_weights ? 1 : 0);
}

namespace {
// Dense index: thread t = cell * n_views + view descends the view's octree
// towards the level-T cell and records where it stops.
__global__ void k_view_table(ViewDev vd, int T, int64_t n, uint32_t *table) {
    const int64_t t = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    if (t >= n) return;
    const uint64_t cell = (uint64_t)(t / vd.n_views);
    const int j = (int)(t % vd.n_views);
    uint32_t node = vd.root[j];
    int l = 0;
    while (l < T) {
        const uint32_t ch = vd.child[node];
        if (ch == kNone) break;
        node = ch + (uint32_t)((cell >> (3 * (T - l - 1))) & 7u);
        ++l;
    }
    table[t] = ((uint32_t)l << kTableIdxBits) | node;
}
constexpr int kTableLevel = 6;        // 8^6 cells x up to 64 views x 4 bytes = 64 MiB
constexpr int kTableLevelCoarse = 3;  // 512 cells x up to 64 views
}  // namespace

void build_view_table(Ctx &c) {
    ViewStore &vs = c.views;
    vs.table_level = vs.table_c_level = -1;
    if (vs.n_nodes >= (int64_t(1) << kTableIdxBits) || c.n_views <= 0) return;  // indices do not fit: no index
    const int T = std::min(c.prm.max_depth, kTableLevel);
    const int64_t n = (int64_t(1) << (3 * T)) * c.n_views;
    vs.table.reserve(n);
    hipLaunchKernelGGL(k_view_table, dim3((unsigned)cdiv(n, kBlk)), dim3(kBlk), 0, c.stream, c.view_dev(), T, n,
                       vs.table.p);
    OTF_LAUNCH_CHECK("k_view_table");
    if (T > kTableLevelCoarse) {  // a coarser index for targets above the fine one
        const int Tc = kTableLevelCoarse;
        const int64_t nc = (int64_t(1) << (3 * Tc)) * c.n_views;
        vs.table_c.reserve(nc);
        hipLaunchKernelGGL(k_view_table, dim3((unsigned)cdiv(nc, kBlk)), dim3(kBlk), 0, c.stream, c.view_dev(), Tc,
                           nc, vs.table_c.p);
        OTF_LAUNCH_CHECK("k_view_table");
        vs.table_c_level = Tc;
    }
    vs.table_level = T;
}

// Observation pool for every leaf of the current store, in leaf order.
void gather_all_leaves(Ctx &c, bool init_values) {
    LeafStore &s = c.lv();
    gather_count(c, c.L, s.key.p, s.level.p, nullptr, s.obs_m.p);
    const uint32_t total = scan_exclusive_u8(c, s.obs_m.p, s.obs_off.p, c.L);
    c.ocur = 0;
    c.op().reserve(total + total / 4 + 1024);  // headroom for observations of new leaves
    c.op().used = total;
    gather_fill(c, c.L, s.key.p, s.level.p, nullptr, s.obs_off.p, 0, 0, c.op().F.p, c.op().W.p, c.op().P.p, s.obs_m.p,
                s.obs_unit.p, s.inv.p, s.wtot.p, init_values ? s.u.p : nullptr, nullptr);
}

}  // namespace otf
