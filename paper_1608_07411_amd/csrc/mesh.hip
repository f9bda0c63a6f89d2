// Evaluation on the fused octree (Sec. 3.2, the meshing step; Sec. 4, the
// quantisation error of Eq. 7):
//  - resampling of u to the finest grid (piecewise constant per leaf);
//  - marching cubes on that grid: cells between 8 finest-voxel centres, a
//    vertex on every cell edge whose end values straddle the iso-value
//    (linear interpolation), triangles from a case table built here;
//  - Eq. 7: sum over leaves of |u(n) - mean of a finest-grid field over n|.
//
// The case table is derived, not transcribed: for each of the 256 inside /
// outside corner patterns, every cube face with a sign change contributes
// segments between its crossing edges (on a face with two diagonal inside
// corners, the segments cut off the inside corners), the segments are linked
// into closed polygons through the edges they share, and each polygon is
// triangulated as a fan. Neighbouring cells see the same signs on a shared
// face, so they make the same segments there and the mesh is closed.
#include <algorithm>
#include <vector>

#include "otf_internal.h"

namespace otf {

namespace {

constexpr int kBlk = 256;
constexpr int kMaxTri = 12;

struct McCase {
    int8_t ntri;
    int8_t edge[kMaxTri * 3];
};

// corner c = x + 2y + 4z; edge id = 4 axis + (the other two coordinates,
// lower axis first, as bits)
int corner_of(int x, int y, int z) { return x | (y << 1) | (z << 2); }

int edge_between(int ca, int cb) {
    const int diff = ca ^ cb;
    const int axis = diff == 1 ? 0 : diff == 2 ? 1 : 2;
    const int lo = ca & cb;  // the endpoint with the axis coordinate 0
    const int x = lo & 1, y = (lo >> 1) & 1, z = (lo >> 2) & 1;
    const int o = axis == 0 ? (y | (z << 1)) : axis == 1 ? (x | (z << 1)) : (x | (y << 1));
    return 4 * axis + o;
}

std::vector<McCase> make_table() {
    std::vector<McCase> tab(256);
    for (int cs = 0; cs < 256; ++cs) {
        auto in = [&](int c) { return (cs >> c) & 1; };
        std::vector<std::pair<int, int>> seg;
        for (int a = 0; a < 3; ++a) {
            const int u = a == 0 ? 1 : 0, v = a == 2 ? 1 : 2;
            for (int b = 0; b < 2; ++b) {
                int cyc[4];
                const int uv[4][2] = {{0, 0}, {1, 0}, {1, 1}, {0, 1}};
                for (int k = 0; k < 4; ++k) {
                    int q[3];
                    q[a] = b;
                    q[u] = uv[k][0];
                    q[v] = uv[k][1];
                    cyc[k] = corner_of(q[0], q[1], q[2]);
                }
                int cross[4], nc = 0;
                for (int k = 0; k < 4; ++k)
                    if (in(cyc[k]) != in(cyc[(k + 1) & 3])) cross[nc++] = k;  // edge k joins corners k, k+1
                if (nc == 2) {
                    seg.push_back({edge_between(cyc[cross[0]], cyc[(cross[0] + 1) & 3]),
                                   edge_between(cyc[cross[1]], cyc[(cross[1] + 1) & 3])});
                } else if (nc == 4) {
                    for (int k = 0; k < 4; ++k)
                        if (in(cyc[k])) {  // cut off inside corner k: its edges k-1 and k
                            const int km = (k + 3) & 3;
                            seg.push_back({edge_between(cyc[km], cyc[k]), edge_between(cyc[k], cyc[(k + 1) & 3])});
                        }
                }
            }
        }
        // link the segments into closed polygons (every crossing edge lies on two faces)
        std::vector<int> used(seg.size(), 0);
        McCase &m = tab[cs];
        m.ntri = 0;
        for (size_t s0 = 0; s0 < seg.size(); ++s0) {
            if (used[s0]) continue;
            std::vector<int> poly;
            used[s0] = 1;
            poly.push_back(seg[s0].first);
            int cur = seg[s0].second;
            while (cur != poly[0]) {
                poly.push_back(cur);
                int nxt = -1;
                for (size_t s = 0; s < seg.size(); ++s) {
                    if (used[s]) continue;
                    if (seg[s].first == cur) nxt = seg[s].second;
                    else if (seg[s].second == cur) nxt = seg[s].first;
                    else continue;
                    used[s] = 1;
                    break;
                }
                if (nxt < 0) fail(OTF_E_DEVICE, "marching-cubes table: open polygon");
                cur = nxt;
            }
            for (size_t k = 1; k + 1 < poly.size(); ++k) {
                if (m.ntri >= kMaxTri) fail(OTF_E_DEVICE, "marching-cubes table: too many triangles");
                m.edge[3 * m.ntri] = (int8_t)poly[0];
                m.edge[3 * m.ntri + 1] = (int8_t)poly[k];
                m.edge[3 * m.ntri + 2] = (int8_t)poly[k + 1];
                ++m.ntri;
            }
        }
    }
    return tab;
}

// The finest grid is processed in chunks: chunk c is the cube of
// (2^cl)^3 voxels at Morton index c of its level (cl = min(D, 4)), i.e. the
// finest Morton codes [c 8^cl, (c + 1) 8^cl). Leaves are aligned cubes in
// Morton order, so a chunk either lies inside one leaf or holds a run of
// whole leaves; inside the chunk a voxel's Morton offset is morton3(dx, dy, dz).
constexpr int kChunkLevel = 4;
constexpr int kChunkMax = 1 << (3 * kChunkLevel);  // voxels of a chunk

// A block takes `pair` consecutive chunks (2 when there are several): chunks
// 2m and 2m + 1 differ in x only, so together they are a box whose rows span
// 2 ce voxels, a whole 128-byte line at the full chunk size, where a single
// chunk's rows would load and store half lines.
struct Chunking {
    int D, cl;
    uint32_t ce, cv;  // edge and voxels of a chunk
    int64_t n;        // chunks
    uint32_t pair;    // chunks per block (1 or 2)
};

constexpr int kPairBlk = 2 * kBlk;  // threads of a block: kBlk per chunk

Chunking chunking(int D) {
    const int cl = std::min(D, kChunkLevel);
    const int64_t n = int64_t(1) << (3 * (D - cl));
    return Chunking{D, cl, 1u << cl, 1u << (3 * cl), n, n > 1 ? 2u : 1u};
}

// The most voxels of a block's box per thread (pair cv / blockDim, both pair
// forms: 2 cv / 2 kBlk or cv / kBlk).
constexpr int kBoxPerThread = kChunkMax / kBlk;
constexpr int kLeafBatch = 4;  // a chunk's leaves loaded together per thread

// The block's box (rows of pair ce voxels, row-major) is walked with the
// thread's x and y fixed (the block covers whole rows and a whole number of z
// layers per step) and z stepping: fn(sub, m, g) for each of the thread's
// voxels, sub = its chunk within the pair, m = its Morton offset in that
// chunk, g = its grid index (dense[g]).
template <class F>
__device__ inline void for_box_voxels(const Chunking &ck, uint32_t c0, F fn) {
    const int lw = ck.cl + (ck.pair == 2 ? 1 : 0);  // log2 of the row length
    const uint32_t dx = threadIdx.x & ((1u << lw) - 1), row0 = threadIdx.x >> lw;
    const uint32_t dy = row0 & (ck.ce - 1), dz0 = row0 >> ck.cl, dzs = (blockDim.x >> lw) >> ck.cl;
    const uint32_t sub = dx >> ck.cl, mxy = part1by2(dx & (ck.ce - 1)) | (part1by2(dy) << 1);
    uint32_t cx, cy, cz;
    demorton3(c0, cx, cy, cz);
    const int64_t G = int64_t(1) << ck.D;
    const int64_t gxy = (int64_t)((cy << ck.cl) + dy) * G + (cx << ck.cl) + dx;
    for (uint32_t dz = dz0; dz < ck.ce; dz += dzs)
        fn(sub, mxy | (part1by2(dz) << 2), ((int64_t)(cz << ck.cl) + dz) * G * G + gxy);
}

// first[c] = the leaf containing chunk c's first voxel, first[n] = L
__global__ void k_chunk_first(KeyIndex ki, Chunking ck, uint32_t *first) {
    const int64_t c = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    if (c < ck.n) first[c] = (uint32_t)find_leaf(ki, (uint32_t)c << (3 * ck.cl));
    if (c == ck.n) first[c] = (uint32_t)ki.L;
}

// the leaves of chunk c: [i0, i1). When the chunk lies inside one leaf the
// next chunk may start in the same leaf: then i1 = i0 + 1.
__device__ inline void chunk_leaves(const uint32_t *first, uint32_t c, int64_t &i0, int64_t &i1) {
    i0 = first[c];
    i1 = max((int64_t)first[c + 1], i0 + 1);
}

// u of the leaf containing every finest voxel, dense[(z G + y) G + x]: per
// chunk, its leaves fill the chunk's Morton-ordered values in LDS, which are
// written out row by row (kBlk threads per chunk of the block's pair).
__global__ void __launch_bounds__(kPairBlk) k_dense(const uint32_t *__restrict__ key,
                                                    const uint8_t *__restrict__ level, const float *__restrict__ u,
                                                    const uint32_t *__restrict__ first, Chunking ck, float *dense) {
    __shared__ __align__(16) float val[2][kChunkMax];
    __shared__ float s_uw[2];
    __shared__ int s_whole[2];
    const uint32_t h = threadIdx.x / kBlk, lt = threadIdx.x % kBlk;
    const uint32_t c0 = blockIdx.x * ck.pair, c = c0 + h, a = c << (3 * ck.cl);
    int64_t i0, i1;
    chunk_leaves(first, c, i0, i1);
    const bool whole = i1 - i0 == 1;
    if (lt == 0) {
        s_whole[h] = whole;
        s_uw[h] = u[i0];
    }
    if (!whole) {
        // kLeafBatch leaves' loads in flight at a time (a fully refined chunk
        // gives each thread 16 leaves)
        for (int64_t ib = i0 + lt; ib < i1; ib += kLeafBatch * kBlk) {
            uint32_t kk[kLeafBatch];
            uint8_t lv[kLeafBatch];
            float uu[kLeafBatch];
#pragma unroll
            for (int q = 0; q < kLeafBatch; ++q) {
                const int64_t i = ib + q * kBlk;
                if (i < i1) {
                    kk[q] = key[i];
                    lv[q] = level[i];
                    uu[q] = u[i];
                }
            }
#pragma unroll
            for (int q = 0; q < kLeafBatch; ++q) {
                if (ib + q * kBlk >= i1) break;
                const uint32_t o = kk[q] - a, vol = 1u << (3 * (ck.D - lv[q]));
                const float v = uu[q];
                if (vol < 8) {
                    val[h][o] = v;
                } else {
                    float4 *p4 = reinterpret_cast<float4 *>(&val[h][o]);
                    for (uint32_t r = 0; r < vol / 4; ++r) p4[r] = make_float4(v, v, v, v);
                }
            }
        }
    }
    __syncthreads();
    for_box_voxels(ck, c0, [&](uint32_t sub, uint32_t m, int64_t g) {
        dense[g] = s_whole[sub] ? s_uw[sub] : val[sub][m];
    });
}

// Marching cubes, one wave per row of cells (y, z), y, z < G - 1: the lanes
// take 64 consecutive cells at a time. Each lane packs the below-iso bits of
// its voxel x in the four voxel rows (y or y + 1, z or z + 1; bit k for row
// (y + (k & 1), z + (k >> 1))); a cell's x + 1 corners are the next lane's
// pack (lane 63: the next 64 voxels' lane 0). The loads of up to kSegs
// segments of the four rows are issued together.
constexpr int kSegs = 8;

// 4 bits to the even bits of a byte
__device__ inline uint32_t spread4(uint32_t v) {
    v = (v | (v << 2)) & 0x33u;
    return (v | (v << 1)) & 0x55u;
}

// the pack of the lane's x + 1 voxel
__device__ inline uint32_t upper_pack(uint32_t pc, uint32_t pn) {
    const uint32_t up = (uint32_t)__shfl_down((int)pc, 1, 64), nx = (uint32_t)__shfl((int)pn, 0, 64);
    return (threadIdx.x & 63) < 63 ? up : nx;
}

// calls fn(x0, pc, pn, vc, vn) for the 64 cells from x0 of the row whose first
// voxel row starts at r00, every segment once, in order: pc, pn the lane's
// packs in this and the next segment, vc, vn its values of the four voxel rows
template <class F>
__device__ inline void for_row_segments(const float *__restrict__ r00, int G, float iso, F fn) {
    const int lane = threadIdx.x & 63;
    const int nseg = (G + 63) / 64;
    const int64_t GG = (int64_t)G * G;
    uint32_t ppend = 0;
    float pv[4] = {0.f, 0.f, 0.f, 0.f};
    for (int s0 = 0; s0 < nseg; s0 += kSegs) {
        float v[kSegs][4];
#pragma unroll
        for (int j = 0; j < kSegs; ++j) {
            const int x = (s0 + j) * 64 + lane;
            const int xi = x < G ? x : 0;
            v[j][0] = r00[xi];
            v[j][1] = r00[G + xi];
            v[j][2] = r00[GG + xi];
            v[j][3] = r00[GG + G + xi];
        }
        uint32_t pk[kSegs];
#pragma unroll
        for (int j = 0; j < kSegs; ++j) {
            const bool in = (s0 + j) * 64 + lane < G;
            pk[j] = in ? (uint32_t)(v[j][0] < iso) | ((uint32_t)(v[j][1] < iso) << 1) |
                             ((uint32_t)(v[j][2] < iso) << 2) | ((uint32_t)(v[j][3] < iso) << 3)
                       : 0u;
        }
        if (s0 > 0) fn((s0 - 1) * 64, ppend, pk[0], pv, v[0]);
#pragma unroll
        for (int j = 0; j + 1 < kSegs; ++j) fn((s0 + j) * 64, pk[j], pk[j + 1], v[j], v[j + 1]);
        ppend = pk[kSegs - 1];
#pragma unroll
        for (int k = 0; k < 4; ++k) pv[k] = v[kSegs - 1][k];
    }
    const float nv[4] = {0.f, 0.f, 0.f, 0.f};
    fn((((nseg + kSegs - 1) / kSegs) * kSegs - 1) * 64, ppend, 0u, pv, nv);
}

__global__ void __launch_bounds__(kBlk) k_mc_count(const float *__restrict__ dense, int D, float iso,
                                                   const McCase *__restrict__ tab, uint32_t *row_tri) {
    __shared__ uint8_t ntab[256];
    for (int i = threadIdx.x; i < 256; i += kBlk) ntab[i] = (uint8_t)tab[i].ntri;
    __syncthreads();
    const int G = 1 << D, C = G - 1;
    const int64_t row = (int64_t)blockIdx.x * (kBlk / 64) + (threadIdx.x >> 6);
    if (row >= (int64_t)C * C) return;
    const int y = (int)(row % C), z = (int)(row / C);
    const int lane = threadIdx.x & 63;
    uint32_t n = 0;
    for_row_segments(dense + ((int64_t)z * G + y) * G, G, iso,
                     [&](int x0, uint32_t pc, uint32_t pn, const float *, const float *) {
                         const uint32_t cs = spread4(pc) | (spread4(upper_pack(pc, pn)) << 1);
                         if (x0 + lane < C) n += ntab[cs];
                     });
    for (int o = 32; o > 0; o >>= 1) n += __shfl_xor(n, o, 64);
    if (lane == 0) row_tri[row] = n;
}

// triangle t of the mesh: xyz[9 t ..] its 3 vertices (world), edge[3 t ..]
// their grid edges: 3 ((z G + y) G + x) + axis of the edge's lower voxel.
// Triangles are written row by row (from the row's offset), in a row by x.
// The triangles of 64 cells are spread over the wave's lanes, one each (in
// rounds of 64), the cell of a triangle found through a per-wave list in LDS.
__global__ void __launch_bounds__(kBlk) k_mc_emit(const float *__restrict__ dense, int D, float iso,
                                                  const McCase *__restrict__ tab, const uint32_t *__restrict__ row_first,
                                                  float *xyz, unsigned long long *edge) {
    __shared__ McCase stab[256];
    __shared__ uint8_t owner[kBlk / 64][64 * kMaxTri];
    for (int i = threadIdx.x; i < (int)sizeof(stab); i += kBlk)
        reinterpret_cast<int8_t *>(stab)[i] = reinterpret_cast<const int8_t *>(tab)[i];
    __syncthreads();
    const int G = 1 << D, C = G - 1;
    const int64_t row = (int64_t)blockIdx.x * (kBlk / 64) + (threadIdx.x >> 6);
    if (row >= (int64_t)C * C) return;
    const int lane = threadIdx.x & 63;
    uint8_t *own = owner[threadIdx.x >> 6];
    const int y = (int)(row % C), z = (int)(row / C);
    const float h = ldexpf(1.0f, -D);
    uint32_t w = row_first[row];
    for_row_segments(dense + ((int64_t)z * G + y) * G, G, iso,
                     [&](int x0, uint32_t pc, uint32_t pn, const float *vc, const float *vn) {
        const uint32_t cs = spread4(pc) | (spread4(upper_pack(pc, pn)) << 1);
        const uint32_t cnt = x0 + lane < C ? (uint32_t)stab[cs].ntri : 0u;
        if (__ballot(cnt != 0) == 0) return;  // most segments: no triangle
        uint32_t incl = cnt;
        for (int o = 1; o < 64; o <<= 1) {
            const uint32_t t = __shfl_up(incl, o, 64);
            if (lane >= o) incl += t;
        }
        const uint32_t excl = incl - cnt, total = (uint32_t)__shfl((int)incl, 63, 64);
        const uint32_t w0 = w;
        w += total;
        // the cell's corner values: x from this lane, x + 1 from the next lane
        // (lane 63: the next segment's lane 0)
        float lo[4], hi[4];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const float up = __shfl_down(vc[k], 1, 64), nx = __shfl(vn[k], 0, 64);
            lo[k] = vc[k];
            hi[k] = lane < 63 ? up : nx;
        }
        for (uint32_t j = 0; j < cnt; ++j) own[excl + j] = (uint8_t)lane;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (uint32_t b = 0; b < total; b += 64) {
            const uint32_t t = b + lane;
            const int ow = t < total ? own[t] : 0;
            const uint32_t tcs = (uint32_t)__shfl((int)cs, ow, 64);
            const uint32_t tri = t - (uint32_t)__shfl((int)excl, ow, 64);
            float clo[4], chi[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                clo[k] = __shfl(lo[k], ow, 64);
                chi[k] = __shfl(hi[k], ow, 64);
            }
            if (t >= total) continue;
            auto corner = [&](int cix) {
                const int k = cix >> 1;
                const float l = k == 0 ? clo[0] : k == 1 ? clo[1] : k == 2 ? clo[2] : clo[3];
                const float u = k == 0 ? chi[0] : k == 1 ? chi[1] : k == 2 ? chi[2] : chi[3];
                return (cix & 1) ? u : l;
            };
            const int x = x0 + ow;
            const int8_t *eds = stab[tcs].edge + 3 * tri;
            const int64_t at = (int64_t)w0 + t;
            for (int jv = 0; jv < 3; ++jv) {
                const int ed = eds[jv];
                const int axis = ed >> 2, o = ed & 3;
                int d[3] = {0, 0, 0};
                const int pu = axis == 0 ? 1 : 0, pv = axis == 2 ? 1 : 2;
                d[pu] = o & 1;
                d[pv] = (o >> 1) & 1;
                const int lower = d[0] | (d[1] << 1) | (d[2] << 2);
                const float v0 = corner(lower), v1 = corner(lower | (1 << axis));
                const float tt = (iso - v0) / (v1 - v0);
                const int p[3] = {x + d[0], y + d[1], z + d[2]};
                float cc[3];
                for (int dd = 0; dd < 3; ++dd) {
                    const float base = (float)p[dd] + 0.5f;
                    cc[dd] = (dd == axis ? base + tt : base) * h;
                }
                const uint32_t q0 = ((uint32_t)p[2] * (uint32_t)G + (uint32_t)p[1]) * (uint32_t)G + (uint32_t)p[0];
                xyz[9 * at + 3 * jv] = cc[0];
                xyz[9 * at + 3 * jv + 1] = cc[1];
                xyz[9 * at + 3 * jv + 2] = cc[2];
                edge[3 * at + jv] = 3ull * (unsigned long long)q0 + (unsigned long long)axis;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    });
}

// Eq. 7 terms |u(n) - mean of dense over n|. Sums over aligned cubes form an
// octree pyramid of the field in Morton order (each node the sum of its 8
// children in Morton order, in double): a leaf's sum is the node of its own
// cube. Per chunk the pyramid up to the chunk is built in LDS and the chunk's
// leaves take their terms from it (summed per block in a fixed order); the
// chunk totals go to `csum`, the bottom of the pyramid's upper levels, where
// the leaves larger than a chunk take theirs.
__global__ void __launch_bounds__(kPairBlk) k_quant_chunk(const uint32_t *__restrict__ key,
                                                          const uint8_t *__restrict__ level,
                                                          const float *__restrict__ u,
                                                          const uint32_t *__restrict__ first, Chunking ck,
                                                          const float *__restrict__ dense, double *csum,
                                                          double *partial) {
    constexpr int kPyr = kChunkMax / 8 + kChunkMax / 64 + kChunkMax / 512 + 1;
    __shared__ __align__(16) float val[2][kChunkMax];
    __shared__ double pyr[2][kPyr];
    __shared__ double red[kPairBlk / 64];
    const uint32_t h = threadIdx.x / kBlk, lt = threadIdx.x % kBlk;
    const uint32_t c0 = blockIdx.x * ck.pair, c = c0 + h, a = c << (3 * ck.cl);
    {
        // all of the thread's loads first, then the LDS stores
        float t[kBoxPerThread];
        uint32_t at[kBoxPerThread];
        int q = 0;
        for_box_voxels(ck, c0, [&](uint32_t sub, uint32_t m, int64_t g) {
            t[q] = dense[g];
            at[q++] = sub * kChunkMax + m;
        });
        for (int j = 0; j < q; ++j) (&val[0][0])[at[j]] = t[j];
    }
    int64_t i0, i1;
    chunk_leaves(first, c, i0, i1);
    __syncthreads();
    // level 1 (cubes of 8) from the values, then each level from the one below
    uint32_t base[kChunkLevel + 1];
    base[1] = 0;
    for (uint32_t n = lt; n < (ck.cv >> 3); n += kBlk) {
        const float4 a = reinterpret_cast<const float4 *>(&val[h][8 * n])[0];
        const float4 b = reinterpret_cast<const float4 *>(&val[h][8 * n])[1];
        const float e[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
        double t = 0.0;
        for (int j = 0; j < 8; ++j) t += (double)e[j];
        pyr[h][n] = t;
    }
    __syncthreads();
    for (int k = 2; k <= ck.cl; ++k) {
        base[k] = base[k - 1] + (ck.cv >> (3 * (k - 1)));
        const uint32_t nk = ck.cv >> (3 * k);
        for (uint32_t n = lt; n < nk; n += kBlk) {
            double t = 0.0;
            for (int j = 0; j < 8; ++j) t += pyr[h][base[k - 1] + 8 * n + j];
            pyr[h][base[k] + n] = t;
        }
        __syncthreads();
    }
    double err = 0.0;
    for (int64_t ib = i0 + lt; ib < i1; ib += kLeafBatch * kBlk) {
        uint32_t kk[kLeafBatch];
        uint8_t lv[kLeafBatch];
        float uu[kLeafBatch];
#pragma unroll
        for (int q = 0; q < kLeafBatch; ++q) {
            const int64_t i = ib + q * kBlk;
            if (i < i1) {
                kk[q] = key[i];
                lv[q] = level[i];
                uu[q] = u[i];
            }
        }
#pragma unroll
        for (int q = 0; q < kLeafBatch; ++q) {
            if (ib + q * kBlk >= i1) break;
            const int k = ck.D - lv[q];  // the leaf is a cube of 8^k voxels
            if (k > ck.cl) continue;     // larger than the chunk
            const uint32_t o = kk[q] - a;
            const double t = k == 0 ? (double)val[h][o] : pyr[h][base[k] + (o >> (3 * k))];
            // the mean: times 8^-k, exact like the division by the power of two
            err += fabs((double)uu[q] - t * ldexp(1.0, -3 * k));
        }
    }
    // per wave (a fixed shuffle tree), then the chunk's waves in order
    for (int off = 32; off > 0; off >>= 1) err += __shfl_down(err, off, 64);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = err;
    __syncthreads();
    if (lt == 0) {
        double t = 0.0;
        for (int wv = 0; wv < kBlk / 64; ++wv) t += red[h * (kBlk / 64) + wv];
        partial[c] = t;
        csum[c] = pyr[h][base[ck.cl]];
    }
}

// one level of the pyramid above the chunks: out[n] = sum of in[8 n .. 8 n + 7]
__global__ void k_pyr_up(const double *in, int64_t n_out, double *out) {
    const int64_t n = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    if (n >= n_out) return;
    double s = 0.0;
    for (int j = 0; j < 8; ++j) s += in[8 * n + j];
    out[n] = s;
}

struct PyrLevels {
    const double *lev[kMaxDepth + 1];  // lev[q]: sums of the level-q cubes (q below the chunks' level)
};

// Eq. 7 terms of the leaves larger than a chunk, summed per block
__global__ void __launch_bounds__(kBlk) k_quant_coarse(int64_t L, int D, int q0, const uint32_t *__restrict__ key,
                                                       const uint8_t *__restrict__ level,
                                                       const float *__restrict__ u, PyrLevels pl, double *partial) {
    __shared__ double red[kBlk];
    const int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    double err = 0.0;
    if (i < L && level[i] < q0) {
        const int l = level[i], k = D - l;
        const double s = pl.lev[l][key[i] >> (3 * k)];
        err = fabs((double)u[i] - s * ldexp(1.0, -3 * k));
    }
    red[threadIdx.x] = err;
    __syncthreads();
    for (int st = kBlk / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
        __syncthreads();
    }
    if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

KeyIndex key_index(Ctx &c) {
    LeafStore &s = c.lv();
    const int D = c.prm.max_depth, shift = key_table_shift(D);
    return KeyIndex{s.key.p, c.L, c.s.key_table.p, shift, 1u << (3 * D - shift)};
}

}  // namespace

namespace {

// first leaf of every chunk (scratch c.s.mesh_first)
const uint32_t *chunk_first(Ctx &c, const Chunking &ck) {
    c.s.mesh_first.reserve((size_t)ck.n + 1);
    hipLaunchKernelGGL(k_chunk_first, dim3((unsigned)cdiv(ck.n + 1, kBlk)), dim3(kBlk), 0, c.stream, key_index(c),
                       ck, c.s.mesh_first.p);
    OTF_LAUNCH_CHECK("k_chunk_first");
    return c.s.mesh_first.p;
}

}  // namespace

void dense_field(Ctx &c, float *dense) {
    const Chunking ck = chunking(c.prm.max_depth);
    const uint32_t *first = chunk_first(c, ck);
    LeafStore &s = c.lv();
    prof_begin(c);
    hipLaunchKernelGGL(k_dense, dim3((unsigned)(ck.n / ck.pair)), dim3(kBlk * ck.pair), 0, c.stream, s.key.p,
                       s.level.p, s.u.p, first, ck, dense);
    prof_end(c, kProfField);
    OTF_LAUNCH_CHECK("k_dense");
}

int64_t marching_cubes(Ctx &c, float iso, int64_t cap, float *h_xyz, unsigned long long *h_edge) {
    const int D = c.prm.max_depth;
    if (D < 1) return 0;
    const int64_t G = int64_t(1) << D, rows = (G - 1) * (G - 1);
    if (!c.s.mc_table.p) {
        const std::vector<McCase> tab = make_table();
        c.s.mc_table.reserve(sizeof(McCase) * 256);
        OTF_HIP(hipMemcpy(c.s.mc_table.p, tab.data(), sizeof(McCase) * 256, hipMemcpyHostToDevice));
    }
    const McCase *tab = reinterpret_cast<const McCase *>(c.s.mc_table.p);
    DBuf<float> dense;
    dense.reserve((size_t)(G * G * G));
    dense_field(c, dense.p);
    DBuf<uint32_t> cnt, first;
    cnt.reserve((size_t)rows);
    first.reserve((size_t)rows + 1);
    const unsigned blocks = (unsigned)cdiv(rows, kBlk / 64);
    prof_begin(c);
    hipLaunchKernelGGL(k_mc_count, dim3(blocks), dim3(kBlk), 0, c.stream, dense.p, D, iso, tab, cnt.p);
    prof_end(c, kProfMcCount);
    OTF_LAUNCH_CHECK("k_mc_count");
    // a row holds at most 12 triangles per cell; past 2^32 in all, the 32-bit
    // offsets would wrap
    if ((double)rows * (G - 1) * kMaxTri >= 4294967296.0) {
        std::vector<uint32_t> h((size_t)rows);
        OTF_HIP(hipMemcpyAsync(h.data(), cnt.p, sizeof(uint32_t) * rows, hipMemcpyDeviceToHost, c.stream));
        OTF_HIP(hipStreamSynchronize(c.stream));
        uint64_t t = 0;
        for (uint32_t v : h) t += v;
        if (t >= 4294967296ull) fail(OTF_E_CAPACITY, "mesh of 2^32 triangles or more");
    }
    const int64_t ntri = scan_exclusive_u32(c, cnt.p, first.p, rows);
    if (ntri > cap || !h_xyz || !h_edge) return ntri;
    if (ntri == 0) return 0;
    DBuf<float> xyz;
    DBuf<unsigned long long> edge;
    xyz.reserve((size_t)(9 * ntri));
    edge.reserve((size_t)(3 * ntri));
    prof_begin(c);
    hipLaunchKernelGGL(k_mc_emit, dim3(blocks), dim3(kBlk), 0, c.stream, dense.p, D, iso, tab, first.p, xyz.p,
                       edge.p);
    prof_end(c, kProfMcEmit);
    OTF_LAUNCH_CHECK("k_mc_emit");
    OTF_HIP(hipMemcpyAsync(h_xyz, xyz.p, sizeof(float) * 9 * ntri, hipMemcpyDeviceToHost, c.stream));
    OTF_HIP(hipMemcpyAsync(h_edge, edge.p, sizeof(unsigned long long) * 3 * ntri, hipMemcpyDeviceToHost, c.stream));
    OTF_HIP(hipStreamSynchronize(c.stream));
    return ntri;
}

double quantisation_error(Ctx &c, const float *dense_dev) {
    const int D = c.prm.max_depth;
    const Chunking ck = chunking(D);
    const int q0 = D - ck.cl;  // level of the chunks
    const int64_t L = c.L, nb = cdiv(L, kBlk);
    // the pyramid's levels q0 (chunk totals), q0 - 1, ..., 0
    int64_t up = 0;
    for (int q = 0; q < q0; ++q) up += int64_t(1) << (3 * q);
    DBuf<double> csum, upper, part;
    csum.reserve((size_t)ck.n);
    upper.reserve((size_t)std::max<int64_t>(up, 1));
    part.reserve((size_t)(ck.n + nb));
    LeafStore &s = c.lv();
    const uint32_t *first = chunk_first(c, ck);
    prof_begin(c);
    hipLaunchKernelGGL(k_quant_chunk, dim3((unsigned)(ck.n / ck.pair)), dim3(kBlk * ck.pair), 0, c.stream, s.key.p,
                       s.level.p, s.u.p, first, ck, dense_dev, csum.p, part.p);
    OTF_LAUNCH_CHECK("k_quant_chunk");
    PyrLevels pl{};
    const double *below = csum.p;
    int64_t at = 0;
    for (int q = q0 - 1; q >= 0; --q) {
        const int64_t nq = int64_t(1) << (3 * q);
        double *out = upper.p + at;
        hipLaunchKernelGGL(k_pyr_up, dim3((unsigned)cdiv(nq, kBlk)), dim3(kBlk), 0, c.stream, below, nq, out);
        pl.lev[q] = out;
        below = out;
        at += nq;
    }
    OTF_LAUNCH_CHECK("k_pyr_up");
    hipLaunchKernelGGL(k_quant_coarse, dim3((unsigned)nb), dim3(kBlk), 0, c.stream, L, D, q0, s.key.p, s.level.p,
                       s.u.p, pl, part.p + ck.n);
    prof_end(c, kProfEq7);
    OTF_LAUNCH_CHECK("k_quant_coarse");
    std::vector<double> h((size_t)(ck.n + nb));
    OTF_HIP(hipMemcpyAsync(h.data(), part.p, sizeof(double) * h.size(), hipMemcpyDeviceToHost, c.stream));
    OTF_HIP(hipStreamSynchronize(c.stream));
    double t = 0.0;
    for (double v : h) t += v;
    return t;
}

}  // namespace otf
