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

// value of u at every finest voxel: dense[(z G + y) G + x] = u of the leaf containing it
__global__ void k_dense(KeyIndex ki, const float *u, int D, float *dense) {
    const int64_t G = int64_t(1) << D, n = G * G * G;
    for (int64_t v = (int64_t)blockIdx.x * kBlk + threadIdx.x; v < n; v += (int64_t)gridDim.x * kBlk) {
        const uint32_t x = (uint32_t)(v % G), y = (uint32_t)((v / G) % G), z = (uint32_t)(v / (G * G));
        dense[v] = u[find_leaf(ki, morton3(x, y, z))];
    }
}

__device__ inline int cell_case(const float *dense, int64_t G, int64_t x, int64_t y, int64_t z, float iso) {
    int cs = 0;
#pragma unroll
    for (int c = 0; c < 8; ++c) {
        const int64_t q = ((z + ((c >> 2) & 1)) * G + (y + ((c >> 1) & 1))) * G + (x + (c & 1));
        cs |= (dense[q] < iso ? 1 : 0) << c;
    }
    return cs;
}

__global__ void k_mc_count(const float *dense, int D, float iso, const McCase *tab, uint8_t *ntri) {
    const int64_t G = int64_t(1) << D, C = G - 1, n = C * C * C;
    for (int64_t k = (int64_t)blockIdx.x * kBlk + threadIdx.x; k < n; k += (int64_t)gridDim.x * kBlk) {
        const int64_t x = k % C, y = (k / C) % C, z = k / (C * C);
        ntri[k] = (uint8_t)tab[cell_case(dense, G, x, y, z, iso)].ntri;
    }
}

// triangle t of the mesh: xyz[9 t ..] its 3 vertices (world), edge[3 t ..]
// their grid edges: 3 ((z G + y) G + x) + axis of the edge's lower voxel
__global__ void k_mc_emit(const float *dense, int D, float iso, const McCase *tab, const uint32_t *off,
                          float *xyz, unsigned long long *edge) {
    const int64_t G = int64_t(1) << D, C = G - 1, n = C * C * C;
    const float h = ldexpf(1.0f, -D);
    for (int64_t k = (int64_t)blockIdx.x * kBlk + threadIdx.x; k < n; k += (int64_t)gridDim.x * kBlk) {
        const int64_t x = k % C, y = (k / C) % C, z = k / (C * C);
        const McCase &m = tab[cell_case(dense, G, x, y, z, iso)];
        uint32_t w = off[k];
        for (int t = 0; t < m.ntri; ++t, ++w) {
            for (int j = 0; j < 3; ++j) {
                const int e = m.edge[3 * t + j];
                const int axis = e >> 2, o = e & 3;
                int64_t p[3] = {x, y, z};
                const int u = axis == 0 ? 1 : 0, v = axis == 2 ? 1 : 2;
                p[u] += o & 1;
                p[v] += (o >> 1) & 1;
                const int64_t q0 = (p[2] * G + p[1]) * G + p[0];
                const int64_t q1 = q0 + (axis == 0 ? 1 : axis == 1 ? G : G * G);
                const float v0 = dense[q0], v1 = dense[q1];
                const float tt = (iso - v0) / (v1 - v0);
                float c[3];
                for (int d = 0; d < 3; ++d) {
                    const float base = (float)p[d] + 0.5f;
                    c[d] = (d == axis ? base + tt : base) * h;
                }
                xyz[9 * (int64_t)w + 3 * j] = c[0];
                xyz[9 * (int64_t)w + 3 * j + 1] = c[1];
                xyz[9 * (int64_t)w + 3 * j + 2] = c[2];
                edge[3 * (int64_t)w + j] = 3ull * (unsigned long long)q0 + (unsigned long long)axis;
            }
        }
    }
}

// Eq. 7 terms: |u(n) - mean of dense over n| per leaf, summed per block in a
// fixed order. Leaves of more than 512 voxels are averaged by the whole block
// (in wave-ballot order), the others by their own thread.
__global__ void __launch_bounds__(kBlk) k_quant(int64_t L, int D, const uint32_t *key, const uint8_t *level,
                                                const float *u, const float *dense, double *partial) {
    __shared__ double red[kBlk];
    __shared__ uint32_t big[kBlk];
    __shared__ uint32_t wcount[kBlk / 64];
    const int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int64_t G = int64_t(1) << D;
    double err = 0.0;
    bool is_big = false;
    if (i < L) {
        const int64_t s = int64_t(1) << (D - level[i]);
        if (s * s * s > 512) {
            is_big = true;
        } else {
            uint32_t x0, y0, z0;
            demorton3(key[i], x0, y0, z0);
            double sum = 0.0;
            for (int64_t z = 0; z < s; ++z)
                for (int64_t y = 0; y < s; ++y)
                    for (int64_t x = 0; x < s; ++x) sum += (double)dense[((z0 + z) * G + (y0 + y)) * G + (x0 + x)];
            err = fabs((double)u[i] - sum / (double)(s * s * s));
        }
    }
    const uint64_t bm = __ballot(is_big);
    if (lane == 0) wcount[wid] = (uint32_t)__popcll(bm);
    __syncthreads();
    uint32_t base = 0, nbig = 0;
    for (int w = 0; w < kBlk / 64; ++w) {
        if (w < wid) base += wcount[w];
        nbig += wcount[w];
    }
    if (is_big) big[base + __popcll(bm & ((1ull << lane) - 1))] = (uint32_t)threadIdx.x;
    __syncthreads();
    for (uint32_t b = 0; b < nbig; ++b) {
        const int64_t leaf = (int64_t)blockIdx.x * kBlk + big[b];
        const int64_t s = int64_t(1) << (D - level[leaf]), vol = s * s * s;
        uint32_t x0, y0, z0;
        demorton3(key[leaf], x0, y0, z0);
        double sum = 0.0;
        for (int64_t q = threadIdx.x; q < vol; q += kBlk) {
            const int64_t x = q % s, y = (q / s) % s, z = q / (s * s);
            sum += (double)dense[((z0 + z) * G + (y0 + y)) * G + (x0 + x)];
        }
        red[threadIdx.x] = sum;
        __syncthreads();
        for (int st = kBlk / 2; st > 0; st >>= 1) {
            if ((int)threadIdx.x < st) red[threadIdx.x] += red[threadIdx.x + st];
            __syncthreads();
        }
        if (threadIdx.x == big[b]) err = fabs((double)u[leaf] - red[0] / (double)vol);
        __syncthreads();
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

unsigned grid_for(int64_t n) { return (unsigned)std::min<int64_t>(cdiv(n, kBlk), 65536); }

}  // namespace

void dense_field(Ctx &c, float *dense) {
    const int D = c.prm.max_depth;
    const int64_t n = int64_t(1) << (3 * D);
    hipLaunchKernelGGL(k_dense, dim3(grid_for(n)), dim3(kBlk), 0, c.stream, key_index(c), c.lv().u.p, D, dense);
    OTF_LAUNCH_CHECK("k_dense");
}

int64_t marching_cubes(Ctx &c, float iso, int64_t cap, float *h_xyz, unsigned long long *h_edge) {
    const int D = c.prm.max_depth;
    if (D < 1) return 0;
    const int64_t G = int64_t(1) << D, C = G - 1, ncell = C * C * C;
    if (!c.s.mc_table.p) {
        const std::vector<McCase> tab = make_table();
        c.s.mc_table.reserve(sizeof(McCase) * 256);
        OTF_HIP(hipMemcpy(c.s.mc_table.p, tab.data(), sizeof(McCase) * 256, hipMemcpyHostToDevice));
    }
    const McCase *tab = reinterpret_cast<const McCase *>(c.s.mc_table.p);
    DBuf<float> dense;
    dense.reserve((size_t)(G * G * G));
    dense_field(c, dense.p);
    DBuf<uint8_t> cnt;
    cnt.reserve((size_t)ncell);
    hipLaunchKernelGGL(k_mc_count, dim3(grid_for(ncell)), dim3(kBlk), 0, c.stream, dense.p, D, iso, tab, cnt.p);
    OTF_LAUNCH_CHECK("k_mc_count");
    DBuf<uint32_t> off;
    off.reserve((size_t)ncell + 1);
    const int64_t ntri = scan_exclusive_u8(c, cnt.p, off.p, ncell);
    if (ntri > cap || !h_xyz || !h_edge) return ntri;
    if (ntri == 0) return 0;
    DBuf<float> xyz;
    DBuf<unsigned long long> edge;
    xyz.reserve((size_t)(9 * ntri));
    edge.reserve((size_t)(3 * ntri));
    hipLaunchKernelGGL(k_mc_emit, dim3(grid_for(ncell)), dim3(kBlk), 0, c.stream, dense.p, D, iso, tab, off.p, xyz.p,
                       edge.p);
    OTF_LAUNCH_CHECK("k_mc_emit");
    OTF_HIP(hipMemcpyAsync(h_xyz, xyz.p, sizeof(float) * 9 * ntri, hipMemcpyDeviceToHost, c.stream));
    OTF_HIP(hipMemcpyAsync(h_edge, edge.p, sizeof(unsigned long long) * 3 * ntri, hipMemcpyDeviceToHost, c.stream));
    OTF_HIP(hipStreamSynchronize(c.stream));
    return ntri;
}

double quantisation_error(Ctx &c, const float *dense_dev) {
    const int64_t blocks = cdiv(c.L, kBlk);
    DBuf<double> part;
    part.reserve((size_t)blocks);
    LeafStore &s = c.lv();
    hipLaunchKernelGGL(k_quant, dim3((unsigned)blocks), dim3(kBlk), 0, c.stream, c.L, c.prm.max_depth, s.key.p,
                       s.level.p, s.u.p, dense_dev, part.p);
    OTF_LAUNCH_CHECK("k_quant");
    std::vector<double> h((size_t)blocks);
    OTF_HIP(hipMemcpyAsync(h.data(), part.p, sizeof(double) * blocks, hipMemcpyDeviceToHost, c.stream));
    OTF_HIP(hipStreamSynchronize(c.stream));
    double t = 0.0;
    for (double v : h) t += v;
    return t;
}

}  // namespace otf
