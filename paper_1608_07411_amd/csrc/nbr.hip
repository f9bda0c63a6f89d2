// Face adjacency of the fused octree (the neighbourhood of the forward and
// backward differences, Sec. 3.2 and Fig. 5) on the Morton-sorted leaf array.
// For each leaf and face, the same-size cell across the face is looked up by
// binary search on the keys; if it is subdivided, its sub-cells touching the
// face are visited depth first in child order, which yields ascending keys.
// Entries: neighbour index | direction << 26 | neighbour level << 28.
// + list (faces +x,+y,+z) feeds the gradient, - list (-x,-y,-z) the divergence.
#include "otf_internal.h"

namespace otf {
namespace {

constexpr int kBlk = 256;

__device__ inline int64_t find_leaf(const uint32_t *__restrict__ key, int64_t L, uint32_t k) {
    // largest i with key[i] <= k (key[0] == 0)
    int64_t lo = 0, hi = L;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (key[mid] <= k) lo = mid;
        else hi = mid;
    }
    return lo;
}

template <bool FILL>
__global__ void __launch_bounds__(kBlk) k_nbr(int64_t L, const uint32_t *__restrict__ key,
                                              const uint8_t *__restrict__ level, int D, uint32_t *cnt_p,
                                              uint32_t *cnt_m, const uint32_t *__restrict__ off_p,
                                              const uint32_t *__restrict__ off_m, uint32_t *ent_p, uint32_t *ent_m) {
    const int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    if (i >= L) return;
    const uint32_t G = 1u << D;
    const int ln = level[i];
    const uint32_t s = 1u << (D - ln);
    uint32_t xyz[3];
    demorton3(key[i], xyz[0], xyz[1], xyz[2]);
    uint32_t np = 0, nm = 0;
    uint32_t base_p = FILL ? off_p[i] : 0, base_m = FILL ? off_m[i] : 0;
    // explicit DFS stack of (cell min-corner key, cell level)
    uint32_t st_key[40];
    uint8_t st_lvl[40];
    for (int face = 0; face < 6; ++face) {
        const int d = face % 3;
        const bool plus = face < 3;
        uint32_t q[3] = {xyz[0], xyz[1], xyz[2]};
        if (plus) {
            if (q[d] + s >= G) continue;
            q[d] += s;
        } else {
            if (q[d] == 0) continue;
            q[d] -= s;
        }
        int sp = 0;
        st_key[sp] = morton3(q[0], q[1], q[2]);
        st_lvl[sp] = (uint8_t)ln;
        ++sp;
        while (sp > 0) {
            --sp;
            const uint32_t ck = st_key[sp];
            const int cl = st_lvl[sp];
            const int64_t j = find_leaf(key, L, ck);
            const int lj = level[j];
            if (lj <= cl) {
                if (FILL) {
                    const uint32_t e = (uint32_t)j | ((uint32_t)d << kIdxBits) | ((uint32_t)lj << (kIdxBits + 2));
                    if (plus) ent_p[base_p + np] = e;
                    else ent_m[base_m + nm] = e;
                }
                if (plus) ++np;
                else ++nm;
            } else {
                // the 4 children touching the face; pushed in reverse child order
                const int shift = 3 * (D - cl - 1);
                const int want = plus ? 0 : 1;
                for (int ch = 7; ch >= 0; --ch) {
                    if (((ch >> d) & 1) != want) continue;
                    st_key[sp] = ck | ((uint32_t)ch << shift);
                    st_lvl[sp] = (uint8_t)(cl + 1);
                    ++sp;
                }
            }
        }
    }
    if (!FILL) {
        cnt_p[i] = np;
        cnt_m[i] = nm;
    }
}

}  // namespace

void build_neighbours(Ctx &c) {
    LeafStore &s = c.lv();
    const int64_t L = c.L;
    const unsigned g = (unsigned)cdiv(L, kBlk);
    c.s.a.reserve(L + 1);
    c.s.b.reserve(L + 1);
    hipLaunchKernelGGL(k_nbr<false>, dim3(g), dim3(kBlk), 0, c.stream, L, s.key.p, s.level.p, c.prm.max_depth,
                       c.s.a.p, c.s.b.p, (const uint32_t *)nullptr, (const uint32_t *)nullptr, (uint32_t *)nullptr,
                       (uint32_t *)nullptr);
    OTF_LAUNCH_CHECK("k_nbr count");
    scan_exclusive_u32_dev(c, c.s.a.p, s.nbp_off.p, L);
    scan_exclusive_u32_dev(c, c.s.b.p, s.nbm_off.p, L);
    OTF_HIP(hipMemcpyAsync(c.h_counters + 10, s.nbp_off.p + L, sizeof(uint32_t), hipMemcpyDeviceToHost, c.stream));
    OTF_HIP(hipMemcpyAsync(c.h_counters + 11, s.nbm_off.p + L, sizeof(uint32_t), hipMemcpyDeviceToHost, c.stream));
    OTF_HIP(hipStreamSynchronize(c.stream));
    c.n_nbp = c.h_counters[10];
    c.n_nbm = c.h_counters[11];
    c.nbp.reserve(c.n_nbp);
    c.nbm.reserve(c.n_nbm);
    hipLaunchKernelGGL(k_nbr<true>, dim3(g), dim3(kBlk), 0, c.stream, L, s.key.p, s.level.p, c.prm.max_depth,
                       (uint32_t *)nullptr, (uint32_t *)nullptr, (const uint32_t *)s.nbp_off.p,
                       (const uint32_t *)s.nbm_off.p, c.nbp.p, c.nbm.p);
    OTF_LAUNCH_CHECK("k_nbr fill");
}

}  // namespace otf
