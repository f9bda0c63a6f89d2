// Device-wide prefix scans (reduce-then-scan over tiles of 2048 elements;
// wave64 shuffles inside a wave, LDS across the 4 waves of a block). Used for
// compaction: leaf emission, observation and adjacency offsets, split lists.
#include "otf_internal.h"

namespace otf {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;
constexpr int kWaves = kThreads / 64;

struct AddOp {
    __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a + b; }
};
struct MaxOp {
    __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return a > b ? a : b; }
};

// Block-wide scan of one value per thread (identity 0 for both ops).
template <class Op>
__device__ void block_scan(uint32_t v, uint32_t *smem, Op op, uint32_t &excl, uint32_t &total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t n = __shfl_up(incl, off, 64);
        if (lane >= off) incl = op(incl, n);
    }
    if (lane == 63) smem[wid] = incl;
    __syncthreads();
    uint32_t wave_prefix = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kWaves; ++w) {
        uint32_t s = smem[w];
        if (w < wid) wave_prefix = op(wave_prefix, s);
        tot = op(tot, s);
    }
    __syncthreads();
    uint32_t prev = __shfl_up(incl, 1, 64);
    excl = lane == 0 ? wave_prefix : op(wave_prefix, prev);
    total = tot;
}

template <class In, class Op>
__global__ void __launch_bounds__(kThreads) tile_reduce(const In *__restrict__ in, int64_t n,
                                                        uint32_t *__restrict__ tile_sums, Op op) {
    __shared__ uint32_t smem[kWaves];
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k)
        if (base + k < n) acc = op(acc, (uint32_t)in[base + k]);
    uint32_t excl, total;
    block_scan(acc, smem, op, excl, total);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = total;
}

// out[i] = op(tile prefix, in[tile start .. i-1]) (exclusive) or .. i (inclusive).
// May run in place (each thread reads its items before writing them).
template <class In, class Op>
__global__ void __launch_bounds__(kThreads) tile_scan(const In *in, int64_t n, const uint32_t *__restrict__ tile_prefix,
                                                      uint32_t *out, Op op, int exclusive,
                                                      uint32_t *__restrict__ total_out) {
    __shared__ uint32_t smem[kWaves];
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)threadIdx.x * kItems;
    uint32_t v[kItems];
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        v[k] = (base + k < n) ? (uint32_t)in[base + k] : 0u;
        acc = op(acc, v[k]);
    }
    uint32_t excl, total;
    block_scan(acc, smem, op, excl, total);
    const uint32_t tp = tile_prefix ? tile_prefix[blockIdx.x] : 0u;
    uint32_t run = op(tp, excl);
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        if (base + k < n) {
            if (exclusive) {
                out[base + k] = run;
                run = op(run, v[k]);
            } else {
                run = op(run, v[k]);
                out[base + k] = run;
            }
        }
    }
    if (total_out && blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) *total_out = op(tp, total);
}

__global__ void fill_u32(uint32_t *p, int64_t n, uint32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// Exclusive scan of the per-tile values in place (recursive over levels).
template <class Op>
void scan_tiles(Ctx &c, uint32_t *vals, int64_t n, Op op, size_t depth) {
    if (n <= 1) {
        if (n == 1) hipLaunchKernelGGL(fill_u32, dim3(1), dim3(64), 0, c.stream, vals, (int64_t)1, 0u);
        return;
    }
    int64_t tiles = cdiv(n, kTile);
    if (depth >= 4) fail(OTF_E_INVALID, "scan too large");
    c.s.scan_lv[depth].reserve((size_t)tiles);
    uint32_t *sums = c.s.scan_lv[depth].p;
    hipLaunchKernelGGL((tile_reduce<uint32_t, Op>), dim3((unsigned)tiles), dim3(kThreads), 0, c.stream,
                       (const uint32_t *)vals, n, sums, op);
    OTF_LAUNCH_CHECK("tile_reduce");
    scan_tiles(c, sums, tiles, op, depth + 1);
    hipLaunchKernelGGL((tile_scan<uint32_t, Op>), dim3((unsigned)tiles), dim3(kThreads), 0, c.stream,
                       (const uint32_t *)vals, n, (const uint32_t *)sums, vals, op, 1, (uint32_t *)nullptr);
    OTF_LAUNCH_CHECK("tile_scan");
}

template <class In, class Op>
void scan_any(Ctx &c, const In *in, uint32_t *out, int64_t n, Op op, bool exclusive, uint32_t *total_dev) {
    if (n <= 0) {
        if (total_dev) hipLaunchKernelGGL(fill_u32, dim3(1), dim3(64), 0, c.stream, total_dev, (int64_t)1, 0u);
        return;
    }
    int64_t tiles = cdiv(n, kTile);
    c.s.scan_lv[0].reserve((size_t)tiles);
    uint32_t *sums = c.s.scan_lv[0].p;
    if (tiles > 1) {
        hipLaunchKernelGGL((tile_reduce<In, Op>), dim3((unsigned)tiles), dim3(kThreads), 0, c.stream, in, n, sums,
                           op);
        OTF_LAUNCH_CHECK("tile_reduce");
        scan_tiles(c, sums, tiles, op, 1);
    }
    hipLaunchKernelGGL((tile_scan<In, Op>), dim3((unsigned)tiles), dim3(kThreads), 0, c.stream, in, n,
                       tiles > 1 ? (const uint32_t *)sums : (const uint32_t *)nullptr, out, op, exclusive ? 1 : 0,
                       total_dev);
    OTF_LAUNCH_CHECK("tile_scan");
}

uint32_t read_total(Ctx &c, const uint32_t *dev) {
    OTF_HIP(hipMemcpyAsync(c.h_counters + 8, dev, sizeof(uint32_t), hipMemcpyDeviceToHost, c.stream));
    OTF_HIP(hipStreamSynchronize(c.stream));
    return c.h_counters[8];
}

}  // namespace

uint32_t scan_exclusive_u8(Ctx &c, const uint8_t *in, uint32_t *out, int64_t n) {
    scan_any(c, in, out, n, AddOp{}, true, c.counters.p + 8);
    return read_total(c, c.counters.p + 8);
}

uint32_t scan_exclusive_u32(Ctx &c, const uint32_t *in, uint32_t *out, int64_t n) {
    scan_any(c, in, out, n, AddOp{}, true, c.counters.p + 8);
    return read_total(c, c.counters.p + 8);
}

void scan_exclusive_u32_dev(Ctx &c, const uint32_t *in, uint32_t *out, int64_t n) {
    scan_any(c, in, out, n, AddOp{}, true, out + n);
}

void scan_exclusive_u32_dev_u8(Ctx &c, const uint8_t *in, uint32_t *out, int64_t n) {
    scan_any(c, in, out, n, AddOp{}, true, out + n);
}

void scan_inclusive_max_u32(Ctx &c, const uint32_t *in, uint32_t *out, int64_t n) {
    scan_any(c, in, out, n, MaxOp{}, false, (uint32_t *)nullptr);
}

}  // namespace otf
