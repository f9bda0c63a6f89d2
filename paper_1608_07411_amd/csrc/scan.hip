// Device-wide prefix scans (one pass over tiles of 8192 elements with
// decoupled look-back; wave64 shuffles inside a wave, LDS across the 4 waves
// of a block), used for compaction: leaf emission, observation and adjacency
// offsets, split lists. Also the small host read-backs of device counters.
#include "otf_internal.h"

namespace otf {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 32;  // consecutive elements per thread, moved with 16-byte loads and stores
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

// Thread-contiguous loads of kItems elements (16-byte vectors when the whole
// run is in range and aligned) and the matching u32 stores.
__device__ inline void load_items(const uint32_t *in, int64_t first, int64_t n, bool vec, uint32_t (&v)[kItems]) {
    if (vec && first + kItems <= n) {
        const uint4 *q = reinterpret_cast<const uint4 *>(in + first);
#pragma unroll
        for (int k = 0; k < kItems / 4; ++k) {
            const uint4 w = q[k];
            v[4 * k] = w.x;
            v[4 * k + 1] = w.y;
            v[4 * k + 2] = w.z;
            v[4 * k + 3] = w.w;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kItems; ++k) v[k] = (first + k < n) ? in[first + k] : 0u;
    }
}

__device__ inline void load_items(const uint8_t *in, int64_t first, int64_t n, bool vec, uint32_t (&v)[kItems]) {
    if (vec && first + kItems <= n) {
        const uint4 *q = reinterpret_cast<const uint4 *>(in + first);
#pragma unroll
        for (int k = 0; k < kItems / 16; ++k) {
            const uint4 w = q[k];
            const uint32_t x[4] = {w.x, w.y, w.z, w.w};
#pragma unroll
            for (int j = 0; j < 16; ++j) v[16 * k + j] = (x[j >> 2] >> (8 * (j & 3))) & 0xFFu;
        }
    } else {
#pragma unroll
        for (int k = 0; k < kItems; ++k) v[k] = (first + k < n) ? (uint32_t)in[first + k] : 0u;
    }
}

// Input adaptors whose elements are formed from a byte array as they are
// loaded (no intermediate array): FlagBitIn: 1 where flag & mask is non-zero;
// RunHeadIn: i where leaf i starts a run of equal non-zero join bits
// (flag & 6), else 0.
struct FlagBitIn {
    const uint8_t *flag;
    uint32_t mask;
};
struct RunHeadIn {
    const uint8_t *flag;
};

__device__ inline void load_items(const FlagBitIn &in, int64_t first, int64_t n, bool vec, uint32_t (&v)[kItems]) {
    load_items(in.flag, first, n, vec, v);
#pragma unroll
    for (int k = 0; k < kItems; ++k) v[k] = (v[k] & in.mask) ? 1u : 0u;
}

__device__ inline void load_items(const RunHeadIn &in, int64_t first, int64_t n, bool vec, uint32_t (&v)[kItems]) {
    load_items(in.flag, first, n, vec, v);  // 0 past the end
    uint32_t prev = (first > 0 && first - 1 < n) ? (uint32_t)(in.flag[first - 1] & 6u) : 0u;
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const uint32_t j = v[k] & 6u;
        const int64_t i = first + k;
        v[k] = (j != 0u && (i == 0 || prev != j)) ? (uint32_t)i : 0u;
        prev = j;
    }
}

// Whole tiles go through LDS: loaded with coalesced 16-byte accesses (lane
// order across the tile), read back by each thread as its kItems
// consecutive elements, and the results written back the same way. Element i
// of the tile sits at lds_at(i): one pad word per 32 keeps the per-thread
// reads free of bank conflicts.
__device__ inline int lds_at(int i) { return i + (i >> 5); }
constexpr int kTileLds = kTile + kTile / 32;

__device__ inline void tile_to_lds(const uint32_t *in, uint32_t *s) {
    const uint4 *q = reinterpret_cast<const uint4 *>(in);
#pragma unroll
    for (int k = 0; k < kTile / (4 * kThreads); ++k) {
        const int v4 = threadIdx.x + kThreads * k;
        const uint4 w = q[v4];
        const int i = lds_at(4 * v4);  // the 4 words stay inside one group of 32
        s[i] = w.x;
        s[i + 1] = w.y;
        s[i + 2] = w.z;
        s[i + 3] = w.w;
    }
}

__device__ inline void tile_to_lds(const uint8_t *in, uint32_t *s) {
    const uint4 *q = reinterpret_cast<const uint4 *>(in);
#pragma unroll
    for (int k = 0; k < kTile / (16 * kThreads); ++k) {
        const int v4 = threadIdx.x + kThreads * k;
        const uint4 w = q[v4];
        const uint32_t x[4] = {w.x, w.y, w.z, w.w};
        const int i = lds_at(16 * v4);  // the 16 bytes stay inside one group of 32
#pragma unroll
        for (int j = 0; j < 16; ++j) s[i + j] = (x[j >> 2] >> (8 * (j & 3))) & 0xFFu;
    }
}

__device__ inline const uint32_t *raw_of(const uint32_t *in) { return in; }
__device__ inline const uint8_t *raw_of(const uint8_t *in) { return in; }
__device__ inline const uint8_t *raw_of(const FlagBitIn &in) { return in.flag; }
__device__ inline const uint8_t *raw_of(const RunHeadIn &in) { return in.flag; }

// this thread's kItems elements of the tile starting at element base
template <class P>
__device__ inline void lds_items(const P *, const uint32_t *s, int64_t, uint32_t (&v)[kItems]) {
    const int i0 = kItems * threadIdx.x;
#pragma unroll
    for (int k = 0; k < kItems; ++k) v[k] = s[lds_at(i0 + k)];
}
__device__ inline void lds_items(const FlagBitIn &in, const uint32_t *s, int64_t, uint32_t (&v)[kItems]) {
    const int i0 = kItems * threadIdx.x;
#pragma unroll
    for (int k = 0; k < kItems; ++k) v[k] = (s[lds_at(i0 + k)] & in.mask) ? 1u : 0u;
}
__device__ inline void lds_items(const RunHeadIn &in, const uint32_t *s, int64_t base, uint32_t (&v)[kItems]) {
    const int i0 = kItems * threadIdx.x;
    uint32_t prev = i0 > 0 ? (s[lds_at(i0 - 1)] & 6u) : (base > 0 ? (uint32_t)(in.flag[base - 1] & 6u) : 0u);
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const uint32_t j = s[lds_at(i0 + k)] & 6u;
        const int64_t i = base + i0 + k;
        v[k] = (j != 0u && (i == 0 || prev != j)) ? (uint32_t)i : 0u;
        prev = j;
    }
}

__device__ inline void lds_to_tile(const uint32_t *s, uint32_t *out) {
    uint4 *q = reinterpret_cast<uint4 *>(out);
#pragma unroll
    for (int k = 0; k < kTile / (4 * kThreads); ++k) {
        const int v4 = threadIdx.x + kThreads * k;
        const int i = lds_at(4 * v4);
        q[v4] = make_uint4(s[i], s[i + 1], s[i + 2], s[i + 3]);
    }
}

__host__ inline bool host_aligned16(const void *p) { return (uintptr_t)p % 16 == 0; }
__host__ inline bool host_aligned16(const FlagBitIn &in) { return host_aligned16(in.flag); }
__host__ inline bool host_aligned16(const RunHeadIn &in) { return host_aligned16(in.flag); }

__device__ inline void store_items(uint32_t *out, int64_t first, int64_t n, bool vec, const uint32_t (&o)[kItems]) {
    if (vec && first + kItems <= n) {
        uint4 *q = reinterpret_cast<uint4 *>(out + first);
#pragma unroll
        for (int k = 0; k < kItems / 4; ++k) q[k] = make_uint4(o[4 * k], o[4 * k + 1], o[4 * k + 2], o[4 * k + 3]);
    } else {
#pragma unroll
        for (int k = 0; k < kItems; ++k)
            if (first + k < n) out[first + k] = o[k];
    }
}

// Single-pass scan with decoupled look-back. Block b scans tile b: it
// publishes the tile aggregate, then its first wave looks back over the
// states of the preceding tiles, 64 at a time, until it meets a tile whose
// inclusive prefix is published; it then publishes its own inclusive prefix
// and writes its outputs. Workgroups are dispatched in index order, so every
// tile a block waits on belongs to a block that is running or done.
//
// Tile state word: epoch (bits 63..34) | status (33..32: 1 aggregate,
// 2 inclusive prefix) | value (31..0). The epoch changes with every scan, so
// the states never need clearing; a word of another epoch reads as "not yet".
// The wait is bounded: after kSpinLimit polls the block records the failure
// in the health flag (read back by the host) and continues, so a kernel never
// hangs.
constexpr uint32_t kSpinLimit = 1u << 22;

__device__ inline uint64_t pack_state(uint32_t epoch, uint32_t status, uint32_t value) {
    return ((uint64_t)epoch << 34) | ((uint64_t)status << 32) | value;
}

// Two scans of the same length can share one launch: blocks [ntiles,
// 2 ntiles) scan (in2, out2) with their own tile states.
//
// Compaction (bit 0 of `compact` for the first scan, bit 1 for the second;
// inputs of 0 and 1 only, AddOp): instead of the ranks, out[r] = i for the
// r-th element i that is 1 (r < cap), in index order; the total as usual.
template <class In, class Op>
__global__ void __launch_bounds__(kThreads) k_scan(In in, int64_t n, uint32_t *out, Op op, int exclusive,
                                                   int vec, uint32_t *total_out, unsigned long long *state,
                                                   uint32_t epoch, int64_t ntiles, uint32_t *health, In in2,
                                                   uint32_t *out2, uint32_t *total_out2, int compact, uint32_t cap,
                                                   uint32_t cap2) {
    __shared__ uint32_t smem[kWaves];
    __shared__ uint32_t s_tile[kTileLds];
    __shared__ uint32_t s_prefix;
    const bool second = (int64_t)blockIdx.x >= ntiles;
    const int64_t tile = (int64_t)blockIdx.x - (second ? ntiles : 0);
    const bool cmp = (compact & (second ? 2 : 1)) != 0;  // block-uniform
    if (second) {
        in = in2;
        out = out2;
        total_out = total_out2;
        state += ntiles;
        cap = cap2;
    }
    const int64_t first = tile * kTile + (int64_t)threadIdx.x * kItems;
    uint32_t v[kItems];
    const int64_t base = tile * kTile;
    const bool whole = vec != 0 && base + kTile <= n;  // block-uniform
    if (whole) {
        tile_to_lds(raw_of(in) + base, s_tile);
        __syncthreads();
        lds_items(in, s_tile, base, v);
    } else {
        load_items(in, first, n, vec != 0, v);
    }
    uint32_t acc = 0;
#pragma unroll
    for (int k = 0; k < kItems; ++k) acc = op(acc, v[k]);
    uint32_t excl, total;
    block_scan(acc, smem, op, excl, total);
    if (threadIdx.x == 0)
        __hip_atomic_store(&state[tile], pack_state(epoch, tile == 0 ? 2u : 1u, total), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    if (tile > 0 && threadIdx.x < 64) {
        const int lane = threadIdx.x;
        uint32_t prefix = 0;
        int64_t look = tile - 1;  // lane j reads tile look - j
        uint32_t spins = 0;
        while (true) {
            const int64_t t = look - lane;
            uint32_t st = 2, val = 0;  // before tile 0: an empty prefix (never summed)
            if (t >= 0) {
                const uint64_t w = __hip_atomic_load(&state[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                st = ((uint32_t)(w >> 34) == epoch) ? (uint32_t)(w >> 32) & 3u : 0u;
                val = (uint32_t)w;
            }
            const uint64_t have_prefix = __ballot(st == 2);
            const uint64_t not_ready = __ballot(st == 0);
            const int stop = have_prefix ? __ffsll((long long)have_prefix) - 1 : 64;  // nearest published prefix
            const uint64_t needed = stop >= 63 ? ~0ull : ((2ull << stop) - 1);
            if (not_ready & needed) {
                if (++spins > kSpinLimit) {
                    if (lane == 0) atomicOr(health, 1u);
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
                continue;
            }
            uint32_t x = lane <= stop ? val : 0u;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) x = op(x, (uint32_t)__shfl_xor((int)x, off, 64));
            prefix = op(prefix, x);
            if (stop < 64) break;
            look -= 64;
        }
        if (lane == 0) {
            __hip_atomic_store(&state[tile], pack_state(epoch, 2u, op(prefix, total)), __ATOMIC_RELAXED,
                               __HIP_MEMORY_SCOPE_AGENT);
            s_prefix = prefix;
        }
    }
    __syncthreads();
    const uint32_t tp = tile > 0 ? s_prefix : 0u;
    uint32_t run = op(tp, excl);
    if (cmp) {
#pragma unroll
        for (int k = 0; k < kItems; ++k) {
            if (v[k] != 0u && run < cap) out[run] = (uint32_t)(first + k);
            run += v[k];
        }
        if (total_out && tile == ntiles - 1 && threadIdx.x == 0) *total_out = op(tp, total);
        return;
    }
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const uint32_t x = v[k];
        if (exclusive) {
            v[k] = run;
            run = op(run, x);
        } else {
            run = op(run, x);
            v[k] = run;
        }
    }
    if (whole) {
        __syncthreads();  // every thread has read its elements
        const int i0 = kItems * threadIdx.x;
#pragma unroll
        for (int k = 0; k < kItems; ++k) s_tile[lds_at(i0 + k)] = v[k];
        __syncthreads();
        lds_to_tile(s_tile, out + base);
    } else {
        store_items(out, first, n, vec != 0, v);
    }
    if (total_out && tile == ntiles - 1 && threadIdx.x == 0) *total_out = op(tp, total);
}

__global__ void fill_u32(uint32_t *p, int64_t n, uint32_t v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void fill_u64(unsigned long long *p, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ull;
}

template <class In, class Op>
void scan_any(Ctx &c, In in, uint32_t *out, int64_t n, Op op, bool exclusive, uint32_t *total_dev, In in2 = In{},
              uint32_t *out2 = nullptr, uint32_t *total_dev2 = nullptr, int compact = 0, uint32_t cap = 0,
              uint32_t cap2 = 0) {
    const bool pair = out2 != nullptr;
    if (n <= 0) {
        if (total_dev) hipLaunchKernelGGL(fill_u32, dim3(1), dim3(64), 0, c.stream, total_dev, (int64_t)1, 0u);
        if (total_dev2) hipLaunchKernelGGL(fill_u32, dim3(1), dim3(64), 0, c.stream, total_dev2, (int64_t)1, 0u);
        return;
    }
    const int64_t tiles = cdiv(n, kTile);
    const int64_t nstate = pair ? 2 * tiles : tiles;
    ScanState &ss = c.s.scan;
    if ((size_t)nstate > ss.state.n || !ss.state.p) {
        ss.state.reserve((size_t)nstate);
        hipLaunchKernelGGL(fill_u64, dim3((unsigned)cdiv((int64_t)ss.state.n, 256)), dim3(256), 0, c.stream,
                           ss.state.p, (int64_t)ss.state.n);
        ss.epoch = 0;
    }
    if (++ss.epoch >= (1u << 30)) {  // epochs wrap: clear the states and restart
        hipLaunchKernelGGL(fill_u64, dim3((unsigned)cdiv((int64_t)ss.state.n, 256)), dim3(256), 0, c.stream,
                           ss.state.p, (int64_t)ss.state.n);
        ss.epoch = 1;
    }
    const int vec = (host_aligned16(in) && host_aligned16(out) &&
                     (!pair || (host_aligned16(in2) && host_aligned16(out2))))
                        ? 1
                        : 0;
    hipLaunchKernelGGL((k_scan<In, Op>), dim3((unsigned)nstate), dim3(kThreads), 0, c.stream, in, n, out, op,
                       exclusive ? 1 : 0, vec, total_dev, ss.state.p, ss.epoch, tiles,
                       c.counters.p + kScanHealthSlot, pair ? in2 : in, pair ? out2 : out,
                       pair ? total_dev2 : total_dev, compact, cap, pair ? cap2 : cap);
    OTF_LAUNCH_CHECK("k_scan");
}

// dst[j] = sum over b < nblocks of part[j * stride + b], j < k: one block,
// a fixed reduction order (no atomics; many same-address atomics from the
// blocks of a large grid serialise).
__global__ void __launch_bounds__(1024) k_sum_parts(const uint32_t *part, int64_t nblocks, int k, int64_t stride,
                                                    uint32_t *dst) {
    __shared__ uint32_t red[16];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int j = 0; j < k; ++j) {
        uint32_t acc = 0;
        for (int64_t b0 = threadIdx.x; b0 < nblocks; b0 += 8 * 1024) {
            uint32_t x[8];
#pragma unroll
            for (int r = 0; r < 8; ++r) x[r] = b0 + r * 1024 < nblocks ? part[j * stride + b0 + r * 1024] : 0u;
#pragma unroll
            for (int r = 0; r < 8; ++r) acc += x[r];
        }
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) acc += (uint32_t)__shfl_xor((int)acc, off, 64);
        if (lane == 0) red[wid] = acc;
        __syncthreads();
        if (threadIdx.x == 0) {
            uint32_t t = 0;
            for (int w = 0; w < 16; ++w) t += red[w];
            dst[j] = t;
        }
        __syncthreads();
    }
}

struct ReadArgs {
    const uint32_t *src[kReadMax + 1];
    int slot[kReadMax + 1];
    int n;
};

// one lane: the values, then (release, system scope) the sequence number
__global__ void k_read_back(ReadArgs a, uint32_t *host, int seq_slot, uint32_t seq) {
    if (threadIdx.x != 0) return;
    for (int t = 0; t < a.n; ++t)
        __hip_atomic_store(host + a.slot[t], *a.src[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __hip_atomic_store(host + seq_slot, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

uint32_t read_total(Ctx &c, const uint32_t *dev) {
    read_back(c, {{dev, 8}});
    return c.h_counters[8];
}

}  // namespace

namespace {
uint32_t rb_begin(Ctx &c, std::initializer_list<ReadItem> items, hipStream_t st, int seq_slot, uint32_t &counter) {
    if (items.size() > (size_t)kReadMax) fail(OTF_E_INVALID, "too many read-back items");
    ReadArgs a{};
    for (const ReadItem &it : items) {
        a.src[a.n] = it.src;
        a.slot[a.n] = it.slot;
        ++a.n;
    }
    a.src[a.n] = c.counters.p + kScanHealthSlot;
    a.slot[a.n] = kScanHealthSlot;
    ++a.n;
    const uint32_t seq = ++counter;
    hipLaunchKernelGGL(k_read_back, dim3(1), dim3(64), 0, st, a, c.d_h_counters, seq_slot, seq);
    OTF_LAUNCH_CHECK("k_read_back");
    return seq;
}

// Spins until the sequence number reaches the ticket. Every few thousand
// polls the stream is queried: an error fails; a finished stream without the
// number means the store never arrived and fails too.
void rb_wait(Ctx &c, uint32_t ticket, hipStream_t st, int seq_slot) {
    const uint32_t *seqp = c.h_counters + seq_slot;
    auto arrived = [&] { return (int32_t)(__atomic_load_n(seqp, __ATOMIC_ACQUIRE) - ticket) >= 0; };
    for (uint32_t spins = 1; !arrived(); ++spins) {
        if ((spins & 4095u) == 0) {
            const hipError_t e = hipStreamQuery(st);
            if (e == hipSuccess) {
                if (arrived()) break;
                fail(OTF_E_DEVICE, "read-back store did not arrive");
            }
            if (e != hipErrorNotReady) {
                (void)hipGetLastError();
                fail(OTF_E_DEVICE, std::string("stream failed: ") + hipGetErrorString(e));
            }
        }
    }
    if (__atomic_load_n(c.h_counters + kScanHealthSlot, __ATOMIC_ACQUIRE))
        fail(OTF_E_DEVICE, "a device scan's look-back wait timed out");
}
}  // namespace

uint32_t read_back_begin(Ctx &c, std::initializer_list<ReadItem> items) {
    return rb_begin(c, items, c.stream, kSeqSlot, c.read_seq);
}

void read_back_wait(Ctx &c, uint32_t ticket) { rb_wait(c, ticket, c.stream, kSeqSlot); }

uint32_t read_back_begin_side(Ctx &c, std::initializer_list<ReadItem> items) {
    return rb_begin(c, items, c.side, kSideSeqSlot, c.side_seq);
}

void read_back_wait_side(Ctx &c, uint32_t ticket) { rb_wait(c, ticket, c.side, kSideSeqSlot); }

void read_back(Ctx &c, std::initializer_list<ReadItem> items) { read_back_wait(c, read_back_begin(c, items)); }

void finish(Ctx &c) {
    read_back(c, {});
    OTF_HIP(hipStreamSynchronize(c.stream));
    if (const uint32_t b = take_bounds_flag())
        fail(OTF_E_DEVICE, "index out of range in a sweep (bounds-checked build), flags " + std::to_string(b));
}

namespace {
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

void scan_compact_u8(Ctx &c, const uint8_t *flags, uint32_t *list, uint32_t cap, uint32_t *total_dev, int64_t n) {
    scan_any(c, flags, list, n, AddOp{}, true, total_dev, (const uint8_t *)nullptr, nullptr, nullptr, 1, cap, 0u);
}

void scan_compact_pair_u8(Ctx &c, const uint8_t *a, uint32_t *list_a, uint32_t cap_a, uint32_t *total_a,
                          const uint8_t *b, uint32_t *list_b, uint32_t cap_b, uint32_t *total_b, int64_t n) {
    scan_any(c, a, list_a, n, AddOp{}, true, total_a, b, list_b, total_b, 3, cap_a, cap_b);
}

void sum_parts(Ctx &c, const uint32_t *part, int64_t nblocks, int k, int64_t stride, uint32_t *dst) {
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(1024), 0, c.stream, part, nblocks, k, stride, dst);
    OTF_LAUNCH_CHECK("k_sum_parts");
}

void scan_inclusive_max_u32(Ctx &c, const uint32_t *in, uint32_t *out, int64_t n) {
    scan_any(c, in, out, n, MaxOp{}, false, (uint32_t *)nullptr);
}

void scan_exclusive_pair_u8(Ctx &c, const uint8_t *a, uint32_t *out_a, const uint8_t *b, uint32_t *out_b,
                            int64_t n) {
    scan_any(c, a, out_a, n, AddOp{}, true, out_a + n, b, out_b, out_b + n);
}

void scan_exclusive_pair_u32(Ctx &c, const uint32_t *a, uint32_t *out_a, const uint32_t *b, uint32_t *out_b,
                             int64_t n) {
    scan_any(c, a, out_a, n, AddOp{}, true, out_a + n, b, out_b, out_b + n);
}

void scan_run_starts(Ctx &c, const uint8_t *flag, uint32_t *out, int64_t n) {
    scan_any(c, RunHeadIn{flag}, out, n, MaxOp{}, false, (uint32_t *)nullptr);
}

void scan_exclusive_flag_bits(Ctx &c, const uint8_t *flag, uint32_t mask, uint32_t *out, int64_t n) {
    scan_any(c, FlagBitIn{flag, mask}, out, n, AddOp{}, true, out + n);
}

}  // namespace otf
