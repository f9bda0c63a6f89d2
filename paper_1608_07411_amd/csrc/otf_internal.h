// Internal declarations of libotf: device buffers, the context, device-side
// helpers shared by the kernels, and the host launchers of every phase.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>
#include <string>
#include <vector>
#include <initializer_list>

#include "otf.h"

namespace otf {

constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr int kMaxViews = 64;
constexpr int kMaxDepth = 10;
// adjacency entry: neighbour index (26 bits) | direction (2 bits) | level (4 bits)
constexpr int kIdxBits = 26;
constexpr uint32_t kIdxMask = (1u << kIdxBits) - 1u;
constexpr int64_t kLeafLimit = int64_t(1) << kIdxBits;
// adjacency lists longer than this are summed by a whole wave (see sweep.hip)
constexpr uint32_t kLongList = 64;

// ---------------------------------------------------------------------------
// errors
// ---------------------------------------------------------------------------
struct Failure {
    otf_status st;
    std::string msg;
};

[[noreturn]] void fail(otf_status st, const std::string &msg);

// Allocation-failure injection (a test hook): while an entry point runs on a
// context, this points at the context's countdown; the allocation that takes
// it from 1 to 0 fails as if the device were out of memory.
extern thread_local int64_t *t_alloc_countdown;
inline bool alloc_fault_due() {
    return t_alloc_countdown && *t_alloc_countdown > 0 && --*t_alloc_countdown == 0;
}
void hip_check(hipError_t e, const char *what);
#define OTF_HIP(x) ::otf::hip_check((x), #x)
#define OTF_LAUNCH_CHECK(name) ::otf::hip_check(hipGetLastError(), name)

// ---------------------------------------------------------------------------
// device buffer (hipMalloc / hipFree), grows on demand
// ---------------------------------------------------------------------------
#ifdef OTF_DEBUG_BOUNDS
// Bounds-checked build: every buffer is followed by a guard zone of
// kGuardBytes filled with kGuardByte, registered with the place that reserved
// it. A zone is checked when its buffer is freed and after every call on a
// context (guard_check_all); a changed byte means a write past the end of the
// buffer, and the call fails naming the buffer's reserve site.
constexpr size_t kGuardBytes = 65536;
constexpr uint8_t kGuardByte = 0xA5;
void guard_register(void *p, size_t bytes, const char *file, int line);
void guard_release(void *p);
void guard_check_all();
#define OTF_RESERVE_SITE , const char *site_file = __builtin_FILE(), int site_line = __builtin_LINE()
constexpr size_t kGuardAlloc = kGuardBytes;
#else
#define OTF_RESERVE_SITE
constexpr size_t kGuardAlloc = 0;
#endif

template <class T>
struct DBuf {
    T *p = nullptr;
    size_t n = 0;
    DBuf() = default;
    DBuf(const DBuf &) = delete;
    DBuf &operator=(const DBuf &) = delete;
    ~DBuf() { release(); }
    void release() {
        if (p) {
#ifdef OTF_DEBUG_BOUNDS
            guard_release(p);
#endif
            (void)hipFree(p);
        }
        p = nullptr;
        n = 0;
    }
    // ensure capacity for `count` elements; contents are discarded on growth,
    // which leaves a quarter of headroom so that slowly growing sizes do not
    // reallocate (and synchronise) on every call
    void reserve(size_t count OTF_RESERVE_SITE) {
        if (count <= n && p) return;
        release();
        size_t c = count ? count + count / 4 + 64 : 1;
        if (alloc_fault_due()) fail(OTF_E_NOMEM, "device allocation failed (injected)");
        hipError_t e = hipMalloc((void **)&p, c * sizeof(T) + kGuardAlloc);
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            fail(OTF_E_NOMEM, "hipMalloc of " + std::to_string(c * sizeof(T)) + " bytes failed");
        }
        n = c;
#ifdef OTF_DEBUG_BOUNDS
        guard_register(p, c * sizeof(T), site_file, site_line);
#endif
    }
    void swap(DBuf &o) {
        std::swap(p, o.p);
        std::swap(n, o.n);
    }
    T *get() const { return p; }
};

// ---------------------------------------------------------------------------
// geometry helpers
// ---------------------------------------------------------------------------
__host__ __device__ inline uint32_t part1by2(uint32_t v) {
    v &= 0x3FFu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}
__host__ __device__ inline uint32_t compact1by2(uint32_t v) {
    v &= 0x09249249u;
    v = (v ^ (v >> 2)) & 0x030C30C3u;
    v = (v ^ (v >> 4)) & 0x0300F00Fu;
    v = (v ^ (v >> 8)) & 0xFF0000FFu;
    v = (v ^ (v >> 16)) & 0x000003FFu;
    return v;
}
__host__ __device__ inline uint32_t morton3(uint32_t x, uint32_t y, uint32_t z) {
    return part1by2(x) | (part1by2(y) << 1) | (part1by2(z) << 2);
}
__host__ __device__ inline void demorton3(uint32_t k, uint32_t &x, uint32_t &y, uint32_t &z) {
    x = compact1by2(k);
    y = compact1by2(k >> 1);
    z = compact1by2(k >> 2);
}

// Leaf lookup in the Morton-sorted key array: largest i with key[i] <= k
// (key[0] == 0).
__device__ inline int64_t find_leaf(const uint32_t *__restrict__ key, int64_t L, uint32_t k) {
    int64_t lo = 0, hi = L;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (key[mid] <= k) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Bucket index over the key space: table[b] = the leaf containing the first
// point of bucket b (buckets of 2^shift keys), so a lookup only searches
// between two table entries. Built for the current store by the adjacency
// build (Scratch::key_table); key_table_shift gives its bucket size.
struct KeyIndex {
    const uint32_t *key;
    int64_t L;
    const uint32_t *table;
    int shift;
    uint32_t nb;
};

inline int key_table_shift(int D) { return 3 * D > 20 ? 3 * D - 20 : 0; }

// largest i with key[i] <= k
__device__ inline int64_t find_leaf(const KeyIndex &ki, uint32_t k) {
    const uint32_t b = k >> ki.shift;
    int64_t lo = ki.table[b];
    int64_t hi = (b + 1 < ki.nb) ? (int64_t)ki.table[b + 1] + 1 : ki.L;
    while (hi - lo > 1) {
        const int64_t mid = (lo + hi) >> 1;
        if (ki.key[mid] <= k) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Coupling coefficients by level pair, one correctly rounded division of exact
// operands each: c[ln][lk] for the gradient of leaf n toward its + neighbour k,
// cp[lm][ln] for the divergence of leaf n from its - neighbour m.
struct Coef {
    float c[kMaxDepth + 1][kMaxDepth + 1];
    float cp[kMaxDepth + 1][kMaxDepth + 1];
};
Coef make_coef(int max_depth);

struct CamDev {
    float fx, fy, cx, cy;
    int32_t width, height;
    float R[9];
    float C[3];
};

// Eq. 1 at one finest voxel centre; returns whether the voxel is observed.
// Operation order is fixed (one IEEE operation at a time, explicit fma).
__device__ inline bool tsdf_voxel(const CamDev &cam, const float *__restrict__ depth_v, float h, float delta,
                                  float eta, uint32_t a, uint32_t b, uint32_t c, float &f) {
    float dx = __fsub_rn(__fmul_rn(__fadd_rn((float)a, 0.5f), h), cam.C[0]);
    float dy = __fsub_rn(__fmul_rn(__fadd_rn((float)b, 0.5f), h), cam.C[1]);
    float dz = __fsub_rn(__fmul_rn(__fadd_rn((float)c, 0.5f), h), cam.C[2]);
    const float *R = cam.R;
    float X = __fmaf_rn(R[0], dx, __fmaf_rn(R[3], dy, __fmul_rn(R[6], dz)));
    float Y = __fmaf_rn(R[1], dx, __fmaf_rn(R[4], dy, __fmul_rn(R[7], dz)));
    float Z = __fmaf_rn(R[2], dx, __fmaf_rn(R[5], dy, __fmul_rn(R[8], dz)));
    if (!(Z > 0.0f)) return false;
    float pu = __fmaf_rn(cam.fx, X / Z, cam.cx);
    float pv = __fmaf_rn(cam.fy, Y / Z, cam.cy);
    if (!(pu >= 0.0f && pu < (float)cam.width && pv >= 0.0f && pv < (float)cam.height)) return false;
    int pi = (int)pu, pj = (int)pv;
    float Dm = depth_v[(size_t)pj * cam.width + pi];
    if (!(Dm > 0.0f && Dm <= 3.4028234663852886e38f)) return false;
    float r = sqrtf(__fmaf_rn(dx, dx, __fmaf_rn(dy, dy, __fmul_rn(dz, dz))));
    float phi = __fsub_rn(Dm, r);
    if (phi < -eta) return false;
    f = fminf(1.0f, fmaxf(-1.0f, phi / delta));
    return true;
}

// Generalised shrinkage (the prox of the normalised weighted L1 data term):
// the median of {F_(1..M)} and {u' - t S_k, k = 0..M}, S_k = 2 P_k - W_tot.
// p_k is non-increasing and F_(k+1) non-decreasing in k, so the smallest k
// with p_k <= F_(k+1) (F_(M+1) = +inf) selects the median as max(p_k, F_(k))
// (F_(0) = -inf). Unit weights give S_k = 2k - M exactly. A zero is returned
// as +0.
__device__ inline float prox_select(float up, float t, int M, bool unit, const float *__restrict__ F,
                                    const float *__restrict__ W, float wt) {
    if (M == 0) return up + 0.0f;
    int k = 0;
    float pk;
    if (unit) {
        for (;;) {
            pk = __fmaf_rn(-t, (float)(2 * k - M), up);
            if (k == M || !(pk > F[k])) break;
            ++k;
        }
    } else {
        float P = 0.0f;
        for (;;) {
            pk = __fmaf_rn(-t, __fmaf_rn(2.0f, P, -wt), up);
            if (k == M || !(pk > F[k])) break;
            P = P + W[k];
            ++k;
        }
    }
    const float v = (k == 0 || pk >= F[k - 1]) ? pk : F[k - 1];
    return v + 0.0f;
}

// ---------------------------------------------------------------------------
// stores
// ---------------------------------------------------------------------------
// Per-view linear octrees, all views in one pool; each view's nodes in
// (level, key) order with the 8 children of an inner node contiguous.
struct ViewStore {
    DBuf<float> S;
    DBuf<uint32_t> cnt, child, key;
    DBuf<uint8_t> level;
    DBuf<uint32_t> root;               // per view: pool index of the root
    // dense indices at two levels (-1: none): per cell (Morton order) and
    // view, the deepest node containing the cell, (level << 28) | index
    DBuf<uint32_t> table, table_c;
    int table_level = -1, table_c_level = -1;
    std::vector<int64_t> count, base;  // per view node count and pool offset (host)
    int64_t n_nodes = 0;
};

struct ViewDev {
    const float *S;
    const uint32_t *cnt;
    const uint32_t *child;
    const uint32_t *root;
    int n_views;
    int max_depth;
    const uint32_t *table;  // dense index (null: descend from the roots)
    int table_level;
    const uint32_t *table_c;  // coarser dense index (null: none)
    int table_c_level;
};
constexpr uint32_t kTableIdxBits = 28;

// Fused leaves: Morton-sorted structure of arrays.
struct LeafStore {
    DBuf<uint32_t> key;
    DBuf<uint8_t> level;
    DBuf<float> u, ubar, p, ds;  // p: 3 planes of `cap` floats (x, y, z)
    DBuf<uint32_t> obs_off;
    DBuf<uint8_t> obs_m, obs_unit;
    DBuf<float> inv, wtot;
    DBuf<uint32_t> nbp_off, nbm_off;  // cap + 1
    DBuf<uint32_t> nbp, nbm;          // adjacency entries (+ faces, - faces)
    int64_t n_nbp = 0, n_nbm = 0;
    DBuf<uint8_t> flag;
    DBuf<float> uprime, uold;
    DBuf<uint32_t> src;  // restructure: index of the leaf in the previous store, or kNone
    DBuf<uint8_t> need;  // restructure: adjacency must be searched (new, or next to a change)
    DBuf<uint32_t> heavy_p, heavy_m;  // leaves whose + / - list is longer than kLongList
    int64_t n_heavy_p = 0, n_heavy_m = 0;
    int64_t cap = 0;
    void reserve(int64_t n);
};

// Observation pool: per leaf a segment of M entries sorted by (F, view):
// F, the weight W, and P = the sum of the weights before the entry (P_0 = 0,
// formed sequentially in sorted order).
struct ObsPool {
    DBuf<float> F, W, P;
    int64_t used = 0, cap = 0;
    void reserve(int64_t n);
};

// One round of the split cascade: the 8 children of every parent.
struct Round {
    DBuf<uint32_t> porigin;                    // per parent: origin leaf (old index)
    DBuf<uint32_t> ckey, corigin, crank, cnt, pos;
    DBuf<uint8_t> clevel, csplit;
    DBuf<float> cu, cub;
    int64_t np = 0, nc = 0;
};

// Look-back scan state: per-tile state words, epoch-tagged so that they are
// never cleared between scans.
struct ScanState {
    DBuf<unsigned long long> state;
    uint32_t epoch = 0;
};

// Scratch reused across phases.
struct Scratch {
    DBuf<uint32_t> a, b, c, d, e, f, g;
    DBuf<uint32_t> adj_bad;  // adjacency check of the bounds-checked build
    DBuf<uint8_t> u8a, u8b;
    DBuf<float> fa, fb, fc, fd, fe;
    ScanState scan;
    DBuf<uint32_t> hv_leaf, hv_lo, hv_hi;  // adjacency: faces with long ranges
    DBuf<uint8_t> hv_face;
    DBuf<uint32_t> ch_base, ch_item, ch_count, ch_pos;  // chunks of the long ranges
    DBuf<uint32_t> key_table;                           // bucket index over leaf keys
    DBuf<uint32_t> dirty;                               // leaves whose adjacency is searched again
    DBuf<uint32_t> nb_j, nb_m;                          // faces located by the count pass, for the fill
    DBuf<uint32_t> part;                                // per-block partial counts
    DBuf<unsigned char> mc_table;                       // marching-cubes case table (device)
    DBuf<uint32_t> mesh_first;                          // first leaf of each chunk of the finest grid
    // restructure temporaries (grow-only: an allocation or free per iteration
    // would synchronise the device)
    DBuf<uint8_t> r_sf, r_tM, r_tU, r_isnew, r_Mt;
    DBuf<uint32_t> r_nrank, r_tidx, r_moff, r_loff;
    DBuf<uint8_t> r_jcand;          // collapse: leaves that start an inner node inside a collapse
    DBuf<uint32_t> r_jrank, r_jlist;  // their ranks and list
    DBuf<float> r_jv;
    DBuf<double> dred;
    std::vector<Round *> rounds;
    ~Scratch() {
        for (Round *r : rounds) delete r;
    }
};

// Timed kinds: the solver's (read by otf_profile_read) and the evaluation's
// (read by otf_profile_read_eval).
enum ProfKind {
    kProfDual = 0,
    kProfPrimal = 1,
    kProfRestructure = 2,
    kProfEnergy = 3,
    kProfSolverKinds = 4,
    kProfField = 4,    // the finest-grid field kernel
    kProfEq7 = 5,      // the Eq. 7 kernels
    kProfMcCount = 6,  // the marching-cubes count kernel
    kProfMcEmit = 7,   // the marching-cubes emit kernel
    kProfKinds = 8
};

// Solver of the running fuse call: primal-dual, or the paper's gradient
// descent (TV weight lam, step xi, smoothing eps^2); split children follow it.
struct Solver {
    int gd = 0;
    float lam = 0.0f, xi = 0.0f, eps2 = 0.0f;
};

struct Ctx {
    int device = 0;
    int64_t fail_alloc_after = 0;  // allocation-failure injection countdown (0: off)
    std::vector<otf_batch *> batches;  // batches that hold this context as a member
    Solver sol;
    hipStream_t stream = nullptr;
    // a second stream of the library's own (default priority) with fork and
    // join events: a restructure's observation gather runs there beside the
    // adjacency search; every use is joined back into `stream`
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    // frozen structure: a stream on which chunks of iterations are recorded
    // into a graph (recording runs nothing; the graph is launched on
    // `stream`), and how many iterations of the last fuse call were replayed
    hipStream_t capture = nullptr;
    int64_t graph_iterations = 0;
    // per-iteration log (otf_log_every): every log_every-th iteration appends
    // a record to the caller's host array while log_n < log_cap
    bool debug_unwritten_slot = false;  // checked build: the next search leaves + slot 0 unwritten
    int32_t log_every = 0;
    otf_iter_record *log_buf = nullptr;
    int64_t log_cap = 0, log_n = 0;
    otf_params prm{};
    int n_views = 0;
    int64_t iteration = 0;
    bool valid = false;
    ViewStore views;
    LeafStore leaves[2];
    int cur = 0;
    int64_t L = 0;
    ObsPool obs[2];
    int ocur = 0;
    Coef coef{};
    Scratch s;
    // device counters: [0] split flags [1] join flags [2] collapse heads
    // [3] long ranges [4..7] observation totals (2 x u64) [9] long copies
    // [14,15] long-list counts [16..17] accumulated observation totals (u64)
    // [24] scan health flag (non-zero: a look-back wait timed out)
    DBuf<uint32_t> counters;
    uint32_t *h_counters = nullptr;    // pinned, coherent host slots for read-backs (32)
    uint32_t *d_h_counters = nullptr;  // the same slots as the device addresses them
    uint32_t read_seq = 0;             // last read-back sequence number issued
    uint32_t side_seq = 0;             // the same for read-backs on the second stream
    int64_t part_blocks = 0;           // blocks (flag-count partials) of the last primal launch
    int64_t last_splits = 0, last_joins = 0;
    int64_t pool_compactions = 0;  // observation pool compactions by restructures
    bool had_splits = true, had_joins = true;  // flags at the previous restructure
    // profiling: event pairs recorded on the stream, summed when read
    struct ProfRec {
        int kind;
        hipEvent_t a, b;
    };
    bool prof = false;
    std::vector<ProfRec> prof_recs;
    std::vector<hipEvent_t> ev_pool;
    size_t ev_used = 0;
    hipEvent_t prof_open = nullptr;
    double prof_ms[kProfKinds] = {};
    int64_t prof_n[kProfKinds] = {};
    int64_t leaf_updates = 0;     // sum over iterations of the leaf count (always counted)
    // bytes of the dual and primal sweeps (always counted): as implemented
    // [0, 1], and the method's own per leaf-update [2, 3]
    double alg_bytes[4] = {0, 0, 0, 0};
    // structure sizes for the algorithmic byte counts

    std::string err;

    LeafStore &lv() { return leaves[cur]; }
    ObsPool &op() { return obs[ocur]; }
    ViewDev view_dev() const {
        return ViewDev{views.S.p,         views.cnt.p, views.child.p,
                       views.root.p,      n_views,     prm.max_depth,
                       views.table_level >= 0 ? views.table.p : nullptr, views.table_level,
                       views.table_c_level >= 0 ? views.table_c.p : nullptr, views.table_c_level};
    }
};

// ---------------------------------------------------------------------------
// launchers (each issues work on ctx.stream)
// ---------------------------------------------------------------------------
// Host read-back: one small kernel stores up to kReadMax device u32 values into
// the host slots h_counters[slot] and then a sequence number into
// h_counters[kSeqSlot]; the host spins on that number (work queued on the
// stream before the kernel has then finished) instead of synchronising the
// stream, so that work queued after the kernel keeps the device busy while the
// host waits. The scan health flag travels with every read-back and raises
// OTF_E_DEVICE when set. Between read_back_begin and read_back_wait no other
// read-back may use the same slots.
constexpr int kReadMax = 4;
constexpr int kScanHealthSlot = 24;
constexpr int kSideSeqSlot = 30;
constexpr int kSeqSlot = 31;
struct ReadItem {
    const uint32_t *src;
    int slot;
};
uint32_t read_back_begin(Ctx &c, std::initializer_list<ReadItem> items);
void read_back_wait(Ctx &c, uint32_t ticket);
void read_back(Ctx &c, std::initializer_list<ReadItem> items);
// The same on the second stream, with its own sequence slot (kSideSeqSlot),
// so that read-backs of the two streams never overtake each other's number.
uint32_t read_back_begin_side(Ctx &c, std::initializer_list<ReadItem> items);
void read_back_wait_side(Ctx &c, uint32_t ticket);
// While alive, the launchers issue their work on the second stream.
struct OnSideStream {
    Ctx &c;
    hipStream_t saved;
    explicit OnSideStream(Ctx &cc) : c(cc), saved(cc.stream) { c.stream = c.side; }
    ~OnSideStream() { c.stream = saved; }
    OnSideStream(const OnSideStream &) = delete;
    OnSideStream &operator=(const OnSideStream &) = delete;
};
// all work on the stream finished (stream synchronised), scan health checked
void finish(Ctx &c);
// Bounds-checked build: the sweeps' violation flags since the last call
// (cleared); 0 in the default build.
uint32_t take_bounds_flag();
// scans over n elements; the total is returned to the host (synchronises)
uint32_t scan_exclusive_u8(Ctx &c, const uint8_t *in, uint32_t *out, int64_t n);
uint32_t scan_exclusive_u32(Ctx &c, const uint32_t *in, uint32_t *out, int64_t n);
// exclusive scan without a host read-back: out has n+1 entries, out[n] = total
void scan_exclusive_u32_dev(Ctx &c, const uint32_t *in, uint32_t *out, int64_t n);
void scan_exclusive_u32_dev_u8(Ctx &c, const uint8_t *in, uint32_t *out, int64_t n);
// Compaction of 0/1 flags: list[r] = i for the r-th flagged i (r < cap), the
// number of flags at *total_dev (device); the pair form in one launch.
void scan_compact_u8(Ctx &c, const uint8_t *flags, uint32_t *list, uint32_t cap, uint32_t *total_dev, int64_t n);
void scan_compact_pair_u8(Ctx &c, const uint8_t *a, uint32_t *list_a, uint32_t cap_a, uint32_t *total_a,
                          const uint8_t *b, uint32_t *list_b, uint32_t cap_b, uint32_t *total_b, int64_t n);
void scan_inclusive_max_u32(Ctx &c, const uint32_t *in, uint32_t *out, int64_t n);
// two exclusive scans of the same length in one launch (out arrays of n+1)
void scan_exclusive_pair_u8(Ctx &c, const uint8_t *a, uint32_t *out_a, const uint8_t *b, uint32_t *out_b, int64_t n);
void scan_exclusive_pair_u32(Ctx &c, const uint32_t *a, uint32_t *out_a, const uint32_t *b, uint32_t *out_b,
                             int64_t n);
// inclusive max-scan of the run starts of equal non-zero join bits (flag & 6):
// out[i] = the first index of the run containing i (0 outside runs before any)
void scan_run_starts(Ctx &c, const uint8_t *flag, uint32_t *out, int64_t n);
// exclusive scan of (flag[i] & mask) != 0; out has n+1 entries, out[n] = total
void scan_exclusive_flag_bits(Ctx &c, const uint8_t *flag, uint32_t mask, uint32_t *out, int64_t n);
// dst[j] = sum over b < nblocks of part[j * stride + b] for j < k (per-block
// partial counts written by a kernel; a fixed order, no atomics)
void sum_parts(Ctx &c, const uint32_t *part, int64_t nblocks, int k, int64_t stride, uint32_t *dst);

// build: per-view trees, union structure, initial leaves (keys/levels only)
void build_views_and_union(Ctx &c, const float *depth_dev, const std::vector<CamDev> &cams);
// Observation gather for n targets. Target t is the node (tkey[h], tlevel[h])
// with h = tidx ? tidx[t] : t.
// gather_count: Mcount[t] = number of observations.
// gather_fill: observations sorted by (F, view) at base + (out_off ? out_off[t]
// : t * stride) in F / W; header (M, unit, inv, wtot, optional u0 and segment
// offset) written at index h.
void gather_count(Ctx &c, int64_t n, const uint32_t *tkey, const uint8_t *tlevel, const uint32_t *tidx,
                  uint8_t *Mcount);
void gather_fill(Ctx &c, int64_t n, const uint32_t *tkey, const uint8_t *tlevel, const uint32_t *tidx,
                 const uint32_t *out_off, uint32_t base, int stride, float *F, float *W, float *P, uint8_t *M,
                 uint8_t *unit, float *inv, float *wtot, float *u0, uint32_t *off_out);
// gather_fill into rows of `stride` entries (row t at t * stride) that also
// records the per-target count Mt[t]
void gather_rows(Ctx &c, int64_t n, const uint32_t *tkey, const uint8_t *tlevel, const uint32_t *tidx, int stride,
                 float *F, float *W, float *P, uint8_t *Mt, uint8_t *M, uint8_t *unit, float *inv, float *wtot);
// dense index of the view octrees (after they change)
void build_view_table(Ctx &c);
// pool-compacting gather for every leaf of the current store (two passes)
void gather_all_leaves(Ctx &c, bool init_values);
// totals of observations into the device counters (no read-back)
void count_obs(Ctx &c);
// add the observation totals to the per-primal accumulator (device)
void accumulate_obs(Ctx &c, bool all_weights = false);
// face adjacency of the current leaf store
void build_neighbours(Ctx &c);
// Adjacency after a restructure: leaves marked in `need` are searched, the
// others copy their lists from the previous store `old` (leaf src[i]) with
// indices mapped through remap (old index -> new index). Two steps: _begin
// queues the search up to the count of long ranges and starts reading that
// count back; _end (after whatever independent work the caller queues in
// between) finishes it, queueing `overlap` (may be null) while the host waits
// for its first count.
struct NbrOld {  // previous store, for leaves that copy their lists
    const uint8_t *need;      // new leaf: 1 = search its lists, 0 = copy them
    const uint32_t *src;      // new leaf -> old index (kept leaves)
    const uint32_t *off_p, *off_m, *ent_p, *ent_m;
    const uint32_t *remap;    // old index -> its emission offset in the new store (the new index of a
                              // kept leaf), remap[L_old] = L; null for a store built from scratch
    const uint32_t *heavy_p, *heavy_m;  // old leaves with a long + / - list
    uint32_t n_heavy_p, n_heavy_m;
};
struct NbrPending {
    NbrOld old;
    uint32_t ticket, cap;
    const uint32_t *dirty, *n_dirty_dev;
};
// need_scanned: the new store's need flags are already listed in the
// scratch array s.dirty, their number at s.e[0]
NbrPending build_neighbours_begin(Ctx &c, const LeafStore &old, const uint32_t *remap, bool need_scanned);
void build_neighbours_end(Ctx &c, NbrPending &p, void (*overlap)(Ctx &));
// sweeps
void launch_dual(Ctx &c, float sigma);
void launch_primal(Ctx &c, float tau, float tl);
// one step of the paper's gradient descent: the flux sweep (q = Gu / Gamma),
// then the update sweep (flags as the primal sweep's)
void launch_gd_flux(Ctx &c, float eps2);
void launch_gd_update(Ctx &c, float lam, float xi, float eps2);
// split and join flag counts of the last primal sweep into counters[0], [1]
void count_flags(Ctx &c);
// evaluation (meshing and Eq. 7): the finest-grid field of u (G^3 floats,
// index (z G + y) G + x); the marching-cubes mesh at iso (returns the triangle
// count; copies to the host arrays when they hold cap triangles); the
// quantisation error against a finest-grid field on the device
void dense_field(Ctx &c, float *dense);
int64_t marching_cubes(Ctx &c, float iso, int64_t cap, float *h_xyz, unsigned long long *h_edge);
double quantisation_error(Ctx &c, const float *dense_dev);
// energy terms in double; eps > 0: the smoothed terms of the gradient-descent energy
void energy(Ctx &c, double *tv, double *data, double eps = 0.0);
// energy() without device allocation: partials in a static device array
void energy_noalloc(Ctx &c, double *tv, double *data);
// split / join; returns true when the structure changed
bool restructure(Ctx &c, float tl);

// profiling helpers
void prof_begin(Ctx &c);
void prof_end(Ctx &c, ProfKind k);

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }


// ---------------------------------------------------------------------------
// batches: the sweeps of many contexts in the same launches
// ---------------------------------------------------------------------------
struct BatchConfig {
    int blk = 256;  // threads per block = leaves per tile (64, 128, 256 or 512)
    int grid = 0;   // blocks of the sweeps (they stride over the tiles); 0: one per tile
};
struct BatchState {
    std::vector<Ctx *> objs;
    BatchConfig cfg;
    uint32_t ntiles = 0, n_hp = 0, n_hm = 0;  // tiles; long + and - lists over all objects
    DBuf<unsigned char> table;                 // per-object sweep arguments
    DBuf<uint32_t> tile_begin, hp_begin, hm_begin, part;
    DBuf<uint32_t> tile_obj;                   // the member of each tile
    DBuf<Coef> coefs;                          // coupling tables by max depth
    unsigned char *h_stage = nullptr;          // pinned staging for the table uploads
    size_t h_cap = 0;
    hipEvent_t staged = nullptr;               // completion of the last upload
    BatchState() = default;
    BatchState(const BatchState &) = delete;
    BatchState &operator=(const BatchState &) = delete;
    ~BatchState();
};
// (Re)build the device table from the objects' current stores for cfg.blk.
void batch_upload(hipStream_t st, BatchState &b, float sigma, float tau, float tl);
// One iteration's sweeps of every object: dual, long dual, long primal,
// primal, then per object its flag counts and observation totals.
void batch_sweeps(hipStream_t st, BatchState &b);
double dual_bytes(const Ctx &c);
double primal_bytes(const Ctx &c);
void count_sweep_bytes(Ctx &c);  // one iteration's sweep bytes into alg_bytes

}  // namespace otf

struct otf_ctx {
    otf::Ctx c;
};

namespace otf {
// A member context being destroyed leaves its batches (their tables and
// captured graphs are dropped).
void batch_forget(otf_batch *bt, Ctx *c);
}  // namespace otf
