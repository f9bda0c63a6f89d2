// C ABI of libotf: argument validation, context and buffer management, the
// state blob, inspection copies, and the iteration driver.
#include <cmath>
#include <new>
#ifdef OTF_DEBUG_BOUNDS
#include <map>
#include <mutex>
#endif

#include "otf_internal.h"

namespace otf {

void fail(otf_status st, const std::string &msg) { throw Failure{st, msg}; }

#ifdef OTF_DEBUG_BOUNDS
namespace {
struct GuardSite {
    size_t bytes;
    const char *file;
    int line;
    bool reported;  // damage already reported (each zone once)
};
// live buffers of every context (never destroyed: buffers may be freed at exit)
std::map<uintptr_t, GuardSite> &guard_table() {
    static auto *t = new std::map<uintptr_t, GuardSite>();
    return *t;
}
std::mutex &guard_mutex() {
    static auto *m = new std::mutex();
    return *m;
}
std::string g_guard_err;  // the first damaged zone not yet reported

void guard_inspect(uintptr_t p, GuardSite &g, const char *when) {
    if (g.reported) return;
    std::vector<uint8_t> h(kGuardBytes);
    if (hipMemcpy(h.data(), reinterpret_cast<const char *>(p) + g.bytes, kGuardBytes, hipMemcpyDeviceToHost) !=
        hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    for (size_t k = 0; k < kGuardBytes; ++k)
        if (h[k] != kGuardByte) {
            if (g_guard_err.empty()) {
                const char *f = std::strrchr(g.file, '/');
                g_guard_err = "write past the end of a device buffer (bounds-checked build): " +
                              std::to_string(g.bytes) + " bytes reserved at " + (f ? f + 1 : g.file) + ":" +
                              std::to_string(g.line) + ", guard byte " + std::to_string(k) + " changed, found " +
                              when;
            }
            g.reported = true;
            return;
        }
}
}  // namespace

void guard_register(void *p, size_t bytes, const char *file, int line) {
    OTF_HIP(hipMemset(static_cast<char *>(p) + bytes, kGuardByte, kGuardBytes));
    OTF_HIP(hipDeviceSynchronize());
    std::lock_guard<std::mutex> lk(guard_mutex());
    guard_table()[reinterpret_cast<uintptr_t>(p)] = GuardSite{bytes, file, line, false};
}

void guard_release(void *p) {
    (void)hipDeviceSynchronize();  // as hipFree: the buffer's last users have finished
    std::lock_guard<std::mutex> lk(guard_mutex());
    auto it = guard_table().find(reinterpret_cast<uintptr_t>(p));
    if (it == guard_table().end()) return;
    guard_inspect(it->first, it->second, "when it was freed");
    guard_table().erase(it);
}

void guard_check_all() {
    OTF_HIP(hipDeviceSynchronize());
    std::string err;
    {
        std::lock_guard<std::mutex> lk(guard_mutex());
        for (auto &kv : guard_table()) guard_inspect(kv.first, kv.second, "after the call");
        err.swap(g_guard_err);
    }
    if (!err.empty()) fail(OTF_E_DEVICE, err);
}
#endif

void hip_check(hipError_t e, const char *what) {
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Failure{OTF_E_DEVICE, std::string(what) + ": " + hipGetErrorString(e)};
    }
}

Coef make_coef(int D) {
    Coef cf;
    for (int a = 0; a <= kMaxDepth; ++a)
        for (int b = 0; b <= kMaxDepth; ++b) {
            cf.c[a][b] = 0.0f;
            cf.cp[a][b] = 0.0f;
            if (a > D || b > D) continue;
            // gradient of n (level a) toward its + neighbour k (level b)
            float sn = (float)(1u << (D - a)), sk = (float)(1u << (D - b));
            float m = sn < sk ? sn : sk;
            float r = (m / sn) * (m / sn);
            float h = (sn + sk) * 0.5f;
            cf.c[a][b] = r / h;
            // divergence of n (level b) from its - neighbour m (level a)
            float sm = (float)(1u << (D - a));
            float sn2 = (float)(1u << (D - b));
            float mm = sm < sn2 ? sm : sn2;
            float h2 = (sm + sn2) * 0.5f;
            cf.cp[a][b] = (sm * mm * mm) / (h2 * sn2 * sn2 * sn2);
        }
    return cf;
}

void LeafStore::reserve(int64_t n) {
    if (n <= cap && key.p) return;
    int64_t c = n < 1024 ? 1024 : n;
    key.reserve(c);
    level.reserve(c);
    u.reserve(c);
    ubar.reserve(c);
    p.reserve(3 * c);
    ds.reserve(c);
    obs_off.reserve(c);
    obs_m.reserve(c);
    obs_unit.reserve(c);
    inv.reserve(c);
    wtot.reserve(c);
    nbp_off.reserve(c + 1);
    nbm_off.reserve(c + 1);
    flag.reserve(c);
    uprime.reserve(c);
    uold.reserve(c);
    src.reserve(c);
    need.reserve(c);
    cap = c;
}

void ObsPool::reserve(int64_t n) {
    if (n <= cap && F.p) return;
    int64_t c = n < 1024 ? 1024 : n;
    F.reserve(c);
    W.reserve(c);
    P.reserve(c);
    cap = c;
}

namespace {
hipEvent_t next_event(Ctx &c) {
    if (c.ev_used == c.ev_pool.size()) {
        hipEvent_t e;
        OTF_HIP(hipEventCreate(&e));
        c.ev_pool.push_back(e);
    }
    return c.ev_pool[c.ev_used++];
}
}  // namespace

void prof_begin(Ctx &c) {
    if (!c.prof) return;
    c.prof_open = next_event(c);
    OTF_HIP(hipEventRecord(c.prof_open, c.stream));
}

void prof_end(Ctx &c, ProfKind k) {
    if (!c.prof || !c.prof_open) return;
    hipEvent_t b = next_event(c);
    OTF_HIP(hipEventRecord(b, c.stream));
    c.prof_recs.push_back(Ctx::ProfRec{(int)k, c.prof_open, b});
    c.prof_open = nullptr;
}

// Records one event that ends the open interval (credited to kind k, or to
// nothing for k < 0) and opens the next one: consecutive phases share their
// boundary event, so an iteration records one event per phase.
void prof_mark(Ctx &c, int k) {
    if (!c.prof) return;
    hipEvent_t b = next_event(c);
    OTF_HIP(hipEventRecord(b, c.stream));
    if (c.prof_open && k >= 0) c.prof_recs.push_back(Ctx::ProfRec{k, c.prof_open, b});
    c.prof_open = b;
}

// Sum the recorded event pairs into the per-kind totals and recycle the events.
void prof_collect(Ctx &c) {
    if (c.prof_recs.empty()) return;
    OTF_HIP(hipStreamSynchronize(c.stream));
    for (const auto &r : c.prof_recs) {
        float ms = 0.0f;
        OTF_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        c.prof_ms[r.kind] += ms;
        c.prof_n[r.kind] += 1;
    }
    c.prof_recs.clear();
    c.ev_used = 0;
    c.prof_open = nullptr;
}

namespace {

__global__ void k_zero_u32(uint32_t *p, int n) {
    if ((int)threadIdx.x < n) p[threadIdx.x] = 0u;
}

bool finite(float v) { return std::isfinite(v); }

void check_params(const otf_params *p) {
    if (!p) fail(OTF_E_INVALID, "params is null");
    if (p->max_depth < 1 || p->max_depth > kMaxDepth) fail(OTF_E_INVALID, "max_depth must be in 1..10");
    if (!finite(p->delta) || !finite(p->eta) || !finite(p->gamma) || !finite(p->split_tau) ||
        !finite(p->join_tau) || std::isnan(p->spread_tau))
        fail(OTF_E_INVALID, "non-finite parameter");
    if (!(p->delta > 0.0f) || !(p->eta >= p->delta)) fail(OTF_E_INVALID, "need eta >= delta > 0");
    if (!(p->gamma > 0.0f)) fail(OTF_E_INVALID, "need gamma > 0");
    if (!(p->split_tau <= p->join_tau)) fail(OTF_E_INVALID, "need split_tau <= join_tau");
    if (p->restructure_every < 0) fail(OTF_E_INVALID, "restructure_every < 0");
    if (p->max_leaves < 0) fail(OTF_E_INVALID, "max_leaves < 0");
}

void init_state_values(Ctx &c) {
    LeafStore &s = c.lv();
    OTF_HIP(hipMemcpyAsync(s.ubar.p, s.u.p, c.L * sizeof(float), hipMemcpyDeviceToDevice, c.stream));
    for (int d = 0; d < 3; ++d) OTF_HIP(hipMemsetAsync(s.p.p + d * s.cap, 0, c.L * sizeof(float), c.stream));
}

template <class T>
std::vector<T> download(Ctx &c, const T *src, int64_t n) {
    std::vector<T> h((size_t)(n > 0 ? n : 0));
    if (n > 0) OTF_HIP(hipMemcpyAsync(h.data(), src, n * sizeof(T), hipMemcpyDeviceToHost, c.stream));
    return h;
}

template <class T>
void upload(Ctx &c, T *dst, const std::vector<T> &h) {
    if (!h.empty()) OTF_HIP(hipMemcpyAsync(dst, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice, c.stream));
}

struct Writer {
    uint8_t *p;
    int64_t cap, n = 0;
    void put(const void *src, int64_t k) {
        if (p && n + k <= cap) std::memcpy(p + n, src, (size_t)k);
        n += k;
    }
};

struct Reader {
    const uint8_t *p;
    int64_t n, at = 0;
    void get(void *dst, int64_t k) {
        if (at + k > n) fail(OTF_E_INVALID, "state blob truncated");
        std::memcpy(dst, p + at, (size_t)k);
        at += k;
    }
};

#pragma pack(push, 1)
struct NodeRec {
    uint32_t key;
    uint8_t level, leaf;
    uint16_t zero;
    float S;
    uint32_t cnt;
};
struct LeafRec {
    uint32_t key;
    uint8_t level, pad[3];
    float v[5];
};
#pragma pack(pop)
static_assert(sizeof(NodeRec) == 16, "node record");
static_assert(sizeof(LeafRec) == 28, "leaf record");
static_assert(sizeof(otf_params) == 40, "params record");
static_assert(sizeof(otf_camera) == 72, "camera record");

void setup_after_structure(Ctx &c, bool init_values) {
    build_view_table(c);
    gather_all_leaves(c, init_values);
    if (init_values) init_state_values(c);
    build_neighbours(c);
    count_obs(c);
}

}  // namespace

// Bytes the two leaf sweeps of one iteration move as implemented, per sweep.
// Dual: every leaf reads its level, ubar and p and its + adjacency (offset
// and entries), writes p and ds; a neighbour's ubar is counted once per
// leaf, not per entry (a Morton sweep reuses it).
double dual_bytes(const Ctx &c) {
    const double L = (double)c.L;
    return L * (1 + 4 + 12 + 4) + 4.0 * (double)c.leaves[c.cur].n_nbp + L * (12 + 4);
}

// Primal: level, ds, u, the - adjacency, p once per leaf, the observation
// header (offset, count, normaliser, total weight); writes u, ubar and the
// flag byte. The observation segments (F, plus P for leaves with fractional
// weights, 4 bytes each) are added from the device-side accumulator when
// read.
double primal_bytes(const Ctx &c) {
    const double L = (double)c.L;
    return L * (1 + 4 + 4 + 12) + 4.0 * (double)c.leaves[c.cur].n_nbm + L * (4 + 1 + 4 + 4) + L * (4 + 4 + 1);
}

// The method's own bytes per leaf-update of one whole leaf sweep, with no
// reuse across iterations: u, ubar and p each read and written (40), 4 per
// face-adjacency entry of both lists, the observation header (segment offset
// and normaliser, 8), 4 per sorted observation value and 4 per prefix weight
// of a leaf with fractional weights (the latter two from the device-side
// accumulator when read). Attributed to the kernel that moves them: the dual
// reads ubar and p, writes p and reads the + list (28 + 4 E+); the primal
// reads u, writes u and ubar, reads the header and the - list
// (20 + 4 E- + observations).
double dual_method_bytes(const Ctx &c) {
    return 28.0 * (double)c.L + 4.0 * (double)c.leaves[c.cur].n_nbp;
}

double primal_method_bytes(const Ctx &c) {
    return 20.0 * (double)c.L + 4.0 * (double)c.leaves[c.cur].n_nbm;
}

void count_sweep_bytes(Ctx &c) {
    c.alg_bytes[0] += dual_bytes(c);
    c.alg_bytes[1] += primal_bytes(c);
    c.alg_bytes[2] += dual_method_bytes(c);
    c.alg_bytes[3] += primal_method_bytes(c);
}

}  // namespace otf

namespace otf {
thread_local int64_t *t_alloc_countdown = nullptr;
}  // namespace otf

using namespace otf;

namespace {

// Points the allocation-failure countdown at the context for one call.
struct AllocHook {
    int64_t *saved;
    explicit AllocHook(otf_ctx *ctx) : saved(t_alloc_countdown) {
        t_alloc_countdown = ctx ? &ctx->c.fail_alloc_after : nullptr;
    }
    ~AllocHook() { t_alloc_countdown = saved; }
};

template <class F>
otf_status guard(otf_ctx *ctx, bool invalidates, F &&f) {
    AllocHook hook(ctx);
    if (ctx) {
        if (hipSetDevice(ctx->c.device) != hipSuccess) {
            (void)hipGetLastError();
            ctx->c.err = "hipSetDevice failed";
            return OTF_E_DEVICE;
        }
    }
    // after a failure, work the call left on the second stream is waited for
    // (a later call may reuse its buffers)
    auto settle = [&] {
        if (ctx && ctx->c.side) (void)hipStreamSynchronize(ctx->c.side);
    };
    try {
        f();
#ifdef OTF_DEBUG_BOUNDS
        guard_check_all();
#endif
        if (ctx) ctx->c.err.clear();
        return OTF_OK;
    } catch (const Failure &e) {
        settle();
        if (ctx) {
            ctx->c.err = e.msg;
            if (invalidates && e.st != OTF_E_INVALID) ctx->c.valid = false;
        }
        return e.st;
    } catch (const std::bad_alloc &) {
        settle();
        if (ctx) {
            ctx->c.err = "host allocation failed";
            if (invalidates) ctx->c.valid = false;
        }
        return OTF_E_NOMEM;
    } catch (...) {
        settle();
        if (ctx) {
            ctx->c.err = "unexpected failure";
            if (invalidates) ctx->c.valid = false;
        }
        return OTF_E_DEVICE;
    }
}

}  // namespace

extern "C" {

otf_status otf_create(int device, void *hip_stream, otf_ctx **out) {
    if (!out) return OTF_E_INVALID;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        (void)hipGetLastError();
        return OTF_E_INVALID;
    }
    otf_ctx *ctx = new (std::nothrow) otf_ctx();
    if (!ctx) return OTF_E_NOMEM;
    ctx->c.device = device;
    ctx->c.stream = (hipStream_t)hip_stream;
    otf_status st = guard(ctx, false, [&] {
        ctx->c.counters.reserve(32);
        OTF_HIP(hipMemsetAsync(ctx->c.counters.p, 0, 32 * sizeof(uint32_t), ctx->c.stream));
        OTF_HIP(hipStreamSynchronize(ctx->c.stream));
        void *h = nullptr;
        OTF_HIP(hipHostMalloc(&h, 32 * sizeof(uint32_t), hipHostMallocMapped | hipHostMallocCoherent));
        ctx->c.h_counters = (uint32_t *)h;
        std::memset(h, 0, 32 * sizeof(uint32_t));
        void *d = nullptr;
        OTF_HIP(hipHostGetDevicePointer(&d, h, 0));
        ctx->c.d_h_counters = (uint32_t *)d;
        OTF_HIP(hipStreamCreateWithFlags(&ctx->c.side, hipStreamNonBlocking));
        OTF_HIP(hipEventCreateWithFlags(&ctx->c.ev_fork, hipEventDisableTiming));
        OTF_HIP(hipEventCreateWithFlags(&ctx->c.ev_join, hipEventDisableTiming));
    });
    if (st != OTF_OK) {
        otf_destroy(ctx);
        return st;
    }
    *out = ctx;
    return OTF_OK;
}

otf_status otf_destroy(otf_ctx *ctx) {
    if (!ctx) return OTF_E_INVALID;
    (void)hipSetDevice(ctx->c.device);
    (void)hipStreamSynchronize(ctx->c.stream);
    for (otf_batch *bt : std::vector<otf_batch *>(ctx->c.batches)) batch_forget(bt, &ctx->c);
    if (ctx->c.side) {
        (void)hipStreamSynchronize(ctx->c.side);
        (void)hipStreamDestroy(ctx->c.side);
    }
    if (ctx->c.capture) (void)hipStreamDestroy(ctx->c.capture);
    if (ctx->c.ev_fork) (void)hipEventDestroy(ctx->c.ev_fork);
    if (ctx->c.ev_join) (void)hipEventDestroy(ctx->c.ev_join);
    if (ctx->c.h_counters) (void)hipHostFree(ctx->c.h_counters);
    for (auto &e : ctx->c.ev_pool) (void)hipEventDestroy(e);
    delete ctx;
    return OTF_OK;
}

const char *otf_last_error(const otf_ctx *ctx) { return ctx ? ctx->c.err.c_str() : "null context"; }

// A batch member is swept, restructured and replaced only through its batch
// (the batch's table holds its store pointers).
static bool batch_member(otf_ctx *ctx) {
    if (ctx->c.batches.empty()) return false;
    ctx->c.err = "the context is a batch member: fuse it through the batch, or destroy the batch first";
    return true;
}

otf_status otf_build_octree(otf_ctx *ctx, const float *depth, int32_t depth_is_device, int32_t n_views,
                            const otf_camera *cams, const otf_params *prm) {
    if (!ctx) return OTF_E_INVALID;
    if (batch_member(ctx)) return OTF_E_STATE;
    return guard(ctx, true, [&] {
        Ctx &c = ctx->c;
        check_params(prm);
        if (!depth || !cams) fail(OTF_E_INVALID, "depth or cams is null");
        if (n_views < 1 || n_views > kMaxViews) fail(OTF_E_INVALID, "n_views must be in 1..64");
        std::vector<CamDev> cd(n_views);
        for (int v = 0; v < n_views; ++v) {
            const otf_camera &k = cams[v];
            if (k.width <= 0 || k.height <= 0 || k.width != cams[0].width || k.height != cams[0].height)
                fail(OTF_E_INVALID, "cameras must share one positive image size");
            const float *vals[] = {&k.fx, &k.fy, &k.cx, &k.cy};
            for (const float *q : vals)
                if (!std::isfinite(*q)) fail(OTF_E_INVALID, "non-finite intrinsics");
            for (int r = 0; r < 9; ++r)
                if (!std::isfinite(k.R_cw[r])) fail(OTF_E_INVALID, "non-finite rotation");
            for (int r = 0; r < 3; ++r)
                if (!std::isfinite(k.C[r])) fail(OTF_E_INVALID, "non-finite camera centre");
            cd[v] = CamDev{k.fx, k.fy, k.cx, k.cy, k.width, k.height, {}, {}};
            std::memcpy(cd[v].R, k.R_cw, sizeof(cd[v].R));
            std::memcpy(cd[v].C, k.C, sizeof(cd[v].C));
        }
        c.valid = false;
        c.prm = *prm;
        c.n_views = n_views;
        c.iteration = 0;
        c.coef = make_coef(prm->max_depth);
        c.last_splits = c.last_joins = 0;
        const size_t npix = (size_t)n_views * cams[0].width * cams[0].height;
        DBuf<float> dtmp;
        const float *ddev = depth;
        if (!depth_is_device) {
            dtmp.reserve(npix);
            OTF_HIP(hipMemcpyAsync(dtmp.p, depth, npix * sizeof(float), hipMemcpyHostToDevice, c.stream));
            ddev = dtmp.p;
        }
        build_views_and_union(c, ddev, cd);
        setup_after_structure(c, true);
        c.valid = true;
    });
}

namespace {
// Iterations recorded per graph when the structure is frozen.
constexpr int kFuseGraphChunk = 8;

// The device work of one frozen iteration (no restructure): the two sweeps,
// the flag totals and the observation totals, on c.stream.
void sweep_work(Ctx &c, const Solver &sol, float sigma, float tau, float tl) {
    if (sol.gd) {
        launch_gd_flux(c, sol.eps2);
        launch_gd_update(c, sol.lam, sol.xi, sol.eps2);
    } else {
        launch_dual(c, sigma);
        launch_primal(c, tau, tl);
    }
    count_flags(c);
    accumulate_obs(c, sol.gd != 0);
}

// Host bookkeeping of one iteration whose device work is already queued.
void sweep_books(Ctx &c) {
    c.iteration++;
    c.leaf_updates += c.L;
    count_sweep_bytes(c);
    c.last_splits = c.last_joins = 0;
}

// Records `chunk` frozen iterations into an executable graph. Run after an
// eager iteration of the same structure, so that every scratch buffer the
// sweeps use already has its size (nothing is allocated while recording).
hipGraphExec_t record_sweeps(Ctx &c, int chunk, const Solver &sol, float sigma, float tau, float tl) {
    if (!c.capture) OTF_HIP(hipStreamCreateWithFlags(&c.capture, hipStreamNonBlocking));
    hipStream_t own = c.stream;
    hipGraph_t g = nullptr;
    OTF_HIP(hipStreamBeginCapture(c.capture, hipStreamCaptureModeThreadLocal));
    c.stream = c.capture;
    try {
        for (int k = 0; k < chunk; ++k) sweep_work(c, sol, sigma, tau, tl);
    } catch (...) {
        c.stream = own;
        (void)hipStreamEndCapture(c.capture, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    c.stream = own;
    OTF_HIP(hipStreamEndCapture(c.capture, &g));
    hipGraphExec_t e = nullptr;
    const hipError_t r = hipGraphInstantiate(&e, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    OTF_HIP(r);
    return e;
}

// A frozen structure (restructure_every = 0) without kernel timing: one
// eager iteration, then chunks of kFuseGraphChunk iterations replayed from
// one recorded graph, then the rest eagerly. Returns the iterations done.
int fuse_frozen(Ctx &c, int iterations, float sigma, float tau, float tl) {
    const Solver sol = c.sol;
    sweep_work(c, sol, sigma, tau, tl);
    sweep_books(c);
    int done = 1;
    const int reps = (iterations - done) / kFuseGraphChunk;
    hipGraphExec_t e = record_sweeps(c, kFuseGraphChunk, sol, sigma, tau, tl);
    try {
        for (int r = 0; r < reps; ++r) {
            OTF_HIP(hipGraphLaunch(e, c.stream));
            for (int k = 0; k < kFuseGraphChunk; ++k) sweep_books(c);
        }
        OTF_HIP(hipStreamSynchronize(c.stream));
    } catch (...) {
        (void)hipStreamSynchronize(c.stream);
        (void)hipGraphExecDestroy(e);
        throw;
    }
    (void)hipGraphExecDestroy(e);
    done += reps * kFuseGraphChunk;
    c.graph_iterations = (int64_t)reps * kFuseGraphChunk;
    for (; done < iterations; ++done) {
        sweep_work(c, sol, sigma, tau, tl);
        sweep_books(c);
    }
    return done;
}

bool graph_replay_applies(const Ctx &c, int iterations) {
    return c.prm.restructure_every == 0 && !c.prof && c.log_every == 0 && iterations > 2 * kFuseGraphChunk;
}

// the per-iteration record of the state after an iteration (otf_log_every)
void log_iteration(Ctx &c) {
    if (c.log_every <= 0 || c.iteration % c.log_every != 0 || c.log_n >= c.log_cap) return;
    otf_iter_record r{};
    r.iteration = c.iteration;
    r.leaves = c.L;
    r.splits = c.last_splits;
    r.joins = c.last_joins;
    energy(c, &r.tv, &r.data);
    c.log_buf[c.log_n++] = r;
}
}  // namespace

otf_status otf_fuse(otf_ctx *ctx, int32_t iterations, float lambda, float tau, float sigma) {
    if (!ctx) return OTF_E_INVALID;
    if (batch_member(ctx)) return OTF_E_STATE;
    if (iterations < 0 || !std::isfinite(lambda) || !std::isfinite(tau) || !std::isfinite(sigma) || lambda < 0.0f ||
        !(tau > 0.0f) || !(sigma > 0.0f)) {
        ctx->c.err = "bad fuse arguments";
        return OTF_E_INVALID;
    }
    if (!ctx->c.valid) {
        ctx->c.err = "no valid state";
        return OTF_E_STATE;
    }
    return guard(ctx, true, [&] {
        Ctx &c = ctx->c;
        const float tl = tau * lambda;
        c.sol = Solver{};
        c.graph_iterations = 0;
        if (graph_replay_applies(c, iterations)) {
            fuse_frozen(c, iterations, sigma, tau, tl);
            finish(c);
            return;
        }
        prof_mark(c, -1);
        for (int it = 0; it < iterations; ++it) {
            c.iteration++;
            launch_dual(c, sigma);
            prof_mark(c, kProfDual);
            launch_primal(c, tau, tl);
            prof_mark(c, kProfPrimal);
            count_flags(c);
            c.leaf_updates += c.L;
            count_sweep_bytes(c);
            accumulate_obs(c);
            c.last_splits = c.last_joins = 0;
            // the flag totals and the restructure form one timed phase
            if (c.prm.restructure_every > 0 && c.iteration % c.prm.restructure_every == 0) {
                restructure(c, tl);
                prof_mark(c, kProfRestructure);
            } else {
                prof_mark(c, -1);
            }
            log_iteration(c);
        }
        c.prof_open = nullptr;
        finish(c);  // synchronises and checks the scan health flag
    });
}

otf_status otf_log_every(otf_ctx *ctx, int32_t k, otf_iter_record *records, int64_t capacity) {
    if (!ctx || k < 0 || capacity < 0 || (k > 0 && capacity > 0 && !records)) return OTF_E_INVALID;
    Ctx &c = ctx->c;
    c.log_every = capacity > 0 ? k : 0;
    c.log_buf = c.log_every > 0 ? records : nullptr;
    c.log_cap = c.log_every > 0 ? capacity : 0;
    c.log_n = 0;
    return OTF_OK;
}

otf_status otf_log_count(const otf_ctx *ctx, int64_t *n) {
    if (!ctx || !n) return OTF_E_INVALID;
    *n = ctx->c.log_n;
    return OTF_OK;
}

otf_status otf_fuse_gd(otf_ctx *ctx, int32_t iterations, float lambda, float step, float epsilon) {
    if (!ctx) return OTF_E_INVALID;
    if (batch_member(ctx)) return OTF_E_STATE;
    if (iterations < 0 || !std::isfinite(lambda) || !std::isfinite(step) || !std::isfinite(epsilon) ||
        lambda < 0.0f || !(step > 0.0f) || !(epsilon > 0.0f)) {
        ctx->c.err = "bad fuse arguments";
        return OTF_E_INVALID;
    }
    if (!ctx->c.valid) {
        ctx->c.err = "no valid state";
        return OTF_E_STATE;
    }
    return guard(ctx, true, [&] {
        Ctx &c = ctx->c;
        c.sol = Solver{1, lambda, step, epsilon * epsilon};
        c.graph_iterations = 0;
        if (graph_replay_applies(c, iterations)) {
            fuse_frozen(c, iterations, 0.0f, 1.0f, 0.0f);
            c.sol = Solver{};
            finish(c);
            return;
        }
        prof_mark(c, -1);
        for (int it = 0; it < iterations; ++it) {
            c.iteration++;
            launch_gd_flux(c, c.sol.eps2);
            prof_mark(c, kProfDual);
            launch_gd_update(c, c.sol.lam, c.sol.xi, c.sol.eps2);
            prof_mark(c, kProfPrimal);
            count_flags(c);
            c.leaf_updates += c.L;
            // same bytes as the primal-dual sweeps, with W in place of P for every observation
            count_sweep_bytes(c);
            accumulate_obs(c, true);
            c.last_splits = c.last_joins = 0;
            if (c.prm.restructure_every > 0 && c.iteration % c.prm.restructure_every == 0) {
                restructure(c, 0.0f);
                prof_mark(c, kProfRestructure);
            } else {
                prof_mark(c, -1);
            }
            log_iteration(c);
        }
        c.prof_open = nullptr;
        c.sol = Solver{};
        finish(c);
    });
}

otf_status otf_selftest_scan(otf_ctx *ctx, int64_t n, uint64_t seed, int64_t *mismatches) {
    if (!ctx || !mismatches || n < 0 || n > (int64_t(1) << 28)) return OTF_E_INVALID;
    return guard(ctx, false, [&] {
        Ctx &c = ctx->c;
        // inputs from splitmix64
        uint64_t st = seed;
        auto next = [&] {
            uint64_t z = (st += 0x9E3779B97F4A7C15ull);
            z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
            z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
            return z ^ (z >> 31);
        };
        std::vector<uint8_t> a(n), b(n), f(n), e(n);
        std::vector<uint32_t> x(n), y(n);
        for (int64_t i = 0; i < n; ++i) {
            const uint64_t r = next();
            a[i] = (uint8_t)(r & 3);
            b[i] = (uint8_t)((r >> 2) & 1);
            // join bits in runs: keep the previous value with probability 7/8
            const uint8_t jb = (uint8_t)(((r >> 3) & 3) << 1);
            f[i] = (uint8_t)((i > 0 && ((r >> 5) & 7) != 0 ? (f[i - 1] & 6) : jb) | ((r >> 8) & 1));
            x[i] = (uint32_t)((r >> 16) & 0xFFF);
            y[i] = (uint32_t)(r >> 40) & 0x3FF;
            e[i] = (uint8_t)(((r >> 60) & 7) == 0);  // sparse flags, 1 in 8
        }
        DBuf<uint8_t> da, db, df, de;
        DBuf<uint32_t> dx, dy, o1, o2, o3, o4, o5, o6, o7, l1, l2, l3, l4, t4;
        const int64_t m = n > 0 ? n : 1;
        da.reserve(m); db.reserve(m); df.reserve(m); de.reserve(m); dx.reserve(m); dy.reserve(m);
        for (DBuf<uint32_t> *o : {&o1, &o2, &o3, &o4, &o5, &o6, &o7, &l1, &l2, &l3, &l4}) o->reserve(m + 1);
        t4.reserve(4);
        upload(c, da.p, a);
        upload(c, db.p, b);
        upload(c, df.p, f);
        upload(c, de.p, e);
        upload(c, dx.p, x);
        upload(c, dy.p, y);
        scan_exclusive_u32_dev_u8(c, da.p, o1.p, n);
        scan_exclusive_pair_u8(c, da.p, o2.p, db.p, o3.p, n);
        scan_exclusive_pair_u32(c, dx.p, o4.p, dy.p, o5.p, n);
        scan_run_starts(c, df.p, o6.p, n);
        scan_exclusive_flag_bits(c, df.p, 1u, o7.p, n);
        // compaction: whole lists, a pair of them, and a list cut at half its length
        uint32_t nb = 0, ne = 0;
        for (int64_t i = 0; i < n; ++i) {
            nb += b[i];
            ne += e[i];
        }
        scan_compact_u8(c, de.p, l1.p, (uint32_t)m, t4.p, n);
        scan_compact_pair_u8(c, db.p, l2.p, (uint32_t)m, t4.p + 1, de.p, l3.p, (uint32_t)m, t4.p + 2, n);
        scan_compact_u8(c, db.p, l4.p, nb / 2, t4.p + 3, n);
        finish(c);
        auto g1 = download(c, o1.p, n + 1), g2 = download(c, o2.p, n + 1), g3 = download(c, o3.p, n + 1);
        auto g4 = download(c, o4.p, n + 1), g5 = download(c, o5.p, n + 1), g6 = download(c, o6.p, n);
        auto g7 = download(c, o7.p, n + 1);
        int64_t bad = 0;
        uint32_t sa = 0, sb = 0, sx = 0, sy = 0, sf = 0, run = 0;
        for (int64_t i = 0; i <= n; ++i) {
            bad += g1[i] != sa;
            bad += g2[i] != sa;
            bad += g3[i] != sb;
            bad += g4[i] != sx;
            bad += g5[i] != sy;
            bad += g7[i] != sf;
            if (i == n) break;
            const uint32_t j = f[i] & 6u;
            if (j && (i == 0 || (f[i - 1] & 6u) != j)) run = (uint32_t)i;
            bad += g6[i] != run;
            sa += a[i];
            sb += b[i];
            sx += x[i];
            sy += y[i];
            sf += f[i] & 1u;
        }
        auto h1 = download(c, l1.p, m), h2 = download(c, l2.p, m), h3 = download(c, l3.p, m);
        auto h4 = download(c, l4.p, m), ht = download(c, t4.p, 4);
        finish(c);
        bad += ht[0] != ne;
        bad += ht[1] != nb;
        bad += ht[2] != ne;
        bad += ht[3] != nb;
        uint32_t kb = 0, ke = 0;
        for (int64_t i = 0; i < n; ++i) {
            if (b[i]) {
                bad += h2[kb] != (uint32_t)i;
                if (kb < nb / 2) bad += h4[kb] != (uint32_t)i;
                ++kb;
            }
            if (e[i]) {
                bad += h1[ke] != (uint32_t)i;
                bad += h3[ke] != (uint32_t)i;
                ++ke;
            }
        }
        *mismatches = bad;
    });
}

otf_status otf_num_leaves(const otf_ctx *ctx, int64_t *n) {
    if (!ctx || !n) return OTF_E_INVALID;
    if (!ctx->c.valid) return OTF_E_STATE;
    *n = ctx->c.L;
    return OTF_OK;
}

otf_status otf_last_counts(const otf_ctx *ctx, int64_t *splits, int64_t *joins) {
    if (!ctx || !splits || !joins) return OTF_E_INVALID;
    *splits = ctx->c.last_splits;
    *joins = ctx->c.last_joins;
    return OTF_OK;
}

otf_status otf_obs_pool_stats(const otf_ctx *ctx, int64_t *used, int64_t *capacity, int64_t *compactions) {
    if (!ctx || !used || !capacity || !compactions) return OTF_E_INVALID;
    if (!ctx->c.valid) return OTF_E_STATE;
    const ObsPool &pool = ctx->c.obs[ctx->c.ocur];
    *used = pool.used;
    *capacity = pool.cap;
    *compactions = ctx->c.pool_compactions;
    return OTF_OK;
}

otf_status otf_extract(const otf_ctx *cctx, int64_t capacity, uint32_t *keys, uint8_t *levels, float *u, float *ubar,
                       float *p_xyz, int64_t *n_written) {
    otf_ctx *ctx = const_cast<otf_ctx *>(cctx);
    if (!ctx || !n_written || capacity < 0) return OTF_E_INVALID;
    if (!ctx->c.valid) return OTF_E_STATE;
    *n_written = ctx->c.L;
    if (capacity < ctx->c.L) return OTF_E_CAPACITY;
    return guard(ctx, false, [&] {
        Ctx &c = ctx->c;
        LeafStore &s = c.lv();
        const int64_t L = c.L;
        if (keys) OTF_HIP(hipMemcpyAsync(keys, s.key.p, L * 4, hipMemcpyDeviceToHost, c.stream));
        if (levels) OTF_HIP(hipMemcpyAsync(levels, s.level.p, L, hipMemcpyDeviceToHost, c.stream));
        if (u) OTF_HIP(hipMemcpyAsync(u, s.u.p, L * 4, hipMemcpyDeviceToHost, c.stream));
        if (ubar) OTF_HIP(hipMemcpyAsync(ubar, s.ubar.p, L * 4, hipMemcpyDeviceToHost, c.stream));
        if (p_xyz) {
            std::vector<float> h = download(c, s.p.p, 3 * s.cap);
            OTF_HIP(hipStreamSynchronize(c.stream));
            for (int64_t i = 0; i < L; ++i)
                for (int d = 0; d < 3; ++d) p_xyz[3 * i + d] = h[(size_t)d * s.cap + i];
        }
        OTF_HIP(hipStreamSynchronize(c.stream));
    });
}

otf_status otf_extract_obs(const otf_ctx *cctx, int64_t cap_leaves, int32_t *M, float *wtot, float *inv,
                           int64_t cap_obs, float *F, float *W, int64_t *n_obs) {
    otf_ctx *ctx = const_cast<otf_ctx *>(cctx);
    if (!ctx || !n_obs) return OTF_E_INVALID;
    if (!ctx->c.valid) return OTF_E_STATE;
    if (cap_leaves < ctx->c.L) return OTF_E_CAPACITY;
    otf_status cap_st = OTF_OK;
    otf_status st = guard(ctx, false, [&] {
        Ctx &c = ctx->c;
        LeafStore &s = c.lv();
        const int64_t L = c.L;
        auto hm = download(c, s.obs_m.p, L);
        auto hoff = download(c, s.obs_off.p, L);
        auto hw = download(c, s.wtot.p, L);
        auto hi = download(c, s.inv.p, L);
        const bool values = F || W;  // counts only: skip the pool download
        auto hF = download(c, c.op().F.p, values ? c.op().used : 0);
        auto hW = download(c, c.op().W.p, values ? c.op().used : 0);
        OTF_HIP(hipStreamSynchronize(c.stream));
        int64_t tot = 0;
        for (int64_t i = 0; i < L; ++i) tot += hm[i];
        *n_obs = tot;
        if (values && tot > cap_obs) {
            cap_st = OTF_E_CAPACITY;
            return;
        }
        int64_t j = 0;
        for (int64_t i = 0; i < L; ++i) {
            if (M) M[i] = hm[i];
            if (wtot) wtot[i] = hw[i];
            if (inv) inv[i] = hi[i];
            for (int k = 0; k < hm[i]; ++k, ++j) {
                if (F) F[j] = hF[hoff[i] + k];
                if (W) W[j] = hW[hoff[i] + k];
            }
        }
    });
    return st != OTF_OK ? st : cap_st;
}

otf_status otf_extract_obs_at(const otf_ctx *cctx, int64_t n, const int64_t *leaves, int32_t *M, float *wtot,
                              float *inv, int64_t cap_obs, float *F, float *W, int64_t *n_obs) {
    otf_ctx *ctx = const_cast<otf_ctx *>(cctx);
    if (!ctx || !n_obs || n < 0 || (n > 0 && !leaves)) return OTF_E_INVALID;
    if (!ctx->c.valid) return OTF_E_STATE;
    for (int64_t t = 0; t < n; ++t)
        if (leaves[t] < 0 || leaves[t] >= ctx->c.L) return OTF_E_INVALID;
    otf_status cap_st = OTF_OK;
    otf_status st = guard(ctx, false, [&] {
        Ctx &c = ctx->c;
        LeafStore &s = c.lv();
        std::vector<uint8_t> hm(n);
        std::vector<uint32_t> hoff(n);
        std::vector<float> hw(n), hi(n);
        for (int64_t t = 0; t < n; ++t) {  // one small copy per field and leaf
            const int64_t i = leaves[t];
            OTF_HIP(hipMemcpyAsync(&hm[t], s.obs_m.p + i, 1, hipMemcpyDeviceToHost, c.stream));
            OTF_HIP(hipMemcpyAsync(&hoff[t], s.obs_off.p + i, 4, hipMemcpyDeviceToHost, c.stream));
            OTF_HIP(hipMemcpyAsync(&hw[t], s.wtot.p + i, 4, hipMemcpyDeviceToHost, c.stream));
            OTF_HIP(hipMemcpyAsync(&hi[t], s.inv.p + i, 4, hipMemcpyDeviceToHost, c.stream));
        }
        OTF_HIP(hipStreamSynchronize(c.stream));
        int64_t tot = 0;
        for (int64_t t = 0; t < n; ++t) tot += hm[t];
        *n_obs = tot;
        const bool values = F || W;
        if (values && tot > cap_obs) {
            cap_st = OTF_E_CAPACITY;
            return;
        }
        int64_t j = 0;
        for (int64_t t = 0; t < n; ++t) {
            if (M) M[t] = hm[t];
            if (wtot) wtot[t] = hw[t];
            if (inv) inv[t] = hi[t];
            if (values && hm[t] > 0) {
                if (F) OTF_HIP(hipMemcpyAsync(F + j, c.op().F.p + hoff[t], 4 * hm[t], hipMemcpyDeviceToHost, c.stream));
                if (W) OTF_HIP(hipMemcpyAsync(W + j, c.op().W.p + hoff[t], 4 * hm[t], hipMemcpyDeviceToHost, c.stream));
            }
            j += hm[t];
        }
        OTF_HIP(hipStreamSynchronize(c.stream));
    });
    return st != OTF_OK ? st : cap_st;
}

otf_status otf_extract_neighbours(const otf_ctx *cctx, int64_t cap_leaves, int32_t *counts, int64_t cap_idx,
                                  int64_t *idx, int64_t *n_idx) {
    otf_ctx *ctx = const_cast<otf_ctx *>(cctx);
    if (!ctx || !n_idx) return OTF_E_INVALID;
    if (!ctx->c.valid) return OTF_E_STATE;
    if (cap_leaves < ctx->c.L) return OTF_E_CAPACITY;
    otf_status cap_st = OTF_OK;
    otf_status st = guard(ctx, false, [&] {
        Ctx &c = ctx->c;
        LeafStore &s = c.lv();
        const int64_t L = c.L;
        auto op = download(c, s.nbp_off.p, L + 1);
        auto om = download(c, s.nbm_off.p, L + 1);
        auto ep = download(c, s.nbp.p, s.n_nbp);
        auto em = download(c, s.nbm.p, s.n_nbm);
        OTF_HIP(hipStreamSynchronize(c.stream));
        *n_idx = s.n_nbp + s.n_nbm;
        if (*n_idx > cap_idx) {
            cap_st = OTF_E_CAPACITY;
            return;
        }
        int64_t j = 0;
        for (int64_t i = 0; i < L; ++i) {
            int32_t cnt[6] = {0, 0, 0, 0, 0, 0};
            for (int side = 0; side < 2; ++side) {
                const auto &off = side ? om : op;
                const auto &ent = side ? em : ep;
                for (int d = 0; d < 3; ++d)
                    for (uint32_t e = off[i]; e < off[i + 1]; ++e)
                        if ((int)((ent[e] >> kIdxBits) & 3u) == d) {
                            cnt[3 * side + d]++;
                            if (idx) idx[j] = ent[e] & kIdxMask;
                            ++j;
                        }
            }
            if (counts)
                for (int f = 0; f < 6; ++f) counts[6 * i + f] = cnt[f];
        }
    });
    return st != OTF_OK ? st : cap_st;
}

otf_status otf_energy(otf_ctx *ctx, double *tv, double *data) {
    if (!ctx || !tv || !data) return OTF_E_INVALID;
    if (!ctx->c.valid) return OTF_E_STATE;
    return guard(ctx, false, [&] {
        prof_begin(ctx->c);
        energy(ctx->c, tv, data);
        prof_end(ctx->c, kProfEnergy);
    });
}

otf_status otf_debug_corrupt_adjacency(otf_ctx *ctx, int64_t leaf) {
#ifdef OTF_DEBUG_BOUNDS
    if (!ctx || leaf < 0) return OTF_E_INVALID;
    if (!ctx->c.valid) return OTF_E_STATE;
    if (leaf >= ctx->c.L) return OTF_E_INVALID;
    return guard(ctx, false, [&] {
        Ctx &c = ctx->c;
        LeafStore &s = c.lv();
        uint32_t off[2];
        OTF_HIP(hipMemcpy(off, s.nbp_off.p + leaf, sizeof off, hipMemcpyDeviceToHost));
        if (off[1] == off[0]) fail(OTF_E_INVALID, "the leaf has no + neighbour");
        uint32_t e = 0;
        OTF_HIP(hipMemcpy(&e, s.nbp.p + off[0], sizeof e, hipMemcpyDeviceToHost));
        e = (e & ~kIdxMask) | (uint32_t)(c.L + 1);  // past the last leaf, inside the index field
        OTF_HIP(hipMemcpy(s.nbp.p + off[0], &e, sizeof e, hipMemcpyHostToDevice));
    });
#else
    (void)leaf;
    if (ctx) ctx->c.err = "only the bounds-checked build corrupts an adjacency entry";
    return OTF_E_INVALID;
#endif
}

otf_status otf_debug_poke_guard(otf_ctx *ctx) {
#ifdef OTF_DEBUG_BOUNDS
    if (!ctx) return OTF_E_INVALID;
    if (!ctx->c.valid) return OTF_E_STATE;
    // not through guard(): the damage is for the next call to find
    LeafStore &s = ctx->c.lv();
    if (hipSetDevice(ctx->c.device) != hipSuccess || hipDeviceSynchronize() != hipSuccess) {
        (void)hipGetLastError();
        return OTF_E_DEVICE;
    }
    const uint8_t b = (uint8_t)(kGuardByte ^ 0xFF);
    char *zone = reinterpret_cast<char *>(s.nbp.p) + s.nbp.n * sizeof(uint32_t);
    if (hipMemcpy(zone + 3, &b, 1, hipMemcpyHostToDevice) != hipSuccess) {
        (void)hipGetLastError();
        return OTF_E_DEVICE;
    }
    return OTF_OK;
#else
    if (ctx) ctx->c.err = "only the bounds-checked build has guard zones";
    return OTF_E_INVALID;
#endif
}

otf_status otf_debug_unwritten_slot(otf_ctx *ctx) {
#ifdef OTF_DEBUG_BOUNDS
    if (!ctx) return OTF_E_INVALID;
    if (!ctx->c.valid) return OTF_E_STATE;
    ctx->c.debug_unwritten_slot = true;
    return OTF_OK;
#else
    if (ctx) ctx->c.err = "only the bounds-checked build checks the adjacency slots";
    return OTF_E_INVALID;
#endif
}

otf_status otf_debug_fail_allocations(otf_ctx *ctx, int64_t after) {
    if (!ctx || after < 0) return OTF_E_INVALID;
    ctx->c.fail_alloc_after = after;
    return OTF_OK;
}

otf_status otf_energy_noalloc(otf_ctx *ctx, double *tv, double *data) {
    if (!ctx || !tv || !data) return OTF_E_INVALID;
    if (!ctx->c.valid) return OTF_E_STATE;
    return guard(ctx, false, [&] { energy_noalloc(ctx->c, tv, data); });
}

otf_status otf_energy_eps(otf_ctx *ctx, double epsilon, double *tv, double *data) {
    if (!ctx || !tv || !data || !std::isfinite(epsilon) || !(epsilon > 0.0)) return OTF_E_INVALID;
    if (!ctx->c.valid) return OTF_E_STATE;
    return guard(ctx, false, [&] {
        prof_begin(ctx->c);
        energy(ctx->c, tv, data, epsilon);
        prof_end(ctx->c, kProfEnergy);
    });
}

otf_status otf_dense_field(otf_ctx *ctx, float *out, int32_t out_is_device, int64_t capacity) {
    if (!ctx || !out) return OTF_E_INVALID;
    if (!ctx->c.valid) return OTF_E_STATE;
    const int64_t n = int64_t(1) << (3 * ctx->c.prm.max_depth);
    if (capacity < n) {
        ctx->c.err = "capacity below (2^max_depth)^3";
        return OTF_E_CAPACITY;
    }
    return guard(ctx, false, [&] {
        Ctx &c = ctx->c;
        if (out_is_device) {
            dense_field(c, out);
            OTF_HIP(hipStreamSynchronize(c.stream));
        } else {
            DBuf<float> d;
            d.reserve((size_t)n);
            dense_field(c, d.p);
            OTF_HIP(hipMemcpyAsync(out, d.p, sizeof(float) * n, hipMemcpyDeviceToHost, c.stream));
            OTF_HIP(hipStreamSynchronize(c.stream));
        }
    });
}

otf_status otf_mesh(otf_ctx *ctx, float iso, int64_t capacity, float *xyz, uint64_t *edges, int64_t *n_tris) {
    if (!ctx || !n_tris || capacity < 0 || !std::isfinite(iso)) return OTF_E_INVALID;
    if (!ctx->c.valid) return OTF_E_STATE;
    otf_status cap_st = OTF_OK;
    otf_status st = guard(ctx, false, [&] {
        const int64_t n = marching_cubes(ctx->c, iso, capacity, xyz, reinterpret_cast<unsigned long long *>(edges));
        *n_tris = n;
        if (n > capacity || (n > 0 && (!xyz || !edges))) cap_st = OTF_E_CAPACITY;
    });
    return st != OTF_OK ? st : cap_st;
}

otf_status otf_quantisation_error(otf_ctx *ctx, const float *dense, int32_t dense_is_device, double *err) {
    if (!ctx || !dense || !err) return OTF_E_INVALID;
    if (!ctx->c.valid) return OTF_E_STATE;
    return guard(ctx, false, [&] {
        Ctx &c = ctx->c;
        if (dense_is_device) {
            *err = quantisation_error(c, dense);
        } else {
            const int64_t n = int64_t(1) << (3 * c.prm.max_depth);
            DBuf<float> d;
            d.reserve((size_t)n);
            OTF_HIP(hipMemcpyAsync(d.p, dense, sizeof(float) * n, hipMemcpyHostToDevice, c.stream));
            *err = quantisation_error(c, d.p);
        }
    });
}

otf_status otf_export_state(const otf_ctx *cctx, void *buf, int64_t cap, int64_t *n_bytes) {
    otf_ctx *ctx = const_cast<otf_ctx *>(cctx);
    if (!ctx || !n_bytes || cap < 0) return OTF_E_INVALID;
    if (!ctx->c.valid) return OTF_E_STATE;
    otf_status cap_st = OTF_OK;
    otf_status st = guard(ctx, false, [&] {
        Ctx &c = ctx->c;
        const ViewStore &vs = c.views;
        auto hk = download(c, vs.key.p, vs.n_nodes);
        auto hl = download(c, vs.level.p, vs.n_nodes);
        auto hS = download(c, vs.S.p, vs.n_nodes);
        auto hc = download(c, vs.cnt.p, vs.n_nodes);
        auto hch = download(c, vs.child.p, vs.n_nodes);
        LeafStore &s = c.lv();
        const int64_t L = c.L;
        auto lk = download(c, s.key.p, L);
        auto ll = download(c, s.level.p, L);
        auto lu = download(c, s.u.p, L);
        auto lb = download(c, s.ubar.p, L);
        auto lp = download(c, s.p.p, 3 * s.cap);
        OTF_HIP(hipStreamSynchronize(c.stream));
        Writer w{(uint8_t *)buf, cap};
        w.put("OTF1", 4);
        uint32_t ver = 1;
        w.put(&ver, 4);
        w.put(&c.prm, sizeof(otf_params));
        w.put(&c.iteration, 8);
        int32_t nv = c.n_views, zero = 0;
        w.put(&nv, 4);
        w.put(&zero, 4);
        for (int v = 0; v < c.n_views; ++v) {
            int64_t nn = vs.count[v];
            w.put(&nn, 8);
            for (int64_t q = 0; q < nn; ++q) {
                const int64_t i = vs.base[v] + q;
                NodeRec r{hk[i], hl[i], (uint8_t)(hch[i] == kNone ? 1 : 0), 0, hS[i], hc[i]};
                w.put(&r, sizeof r);
            }
        }
        w.put(&L, 8);
        for (int64_t i = 0; i < L; ++i) {
            LeafRec r{lk[i], ll[i], {0, 0, 0}, {lu[i], lb[i], lp[i], lp[s.cap + i], lp[2 * s.cap + i]}};
            w.put(&r, sizeof r);
        }
        *n_bytes = w.n;
        if (buf && w.n > cap) cap_st = OTF_E_CAPACITY;
    });
    return st != OTF_OK ? st : cap_st;
}

otf_status otf_import_state(otf_ctx *ctx, const void *buf, int64_t n_bytes) {
    if (!ctx || !buf || n_bytes < 0) return OTF_E_INVALID;
    if (batch_member(ctx)) return OTF_E_STATE;
    return guard(ctx, true, [&] {
        Ctx &c = ctx->c;
        Reader r{(const uint8_t *)buf, n_bytes};
        char magic[4];
        uint32_t ver;
        otf_params prm;
        int64_t iter;
        int32_t nv, zero;
        r.get(magic, 4);
        r.get(&ver, 4);
        r.get(&prm, sizeof prm);
        r.get(&iter, 8);
        r.get(&nv, 4);
        r.get(&zero, 4);
        if (std::memcmp(magic, "OTF1", 4) != 0 || ver != 1) fail(OTF_E_INVALID, "bad blob header");
        check_params(&prm);
        if (nv < 1 || nv > kMaxViews) fail(OTF_E_INVALID, "bad view count");
        const int D = prm.max_depth;
        // view trees: rebuild child links from (level, key) order
        std::vector<uint32_t> key, cnt, child;
        std::vector<uint8_t> level;
        std::vector<float> S;
        std::vector<int64_t> count(nv), base(nv);
        for (int v = 0; v < nv; ++v) {
            int64_t nn;
            r.get(&nn, 8);
            if (nn < 1 || nn > (int64_t)0x7FFFFFFF) fail(OTF_E_INVALID, "bad view node count");
            base[v] = (int64_t)key.size();
            count[v] = nn;
            std::vector<NodeRec> recs((size_t)nn);
            r.get(recs.data(), nn * (int64_t)sizeof(NodeRec));
            int64_t next_child = 1;  // position (within the view) of the next unassigned child group
            for (int64_t q = 0; q < nn; ++q) {
                const NodeRec &nr = recs[q];
                if (q == 0 && (nr.level != 0 || nr.key != 0)) fail(OTF_E_INVALID, "view root");
                if (nr.level > D) fail(OTF_E_INVALID, "view node level");
                uint32_t ch = kNone;
                if (!nr.leaf) {
                    if (nr.level >= D || next_child + 8 > nn) fail(OTF_E_INVALID, "inconsistent view tree");
                    const int sh = 3 * (D - nr.level - 1);
                    for (int k = 0; k < 8; ++k) {
                        const NodeRec &cr = recs[next_child + k];
                        if (cr.level != nr.level + 1 || cr.key != (nr.key | ((uint32_t)k << sh)))
                            fail(OTF_E_INVALID, "inconsistent view tree");
                    }
                    ch = (uint32_t)(base[v] + next_child);
                    next_child += 8;
                }
                key.push_back(nr.key);
                level.push_back(nr.level);
                S.push_back(nr.S);
                cnt.push_back(nr.cnt);
                child.push_back(ch);
            }
            if (next_child != nn) fail(OTF_E_INVALID, "inconsistent view tree");
        }
        int64_t nl;
        r.get(&nl, 8);
        if (nl < 1 || nl >= kLeafLimit) fail(OTF_E_INVALID, "bad leaf count");
        if (prm.max_leaves > 0 && nl > prm.max_leaves) fail(OTF_E_CAPACITY, "leaves exceed max_leaves");
        std::vector<LeafRec> lr((size_t)nl);
        r.get(lr.data(), nl * (int64_t)sizeof(LeafRec));
        uint64_t next = 0;
        for (int64_t i = 0; i < nl; ++i) {
            if (lr[i].level > D) fail(OTF_E_INVALID, "leaf level");
            const uint64_t size = uint64_t(1) << (3 * (D - lr[i].level));
            if (lr[i].key != next || (lr[i].key & (size - 1)) != 0) fail(OTF_E_INVALID, "leaves do not tile the domain");
            next = (uint64_t)lr[i].key + size;
        }
        if (next != (uint64_t(1) << (3 * D))) fail(OTF_E_INVALID, "leaves do not tile the domain");
        // commit
        c.valid = false;
        c.prm = prm;
        c.n_views = nv;
        c.iteration = iter;
        c.coef = make_coef(D);
        c.last_splits = c.last_joins = 0;
        ViewStore &vs = c.views;
        vs.n_nodes = (int64_t)key.size();
        vs.count = count;
        vs.base = base;
        vs.S.reserve(vs.n_nodes);
        vs.cnt.reserve(vs.n_nodes);
        vs.child.reserve(vs.n_nodes);
        vs.key.reserve(vs.n_nodes);
        vs.level.reserve(vs.n_nodes);
        upload(c, vs.S.p, S);
        upload(c, vs.cnt.p, cnt);
        upload(c, vs.child.p, child);
        upload(c, vs.key.p, key);
        upload(c, vs.level.p, level);
        std::vector<uint32_t> roots(nv);
        for (int v = 0; v < nv; ++v) roots[v] = (uint32_t)base[v];
        vs.root.reserve(nv);
        upload(c, vs.root.p, roots);
        c.cur = 0;
        c.L = nl;
        LeafStore &s = c.lv();
        s.reserve(nl);
        std::vector<uint32_t> lk(nl);
        std::vector<uint8_t> ll(nl);
        std::vector<float> lu(nl), lb(nl), lp(3 * s.cap, 0.0f);
        for (int64_t i = 0; i < nl; ++i) {
            lk[i] = lr[i].key;
            ll[i] = lr[i].level;
            lu[i] = lr[i].v[0];
            lb[i] = lr[i].v[1];
            for (int d = 0; d < 3; ++d) lp[(size_t)d * s.cap + i] = lr[i].v[2 + d];
        }
        upload(c, s.key.p, lk);
        upload(c, s.level.p, ll);
        upload(c, s.u.p, lu);
        upload(c, s.ubar.p, lb);
        upload(c, s.p.p, lp);
        OTF_HIP(hipStreamSynchronize(c.stream));
        setup_after_structure(c, false);
        c.valid = true;
    });
}

otf_status otf_fuse_graph_iterations(const otf_ctx *ctx, int64_t *n) {
    if (!ctx || !n) return OTF_E_INVALID;
    *n = ctx->c.graph_iterations;
    return OTF_OK;
}

otf_status otf_profile(otf_ctx *ctx, int32_t enable) {
    if (!ctx) return OTF_E_INVALID;
    return guard(ctx, false, [&] {
        Ctx &c = ctx->c;
        prof_collect(c);
        c.prof = enable != 0;
        for (int k = 0; k < kProfKinds; ++k) {
            c.prof_ms[k] = 0.0;
            c.prof_n[k] = 0;
        }
        c.leaf_updates = 0;
        for (double &b : c.alg_bytes) b = 0.0;
        hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(64), 0, c.stream, c.counters.p + 16, 2);
        OTF_HIP(hipStreamSynchronize(c.stream));
    });
}

otf_status otf_profile_read(otf_ctx *ctx, double *ms, int64_t *launches, int64_t *leaf_updates, double *bytes) {
    if (!ctx) return OTF_E_INVALID;
    return guard(ctx, false, [&] {
        Ctx &c = ctx->c;
        prof_collect(c);
        for (int k = 0; k < kProfSolverKinds; ++k) {
            if (ms) ms[k] = c.prof_ms[k];
            if (launches) launches[k] = c.prof_n[k];
        }
        if (leaf_updates) *leaf_updates = c.leaf_updates;
        if (bytes) {
            read_back(c, {{c.counters.p + 16, 16}, {c.counters.p + 17, 17}});
            unsigned long long obs_acc;
            std::memcpy(&obs_acc, c.h_counters + 16, 8);
            bytes[0] = c.alg_bytes[0];
            bytes[1] = c.alg_bytes[1] + 4.0 * (double)obs_acc;
            bytes[2] = c.alg_bytes[2];
            bytes[3] = c.alg_bytes[3] + 4.0 * (double)obs_acc;
        }
    });
}

otf_status otf_profile_read_eval(otf_ctx *ctx, double *ms, int64_t *launches) {
    if (!ctx) return OTF_E_INVALID;
    return guard(ctx, false, [&] {
        Ctx &c = ctx->c;
        prof_collect(c);
        for (int k = 0; k < kProfKinds - kProfSolverKinds; ++k) {
            if (ms) ms[k] = c.prof_ms[kProfSolverKinds + k];
            if (launches) launches[k] = c.prof_n[kProfSolverKinds + k];
        }
    });
}

}  // extern "C"
