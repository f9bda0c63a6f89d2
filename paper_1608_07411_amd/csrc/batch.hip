// C ABI of batches: the sweeps of many fused octrees in the same launches,
// a small autotuner for the sweep launch shape, and HIP-graph replay of the
// iteration loop when no member restructures.
//
// Every member keeps its own store, observations and split/join; a batch
// iteration is one primal-dual iteration of every member, bit-identical to
// otf_fuse on the member alone (per-leaf arithmetic does not depend on the
// tiling or the launch shape).
#include <array>
#include <algorithm>
#include <cmath>
#include <new>

#include "otf_internal.h"

using namespace otf;

struct otf_batch {
    int device = 0;
    hipStream_t stream = nullptr;
    BatchState b;
    std::string err;
    // table state
    bool table_ok = false;
    float up_sigma = 0.0f, up_tau = 0.0f, up_tl = 0.0f;
    // autotuner: one real iteration per candidate launch shape, timed with
    // events around the sweeps, normalised by the leaves swept
    std::vector<BatchConfig> cands;
    std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
    std::vector<double> cand_leaves;
    size_t next = 0;
    bool tuned = false;
    // graph of a chunk of iterations (members that never restructure)
    hipGraphExec_t exec = nullptr;
    hipStream_t capture = nullptr;  // private stream the graph is recorded on (the caller's may be the null stream)
    int graph_iters = 0;
    // what the recorded launches baked in: the table's device buffers and
    // the launch sizes (a change of any of them records the graph again)
    std::array<uintptr_t, 12> graph_key{};
    int last_graph_iters = 0;
    ~otf_batch() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (capture) (void)hipStreamDestroy(capture);
        for (auto &e : ev) {
            (void)hipEventDestroy(e.first);
            (void)hipEventDestroy(e.second);
        }
    }
};

namespace {

constexpr int kGraphChunk = 16;

template <class F>
otf_status bguard(otf_batch *bt, F &&f) {
    if (hipSetDevice(bt->device) != hipSuccess) {
        (void)hipGetLastError();
        bt->err = "hipSetDevice failed";
        return OTF_E_DEVICE;
    }
    try {
        f();
        bt->err.clear();
        return OTF_OK;
    } catch (const Failure &e) {
        bt->err = e.msg;
        if (e.st != OTF_E_INVALID)
            for (Ctx *c : bt->b.objs) c->valid = false;  // member states are unspecified after a failed iteration
        return e.st;
    } catch (const std::bad_alloc &) {
        bt->err = "host allocation failed";
        for (Ctx *c : bt->b.objs) c->valid = false;
        return OTF_E_NOMEM;
    } catch (...) {
        bt->err = "unexpected failure";
        for (Ctx *c : bt->b.objs) c->valid = false;
        return OTF_E_DEVICE;
    }
}

void ensure_table(otf_batch *bt, float sigma, float tau, float tl) {
    if (bt->table_ok && bt->up_sigma == sigma && bt->up_tau == tau && bt->up_tl == tl) return;
    batch_upload(bt->stream, bt->b, sigma, tau, tl);
    bt->table_ok = true;
    bt->up_sigma = sigma;
    bt->up_tau = tau;
    bt->up_tl = tl;
}

// Host side of one iteration for every member (counts, then split/join where
// due); returns whether any member restructured.
bool after_sweeps(otf_batch *bt, float tl) {
    bool changed = false;
    for (Ctx *c : bt->b.objs) {
        c->iteration++;
        c->leaf_updates += c->L;
        count_sweep_bytes(*c);
        c->last_splits = c->last_joins = 0;
        if (c->prm.restructure_every > 0 && c->iteration % c->prm.restructure_every == 0) {
            restructure(*c, tl);
            changed = true;
        }
    }
    return changed;
}

void finish_tuning(otf_batch *bt) {
    OTF_HIP(hipStreamSynchronize(bt->stream));
    double best = 0.0;
    size_t arg = 0;
    for (size_t k = 0; k < bt->cands.size(); ++k) {
        float ms = 0.0f;
        OTF_HIP(hipEventElapsedTime(&ms, bt->ev[k].first, bt->ev[k].second));
        const double per_leaf = (double)ms / std::max(1.0, bt->cand_leaves[k]);
        if (k == 0 || per_leaf < best) {
            best = per_leaf;
            arg = k;
        }
    }
    bt->b.cfg = bt->cands[arg];
    bt->tuned = true;
    bt->table_ok = false;  // tiles depend on the block size
}

std::array<uintptr_t, 12> graph_key(const otf_batch *bt) {
    const BatchState &b = bt->b;
    return {(uintptr_t)b.table.p,    (uintptr_t)b.tile_obj.p, (uintptr_t)b.tile_begin.p, (uintptr_t)b.part.p,
            (uintptr_t)b.hp_begin.p, (uintptr_t)b.hm_begin.p, (uintptr_t)b.coefs.p,     (uintptr_t)b.ntiles,
            (uintptr_t)b.n_hp,       (uintptr_t)b.n_hm,       (uintptr_t)b.cfg.blk,     (uintptr_t)b.cfg.grid};
}

void build_graph(otf_batch *bt, int iters) {
    if (bt->exec) {
        OTF_HIP(hipGraphExecDestroy(bt->exec));
        bt->exec = nullptr;
    }
    // recording runs nothing; the graph is launched on the batch's stream
    if (!bt->capture) OTF_HIP(hipStreamCreateWithFlags(&bt->capture, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    OTF_HIP(hipStreamBeginCapture(bt->capture, hipStreamCaptureModeThreadLocal));
    try {
        for (int k = 0; k < iters; ++k) batch_sweeps(bt->capture, bt->b);
    } catch (...) {
        (void)hipStreamEndCapture(bt->capture, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    OTF_HIP(hipStreamEndCapture(bt->capture, &g));
    const hipError_t e = hipGraphInstantiate(&bt->exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    OTF_HIP(e);
    bt->graph_iters = iters;
    bt->graph_key = graph_key(bt);
}

}  // namespace

extern "C" {

otf_status otf_batch_create(int device, void *hip_stream, otf_batch **out) {
    if (!out) return OTF_E_INVALID;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        (void)hipGetLastError();
        return OTF_E_INVALID;
    }
    otf_batch *bt = new (std::nothrow) otf_batch();
    if (!bt) return OTF_E_NOMEM;
    bt->device = device;
    bt->stream = (hipStream_t)hip_stream;
    for (int blk : {128, 256, 512})
        for (int grid : {0, 1024, 4096}) bt->cands.push_back(BatchConfig{blk, grid});
    *out = bt;
    return OTF_OK;
}

otf_status otf_batch_destroy(otf_batch *bt) {
    if (!bt) return OTF_E_INVALID;
    (void)hipSetDevice(bt->device);
    (void)hipStreamSynchronize(bt->stream);
    for (Ctx *c : bt->b.objs) c->batches.erase(std::remove(c->batches.begin(), c->batches.end(), bt), c->batches.end());
    delete bt;
    return OTF_OK;
}


otf_status otf_batch_add(otf_batch *bt, otf_ctx *ctx) {
    if (!bt || !ctx) return OTF_E_INVALID;
    if (ctx->c.device != bt->device || ctx->c.stream != bt->stream) {
        bt->err = "a member must use the batch's device and stream";
        return OTF_E_INVALID;
    }
    if (!ctx->c.valid) {
        bt->err = "the context holds no octree";
        return OTF_E_STATE;
    }
    for (Ctx *c : bt->b.objs)
        if (c == &ctx->c) {
            bt->err = "the context is already a member";
            return OTF_E_INVALID;
        }
    return bguard(bt, [&] {
        bt->b.objs.push_back(&ctx->c);
        ctx->c.batches.push_back(bt);
        bt->table_ok = false;
        if (bt->exec) {
            OTF_HIP(hipGraphExecDestroy(bt->exec));
            bt->exec = nullptr;
        }
    });
}

otf_status otf_batch_fuse(otf_batch *bt, int32_t iterations, float lambda, float tau, float sigma) {
    if (!bt) return OTF_E_INVALID;
    if (iterations < 0 || !std::isfinite(lambda) || !std::isfinite(tau) || !std::isfinite(sigma) || lambda < 0.0f ||
        !(tau > 0.0f) || !(sigma > 0.0f)) {
        bt->err = "bad fuse arguments";
        return OTF_E_INVALID;
    }
    for (Ctx *c : bt->b.objs)
        if (!c->valid) {
            bt->err = "a member holds no valid state";
            return OTF_E_STATE;
        }
    if (bt->b.objs.empty() || iterations == 0) return OTF_OK;
    return bguard(bt, [&] {
        const float tl = tau * lambda;
        bool frozen = true;
        for (Ctx *c : bt->b.objs) frozen = frozen && c->prm.restructure_every == 0;
        int it = 0;
        bt->last_graph_iters = 0;
        while (it < iterations) {
            if (!bt->tuned) {
                const size_t k = bt->next;
                if (bt->ev.size() < bt->cands.size()) {
                    hipEvent_t a, b;
                    OTF_HIP(hipEventCreate(&a));
                    OTF_HIP(hipEventCreate(&b));
                    bt->ev.push_back({a, b});
                    bt->cand_leaves.push_back(0.0);
                }
                bt->b.cfg = bt->cands[k];
                bt->table_ok = false;
                ensure_table(bt, sigma, tau, tl);
                double leaves = 0.0;
                for (Ctx *c : bt->b.objs) leaves += (double)c->L;
                bt->cand_leaves[k] = leaves;
                OTF_HIP(hipEventRecord(bt->ev[k].first, bt->stream));
                batch_sweeps(bt->stream, bt->b);
                OTF_HIP(hipEventRecord(bt->ev[k].second, bt->stream));
                if (after_sweeps(bt, tl)) bt->table_ok = false;
                ++it;
                if (++bt->next == bt->cands.size()) finish_tuning(bt);
                continue;
            }
            if (frozen) {
                ensure_table(bt, sigma, tau, tl);
                const int reps = (iterations - it) / kGraphChunk;  // the rest (< kGraphChunk) runs eagerly
                if (reps > 0) {
                    if (!bt->exec || bt->graph_key != graph_key(bt)) build_graph(bt, kGraphChunk);
                    for (int r = 0; r < reps; ++r) {
                        OTF_HIP(hipGraphLaunch(bt->exec, bt->stream));
                        for (int k = 0; k < kGraphChunk; ++k) after_sweeps(bt, tl);
                    }
                    it += reps * kGraphChunk;
                    bt->last_graph_iters += reps * kGraphChunk;
                    continue;
                }
            }
            ensure_table(bt, sigma, tau, tl);
            batch_sweeps(bt->stream, bt->b);
            if (after_sweeps(bt, tl)) bt->table_ok = false;
            ++it;
        }
        for (Ctx *c : bt->b.objs) finish(*c);  // synchronises and checks each member's scan health
    });
}

otf_status otf_batch_config(const otf_batch *bt, int32_t *block, int32_t *grid, int32_t *tuned,
                            int32_t *graph_iterations) {
    if (!bt) return OTF_E_INVALID;
    if (block) *block = bt->b.cfg.blk;
    if (grid) *grid = bt->b.cfg.grid;
    if (tuned) *tuned = bt->tuned ? 1 : 0;
    if (graph_iterations) *graph_iterations = bt->last_graph_iters;
    return OTF_OK;
}

const char *otf_batch_last_error(const otf_batch *bt) { return bt ? bt->err.c_str() : "null batch"; }

}  // extern "C"

namespace otf {
void batch_forget(otf_batch *bt, Ctx *c) {
    (void)hipStreamSynchronize(bt->stream);
    bt->b.objs.erase(std::remove(bt->b.objs.begin(), bt->b.objs.end(), c), bt->b.objs.end());
    bt->table_ok = false;
    if (bt->exec) {
        (void)hipGraphExecDestroy(bt->exec);
        bt->exec = nullptr;
    }
}
}  // namespace otf
