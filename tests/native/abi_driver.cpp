// Drives the library's host-side argument validation through the C ABI, for
// a build of the library's host code under AddressSanitizer and
// UndefinedBehaviorSanitizer: every entry point with a null context, network
// or batch, null outputs and out-of-range arguments, and context creation on
// a machine without a usable device. Each must return an error status without
// touching a device. Exits non-zero on an unexpected status; the sanitizers
// report any memory or undefined-behaviour error. Test infrastructure only.
#include <cmath>
#include <cstdio>

#include "otf.h"

static int failures = 0;

static void expect(bool ok, const char *what) {
    if (!ok) {
        std::fprintf(stderr, "unexpected status: %s\n", what);
        ++failures;
    }
}

#define INVALID(call) expect((call) == OTF_E_INVALID, #call)

int main() {
    int64_t n = 0;
    double d0 = 0.0, d1 = 0.0;
    float f = 0.0f;
    otf_camera cam{};
    otf_params prm{};
    INVALID(otf_create(0, nullptr, nullptr));
    otf_ctx *ctx = nullptr;
    const otf_status st = otf_create(0, nullptr, &ctx);  // no usable device here: an error, no context
    expect(st != OTF_OK || ctx != nullptr, "otf_create");
    if (st == OTF_OK) otf_destroy(ctx);
    expect(otf_destroy(nullptr) == OTF_OK || otf_destroy(nullptr) == OTF_E_INVALID, "otf_destroy(null)");
    INVALID(otf_build_octree(nullptr, &f, 0, 1, &cam, &prm));
    INVALID(otf_fuse(nullptr, 1, 0.5f, 0.3f, 0.3f));
    INVALID(otf_fuse_gd(nullptr, 1, 0.5f, 0.1f, 0.3f));
    INVALID(otf_num_leaves(nullptr, &n));
    INVALID(otf_last_counts(nullptr, &n, &n));
    INVALID(otf_extract(nullptr, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr));
    INVALID(otf_extract_obs(nullptr, 0, nullptr, nullptr, nullptr, 0, nullptr, nullptr, nullptr));
    INVALID(otf_extract_obs_at(nullptr, 0, nullptr, nullptr, nullptr, nullptr, 0, nullptr, nullptr, nullptr));
    INVALID(otf_extract_neighbours(nullptr, 0, nullptr, 0, nullptr, nullptr));
    INVALID(otf_obs_pool_stats(nullptr, &n, &n, &n));
    INVALID(otf_energy(nullptr, &d0, &d1));
    INVALID(otf_energy_noalloc(nullptr, &d0, &d1));
    INVALID(otf_energy_eps(nullptr, 0.3, &d0, &d1));
    INVALID(otf_export_state(nullptr, nullptr, 0, &n));
    INVALID(otf_import_state(nullptr, &f, 4));
    INVALID(otf_profile(nullptr, 1));
    INVALID(otf_profile_read(nullptr, nullptr, nullptr, nullptr, nullptr));
    INVALID(otf_selftest_scan(nullptr, 0, 0, &n));
    INVALID(otf_dense_field(nullptr, &f, 0, 1));
    INVALID(otf_mesh(nullptr, 0.0f, 0, nullptr, nullptr, &n));
    INVALID(otf_quantisation_error(nullptr, &f, 0, &d0));
    INVALID(otf_features(nullptr, &f, 1));
    INVALID(otf_leaf_targets(nullptr, &f, 1));
    INVALID(otf_warm_start(nullptr, nullptr));
    INVALID(otf_warm_start_guarded(nullptr, nullptr, 0.5f, 1, nullptr, nullptr, nullptr));
    INVALID(otf_debug_fail_allocations(nullptr, 1));
    INVALID(otf_debug_corrupt_adjacency(nullptr, 0));
    INVALID(otf_batch_create(0, nullptr, nullptr));
    INVALID(otf_batch_add(nullptr, nullptr));
    INVALID(otf_batch_fuse(nullptr, 1, 0.5f, 0.3f, 0.3f));
    INVALID(otf_mlp_create(0, nullptr, nullptr));
    INVALID(otf_mlp_set_params(nullptr, &f, 1));
    INVALID(otf_mlp_get_params(nullptr, &f, 1));
    INVALID(otf_mlp_forward(nullptr, &f, 1, &f));
    expect(otf_last_error(nullptr) != nullptr, "otf_last_error(null)");
    expect(otf_mlp_num_params() > 0, "otf_mlp_num_params");
    if (failures) return 1;
    std::printf("abi driver ok\n");
    return 0;
}
