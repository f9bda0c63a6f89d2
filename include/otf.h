/*
 * otf.h -- C ABI of the octree TV-L1 range-data fusion library (libotf.so,
 * HIP for gfx950 / MI355X).
 *
 * Method: Kehl, Holl, Tombari, Ilic, Navab, "An Octree-Based Approach towards
 * Efficient Variational Range Data Fusion", BMVC 2016. Range maps become
 * per-view truncated signed distance octrees (Sec. 3.1, Eq. 1-2); their union
 * seeds one fused octree whose leaf values minimise the normalised TV-L1
 * energy (Sec. 3.2, Eq. 3 and Eq. 5) while leaves split and join as the
 * solution evolves (Sec. 3.2, split and join rules). The minimiser is the
 * primal-dual scheme the paper names as an alternative solver (Sec. 5):
 * dual ascent with projection onto the unit ball, divergence, and a per-leaf
 * generalised shrinkage (weighted median) over the leaf's observations.
 *
 * Conventions for every entry point:
 *   - returns otf_status; no C++ exception ever crosses this boundary;
 *   - arguments are validated before any device work (OTF_E_INVALID);
 *   - pointers marked "host" are plain host memory owned by the caller and only
 *     read or written during the call; pointers marked "device" are device
 *     memory on the context's device, owned by the caller;
 *   - the context owns every device buffer it allocates and frees them in
 *     otf_destroy; device work is issued on the stream given at creation,
 *     except that a restructuring step (otf_fuse, otf_fuse_gd with split/join)
 *     runs its new leaves' observation fetch on a second stream that the
 *     context creates (default priority) and joins back into the given stream
 *     with an event before anything reads the result, and a frozen-structure
 *     fuse records a graph on a third stream of its own (nothing runs there;
 *     see otf_fuse_graph_iterations); every entry point returns after its
 *     work on these streams has finished;
 *   - after a failure other than OTF_E_INVALID the fused state is unspecified
 *     and OTF_E_STATE is returned by fuse/extract/energy/export until the next
 *     successful build or import; the context can always be destroyed;
 *   - one context per host thread; contexts share no mutable state;
 *   - a context that is a member of a batch (below) refuses otf_fuse,
 *     otf_fuse_gd, otf_build_octree and otf_import_state with OTF_E_STATE.
 *
 * Geometry: the reconstruction domain is the unit cube [0,1]^3 split into
 * G^3 finest voxels, G = 2^max_depth. A leaf at level L has side
 * s = 2^(max_depth - L) finest voxels; its key is the Morton code of its
 * minimum-corner finest voxel with x in bit 0, y in bit 1, z in bit 2 of each
 * bit triple. Leaves are always kept sorted by key.
 */
#ifndef OTF_H
#define OTF_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct otf_ctx otf_ctx;

typedef enum {
    OTF_OK = 0,
    OTF_E_INVALID = 1,  /* bad argument; nothing was changed */
    OTF_E_NOMEM = 2,    /* a device or host allocation failed */
    OTF_E_CAPACITY = 3, /* leaf count would exceed max_leaves, or a caller buffer is too small */
    OTF_E_DEVICE = 4,   /* a HIP call failed */
    OTF_E_STATE = 5     /* no valid fused state (not built, or a previous call failed) */
} otf_status;

/* Pinhole camera of one range map (Sec. 3.1: the projection pi_i and centre
 * C_i). OpenCV axes: x right, y down, z forward. Pixel (i, j) covers
 * [i, i+1) x [j, j+1); a point with camera coordinates (X, Y, Z), Z > 0,
 * projects to u = fx X/Z + cx, v = fy Y/Z + cy. 72 bytes. */
typedef struct {
    float fx, fy, cx, cy;
    int32_t width, height;
    float R_cw[9]; /* row-major camera->world rotation; columns are the camera axes in world space */
    float C[3];    /* projection centre in world coordinates */
} otf_camera;

/* Construction and restructuring parameters. 40 bytes. */
typedef struct {
    int32_t max_depth;         /* D_max (Sec. 3.1), 1..10 */
    float delta;               /* truncation band of Eq. 1, world units, > 0 */
    float eta;                 /* observation cut-off (Sec. 3.1: voxels with phi < -eta are unseen), >= delta */
    float spread_tau;          /* spread threshold of the construction (Sec. 3.1, 0.1 in the paper);
                                  < 0 refines every observed node to max_depth */
    float gamma;               /* normaliser offset of Eq. 5, > 0 */
    float split_tau, join_tau; /* tau_s, tau_j of the split and join rules (Sec. 3.2); split_tau <= join_tau;
                                  split_tau = 0 never splits, join_tau > 1 never joins (Sec. 4.2) */
    int32_t restructure_every; /* restructure after iteration t when t % restructure_every == 0; 0 = never */
    int64_t max_leaves;        /* leaf capacity limit; 0 = none below the 2^26 index limit and device memory */
} otf_params;

/* Create a context on HIP device `device`. `hip_stream` is a hipStream_t
 * borrowed for the context's lifetime (NULL = the null stream). */
otf_status otf_create(int device, void *hip_stream, otf_ctx **out);
otf_status otf_destroy(otf_ctx *ctx);

/* Build the fused octree from n_views range maps (Sec. 3.1 and the initial
 * structure of Fig. 1).
 *   depth: n_views * H * W floats, row-major per view, the radial range along
 *          each pixel-centre ray (Eq. 1 subtracts the Euclidean distance to
 *          C_i); 0, negative, NaN or infinite = no measurement. Host memory
 *          if depth_is_device == 0, else device memory.
 *   cams:  n_views cameras (host), all of the same width and height.
 *   prm:   parameters (host).
 * Per view: the TSDF of Eq. 1 at every finest voxel centre, observed iff the
 * voxel is in front of the camera, inside the image, the pixel is valid and
 * phi >= -eta; the view octree keeps a node's children iff it is above
 * max_depth, some voxel below is observed and the spread of Eq. 2 over the
 * observed voxels exceeds spread_tau; every stored node keeps the sum and
 * count of its observed voxels (the upward means). The fused octree starts as
 * the union of the view structures; each leaf gathers, per view, the node at
 * its own level or else the deepest view leaf containing it (Fig. 4):
 * F = sum/count, W = count/volume; W = 0 observations are dropped. The start
 * value is sum W F / (sum W + gamma), the dual variable starts at 0.
 * 1 <= n_views <= 64. Replaces any previous state. */
otf_status otf_build_octree(otf_ctx *ctx, const float *depth, int32_t depth_is_device, int32_t n_views,
                            const otf_camera *cams, const otf_params *prm);

/* Run `iterations` primal-dual iterations (Sec. 3.2 energy, Sec. 5 solver):
 *   p  <- P_unit( p + sigma * G ubar )          (forward differences, Sec. 3.2)
 *   u' =  u + tau * div p                        (div = -G^T, volume weighted)
 *   u+ =  argmin_v (v-u')^2/(2 tau) + lambda/(sum W + gamma) * sum_i W_i |v - F_i|
 *   ubar = 2 u+ - u,  u = u+
 * then split and join (Sec. 3.2) when the iteration count says so.
 * lambda >= 0 weights the normalised data term; tau > 0, sigma > 0 are the
 * primal and dual steps (tau * sigma * 12 <= 1 guarantees convergence on a
 * fixed structure). All finite. */
otf_status otf_fuse(otf_ctx *ctx, int32_t iterations, float lambda, float tau, float sigma);

/* Iterations of the last otf_fuse or otf_fuse_gd call that were replayed from
 * a recorded HIP graph. With restructure_every = 0 (a frozen structure),
 * kernel timing off (otf_profile) and more than 16 iterations, a call runs
 * one iteration as usual, records the device work of 8 iterations (the two
 * sweeps and their flag and observation totals) into a graph once, launches
 * that graph for as many whole chunks as remain and runs the rest as usual:
 * fewer host launches per iteration, identical results. *n = 0 otherwise.
 * The graph is recorded on a capture stream of the library's own (default
 * priority; recording runs nothing), launched on the context's stream and
 * destroyed before the call returns. */
otf_status otf_fuse_graph_iterations(const otf_ctx *ctx, int64_t *n);

/* Number of leaves of the fused octree. */
otf_status otf_num_leaves(const otf_ctx *ctx, int64_t *n);

/* Copy the leaves, in key order, into host buffers of `capacity` entries
 * (p_xyz: 3 floats per leaf, x y z). Any output pointer may be NULL. If
 * capacity is too small returns OTF_E_CAPACITY with *n_written = leaf count. */
otf_status otf_extract(const otf_ctx *ctx, int64_t capacity, uint32_t *keys, uint8_t *levels, float *u, float *ubar,
                       float *p_xyz, int64_t *n_written);

/* Inspection: every leaf's observations (Fig. 4 fetch), host buffers.
 * M[i], wtot[i] = sum W, inv[i] = 1/(sum W + gamma) per leaf (cap_leaves
 * entries); F and W concatenated in leaf order, each leaf's sorted by
 * (F, view) (cap_obs entries). *n_obs receives the total; OTF_E_CAPACITY if
 * a buffer is too small. */
otf_status otf_extract_obs(const otf_ctx *ctx, int64_t cap_leaves, int32_t *M, float *wtot, float *inv,
                           int64_t cap_obs, float *F, float *W, int64_t *n_obs);
/* The same for the listed leaves only (indices into the current leaf order,
 * host array of n): M[n], wtot[n], inv[n] and the segments one after another
 * in F / W (host, cap_obs floats; *n_obs = their total, always set).
 * Errors: OTF_E_INVALID (null, or an index out of range), OTF_E_STATE,
 * OTF_E_CAPACITY (cap_obs too small). */
otf_status otf_extract_obs_at(const otf_ctx *ctx, int64_t n, const int64_t *leaves, int32_t *M, float *wtot,
                              float *inv, int64_t cap_obs, float *F, float *W, int64_t *n_obs);

/* Inspection: face adjacency. counts: 6 per leaf for faces +x,+y,+z,-x,-y,-z;
 * idx: neighbour leaf indices concatenated in that order, ascending key
 * within a face. Host buffers; OTF_E_CAPACITY if idx is too small. */
otf_status otf_extract_neighbours(const otf_ctx *ctx, int64_t cap_leaves, int32_t *counts, int64_t cap_idx,
                                  int64_t *idx, int64_t *n_idx);

/* Energy of Eq. 3 with the normaliser of Eq. 5 (lambda on the data term):
 * tv = sum_n vol_n |(G u)_n|, data = sum_n vol_n/(sum W + gamma) sum_i W_i |u_n - F_i|;
 * E = tv + lambda * data. Accumulated in double. */
otf_status otf_energy(otf_ctx *ctx, double *tv, double *data);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the energy
 * of otf_energy, bit for bit, computed without any allocation. Its block
 * partial sums and totals live in a static device array of the library
 * (4 MiB per device, held until the process ends; enough for the 2^26-leaf
 * limit). Every call on one device shares that array, so calls that overlap
 * on one device race; no call leaves anything in it that a later call reads.
 * Errors: OTF_E_INVALID (null), OTF_E_STATE (no state), OTF_E_CAPACITY (more
 * leaves than the array holds), OTF_E_DEVICE. */
otf_status otf_energy_noalloc(otf_ctx *ctx, double *tv, double *data);

/* Per-iteration metrics: the state after one iteration of otf_fuse or
 * otf_fuse_gd, the measures the paper tracks over its runs (the leaf count
 * of Fig. 9, the split and join counts of section 3.3, the energy of Eq. 3). */
typedef struct otf_iter_record {
    int64_t iteration; /* the context's iteration count after it */
    int64_t leaves;    /* leaves after its restructure */
    int64_t splits;    /* leaves split by its restructure (0 without one) */
    int64_t joins;     /* collapses of its restructure (0 without one) */
    double tv, data;   /* as otf_energy, of the state after it */
} otf_iter_record;

/* Arms the per-iteration log: after every iteration of later otf_fuse /
 * otf_fuse_gd calls whose iteration count is a multiple of k, one record is
 * written to records[n] (host memory owned by the caller, which must stay
 * valid while armed) and n is counted up, until n reaches capacity. Each
 * record costs one energy reduction and a synchronisation; while armed, the
 * solver calls do not replay recorded graphs. A new call restarts n at 0;
 * k = 0 or capacity = 0 disarms. Errors: OTF_E_INVALID (null context, k < 0,
 * capacity < 0, null records with k and capacity above 0). */
otf_status otf_log_every(otf_ctx *ctx, int32_t k, otf_iter_record *records, int64_t capacity);

/* Records written since the log was armed. Errors: OTF_E_INVALID (null). */
otf_status otf_log_count(const otf_ctx *ctx, int64_t *n);

/* Splits and joins made by the last restructuring step of the last fuse. */
otf_status otf_last_counts(const otf_ctx *ctx, int64_t *splits, int64_t *joins);

/* Observation pool of the fetched data (Fig. 4) in device memory: entries in
 * use (live segments plus the garbage of replaced leaves; new leaves' segments
 * are appended), entries reserved, and the number of compactions made by
 * restructuring steps so far (a restructure compacts the pool in leaf order
 * when the appended segments would not fit or the garbage exceeds the live
 * entries). Errors: OTF_E_INVALID (null), OTF_E_STATE (no state). */
otf_status otf_obs_pool_stats(const otf_ctx *ctx, int64_t *used, int64_t *capacity, int64_t *compactions);

/* State blob (little-endian, version 1): "OTF1", u32 version, otf_params,
 * i64 iteration, i32 n_views, i32 0; per view i64 n_nodes then n_nodes records
 * {u32 key, u8 level, u8 is_leaf, u16 0, f32 sum, u32 count} in (level, key)
 * order; i64 n_leaves then records {u32 key, u8 level, u8[3] 0, f32 u, ubar,
 * px, py, pz} in key order. Export writes at most cap bytes into host memory
 * and always sets *n_bytes to the size needed (buf may be NULL to query). */
otf_status otf_export_state(const otf_ctx *ctx, void *buf, int64_t cap, int64_t *n_bytes);
otf_status otf_import_state(otf_ctx *ctx, const void *buf, int64_t n_bytes);

/* Per-kernel timing with HIP events recorded on the context's stream around
 * every launch of the solver kernels while enabled (adds event overhead).
 * Kinds: 0 dual sweep, 1 primal sweep, 2 restructure (all its kernels,
 * including the observation gather and the adjacency rebuild), 3 energy.
 * otf_profile_read fills ms[4] (summed milliseconds) and launches[4], and
 * leaf_updates (sum over iterations of the leaf count) and bytes[4], summed
 * over the iterations: [0] and [1] the bytes the dual and the primal sweep
 * move as implemented (level bytes, the divergence hand-over, flags and the
 * whole observation header included); [2] and [3] the method's own bytes of
 * one leaf sweep, per leaf-update 40 (u, ubar and p read and written) + 4 per
 * face-adjacency entry + 8 (observation offset and normaliser) + 4 per
 * observation value + 4 per prefix weight of a leaf with fractional weights,
 * attributed to the dual ([2]: ubar and p read, p written, the + list) and
 * the primal ([3]: the rest). Any pointer may be NULL. */
otf_status otf_profile(otf_ctx *ctx, int32_t enable);
otf_status otf_profile_read(otf_ctx *ctx, double *ms, int64_t *launches, int64_t *leaf_updates, double *bytes);

/* The evaluation's kernels timed the same way while otf_profile is enabled
 * (Sec. 3.2 meshing, Eq. 7): ms[4] (summed milliseconds) and launches[4] for
 * 0 the finest-grid field kernel of otf_dense_field, otf_mesh and
 * otf_quantisation_error, 1 the Eq. 7 kernels, 2 the marching-cubes count
 * kernel, 3 the marching-cubes emit kernel. Reset by otf_profile; either
 * pointer may be NULL. */
otf_status otf_profile_read_eval(otf_ctx *ctx, double *ms, int64_t *launches);

/* Self-test of the device prefix scans every compaction above relies on:
 * n pseudo-random elements (splitmix64 from seed) are scanned on the context's
 * device (exclusive sums of bytes and of words, two scans sharing a launch,
 * the max-scan of join-run starts, the sum of flag bits) and compared with the
 * same scans on the host; *mismatches is the number of differing outputs
 * (0: all equal). Needs no fused state. Errors: OTF_E_INVALID (null, n < 0 or
 * n > 2^28), OTF_E_NOMEM, OTF_E_DEVICE. */
otf_status otf_selftest_scan(otf_ctx *ctx, int64_t n, uint64_t seed, int64_t *mismatches);

/* Test hook: the after-th device allocation made by later calls on this
 * context fails as if the device were out of memory, so that the call returns
 * OTF_E_NOMEM (after = 0 turns the hook off; it fires once). The context stays
 * destroyable and frees everything it holds; a failed fuse leaves no valid
 * state (OTF_E_STATE until the next build or import). Errors: OTF_E_INVALID
 * (null, after < 0). */
otf_status otf_debug_fail_allocations(otf_ctx *ctx, int64_t after);

/* Test hook of the bounds-checked build (compiled with OTF_DEBUG_BOUNDS, where
 * the sweeps check every adjacency range, neighbour index, level code and
 * observation index they read, redirect a bad read to index 0 and report it:
 * the solver call then fails with OTF_E_DEVICE): points the first + entry of
 * `leaf` past the last leaf, so that the next fuse must report it. The
 * default build rejects it with OTF_E_INVALID and changes nothing. Errors:
 * OTF_E_INVALID (null, leaf out of range, no + neighbour, default build),
 * OTF_E_STATE. */
otf_status otf_debug_corrupt_adjacency(otf_ctx *ctx, int64_t leaf);

/* Test hook of the bounds-checked build, where every device buffer is followed
 * by a guard zone of known bytes (checked when the buffer is freed and after
 * every call on a context: a changed byte fails that call with OTF_E_DEVICE,
 * naming where the buffer was reserved), and every adjacency slot is checked
 * after each neighbour search (one that no search wrote, or that holds an
 * index past the last leaf or a level past the maximum depth, fails the call
 * the same way). Changes one byte of the guard zone after the current +
 * adjacency list, so that the next call on the context must report it. The
 * default build rejects it with OTF_E_INVALID and changes nothing. Errors:
 * OTF_E_INVALID (null, default build), OTF_E_STATE (no octree),
 * OTF_E_DEVICE. */
otf_status otf_debug_poke_guard(otf_ctx *ctx);

/* Test hook of the bounds-checked build: the next neighbour search (a build,
 * an import, or the restructure of a solver call) leaves the first + slot as
 * if no search had written it, so that its adjacency check must fail that
 * call with OTF_E_DEVICE before any kernel reads the slot. The default build
 * rejects it with OTF_E_INVALID and changes nothing. Errors: OTF_E_INVALID
 * (null, default build), OTF_E_STATE (no octree). */
otf_status otf_debug_unwritten_slot(otf_ctx *ctx);

/* Message of the last failure on this context (empty if none). Valid until the
 * next call on the context. */
const char *otf_last_error(const otf_ctx *ctx);

/* ---------------------------------------------------------------------------
 * Evaluation (Sec. 3.2, the final meshing step; Sec. 4, Eq. 7).
 * ------------------------------------------------------------------------- */

/* u resampled to the finest grid: out[(z G + y) G + x] = u of the leaf that
 * contains voxel (x, y, z), G = 2^max_depth. `out` holds `capacity` floats,
 * on the device if out_is_device (the context's device) else on the host.
 * Errors: OTF_E_INVALID (null out), OTF_E_STATE, OTF_E_CAPACITY (capacity <
 * G^3; nothing written). */
otf_status otf_dense_field(otf_ctx *ctx, float *out, int32_t out_is_device, int64_t capacity);

/* Marching cubes on the finest-grid field at `iso` (0: the fused surface).
 * Cells join 8 voxel centres; every cell edge whose end values straddle iso
 * (one below, one not) carries a vertex, linearly interpolated; the cell's
 * triangles come from a case table derived from face segments (an ambiguous
 * face separates its inside corners), so the mesh is closed away from the
 * domain boundary. Triangle t: xyz[9t .. 9t+8] its vertices in world
 * coordinates, edges[3t .. 3t+2] their grid edges, 3 ((z G + y) G + x) + axis
 * of the edge's lower voxel (equal ids = the same vertex). Host arrays of
 * `capacity` triangles; *n_tris = the count. Errors: OTF_E_INVALID,
 * OTF_E_STATE, OTF_E_CAPACITY (capacity too small or null arrays; *n_tris is
 * set, nothing copied). Needs 4 bytes of device memory per finest voxel. */
otf_status otf_mesh(otf_ctx *ctx, float iso, int64_t capacity, float *xyz, uint64_t *edges, int64_t *n_tris);

/* Eq. 7: sum over leaves n of |u(n) - mean of `dense` over the finest voxels
 * of n|, in double; `dense` is a finest-grid field laid out as in
 * otf_dense_field (for example a fully refined solve's), on the device if
 * dense_is_device else on the host. Errors: OTF_E_INVALID, OTF_E_STATE. */
otf_status otf_quantisation_error(otf_ctx *ctx, const float *dense, int32_t dense_is_device, double *err);

/* ---------------------------------------------------------------------------
 * Learned warm start, for callers that fuse many similar scenes: a per-leaf
 * network predicts the change from the initial to the converged u, and the
 * converged p, of the primal-dual iteration (Sec. 3.2) from each leaf's
 * sorted observations (Fig. 4 fetch) and its face neighbours, and the
 * iteration starts from that prediction.
 *
 * Network: 32 features -> 128 -> 128 -> 128 -> 4 outputs (change of u, px,
 * py, pz),
 * ReLU on hidden layers; bfloat16 weights and activations (fp32 rounded to
 * nearest, ties to even), fp32 accumulation on the matrix cores, fp32 biases
 * and master weights; loss: mean squared error over rows and outputs;
 * optimiser: Adam (beta 0.9, 0.999, eps 1e-8). Parameters: per layer W (in x
 * out, row-major) then b, otf_mlp_num_params() floats.
 * Features of a leaf: 16 quantiles F[floor((2k+1) M / 32)] of its sorted
 * observations (0 if M = 0), the mean u of its neighbours across each face
 * (+x, +y, +z, -x, -y, -z; 0 without neighbours), u, W/(W + gamma), M/64,
 * level/max_depth, then zeros.
 * Device arrays below are on the network's (context's) device, row-major.
 * ------------------------------------------------------------------------- */
typedef struct otf_mlp otf_mlp;

/* Create a network (parameters 0) on `device` and `hip_stream` (borrowed). */
otf_status otf_mlp_create(int device, void *hip_stream, otf_mlp **out);
otf_status otf_mlp_destroy(otf_mlp *net);
int64_t otf_mlp_num_params(void);
/* Host fp32 parameter vector of exactly otf_mlp_num_params() floats; setting
 * resets the optimiser state. Errors: OTF_E_INVALID (null or wrong size). */
otf_status otf_mlp_set_params(otf_mlp *net, const float *params, int64_t n);
otf_status otf_mlp_get_params(otf_mlp *net, float *params, int64_t n);
/* Y (rows x 4, device) = network(X (rows x 32, device)). */
otf_status otf_mlp_forward(otf_mlp *net, const float *X, int64_t rows, float *Y);
/* Loss against T (rows x 4, device) and its gradient (host, num_params
 * floats, may be null); parameters unchanged. */
otf_status otf_mlp_gradient(otf_mlp *net, const float *X, const float *T, int64_t rows, float *grad, double *loss);
/* One Adam step with learning rate lr > 0 on the loss over these rows. */
otf_status otf_mlp_train_step(otf_mlp *net, const float *X, const float *T, int64_t rows, float lr, double *loss);
const char *otf_mlp_last_error(const otf_mlp *net);
/* Features (L x 32) and current (u, px, py, pz) (L x 4) of the context's
 * leaves into device arrays of cap_rows rows. Errors: OTF_E_INVALID,
 * OTF_E_STATE, OTF_E_CAPACITY (cap_rows < leaves). */
otf_status otf_features(otf_ctx *ctx, float *X, int64_t cap_rows);
otf_status otf_leaf_targets(otf_ctx *ctx, float *T, int64_t cap_rows);
/* Every leaf's u (and ubar) becomes u + output 0 clamped to [-1, 1], its p
 * outputs 1..3 projected onto the unit ball. The network must use the
 * context's device and stream (else OTF_E_INVALID). */
otf_status otf_warm_start(otf_ctx *ctx, otf_mlp *net);
/* The warm start guarded by the energy of the plain method. From the current state (u0,
 * ubar0, p0) the prediction is applied at each step alpha in alphas[0..n_alpha)
 * (u = u0 + alpha * output 0 kept in [-1, 1], ubar = u, p = (1 - alpha) p0 +
 * alpha * the projected outputs 1..3), the energy E = tv + lambda * data of
 * Eq. 3 (as otf_energy) is evaluated for each, and the state with the lowest
 * energy is kept; when none is lower than the current state's, the current
 * state stays (alpha 0). *alpha_used and *energy_used receive the choice and
 * its energy. Every candidate costs one energy evaluation (a sweep and a
 * host read-back). Errors: OTF_E_INVALID (null pointer, n_alpha outside
 * 1..8, an alpha outside (0, 1], lambda negative or not finite, network on
 * another device or stream), OTF_E_STATE (no valid state). */
otf_status otf_warm_start_guarded(otf_ctx *ctx, otf_mlp *net, float lambda, int32_t n_alpha, const float *alphas,
                                 float *alpha_used, double *energy_used);

/* ---------------------------------------------------------------------------
 * The paper's own solver (Sec. 3.2, Eq. 4-6): explicit gradient descent to
 * the steady state of the PDE of Eq. 6, on the energy of Eq. 5 with both
 * terms smoothed as in Eq. 4 (Gamma(x^2) = sqrt(x^2 + epsilon^2)) and lambda
 * on the TV term:
 *   E(u) = sum_n vol_n [ sum_i W_i Gamma((u_n - F_i)^2) / (sum_i W_i + gamma)
 *                        + lambda Gamma(|(Gu)_n|^2) ],
 *   u <- u + step (lambda div(Gu / Gamma(|Gu|^2)) - d'(u)),
 *   d'(u) = sum_i W_i (u - F_i) / Gamma((u - F_i)^2) / (sum_i W_i + gamma),
 * with G and div the same unequal-leaf operators as otf_fuse, Jacobi phases
 * (every flux from the current u, then every update), and split/join after
 * each step as in otf_fuse, a split child taking its parent's step with its
 * own data term. The paper runs 100 steps, the step 0.1 halved every 20; the
 * caller does that by calling this function in chunks.
 * ------------------------------------------------------------------------- */

/* `iterations` descent steps. Errors: OTF_E_INVALID (iterations < 0, a
 * non-finite argument, lambda < 0, step <= 0 or epsilon <= 0; nothing ran),
 * OTF_E_STATE (no octree), otherwise as otf_fuse. */
otf_status otf_fuse_gd(otf_ctx *ctx, int32_t iterations, float lambda, float step, float epsilon);

/* The smoothed terms of the gradient-descent energy in double:
 * tv = sum_n vol_n Gamma(|(Gu)_n|^2), data = sum_n vol_n inv_n sum_i W_i
 * Gamma((u_n - F_i)^2); the energy is data + lambda tv. Errors: OTF_E_INVALID
 * (null outputs, epsilon not finite or <= 0), OTF_E_STATE. */
otf_status otf_energy_eps(otf_ctx *ctx, double epsilon, double *tv, double *data);

/* ---------------------------------------------------------------------------
 * Batches: the primal-dual iterations (Sec. 3.2, Eq. 5; the primal-dual
 * scheme of Chambolle and Pock that Sec. 5 names) of many fused octrees in
 * the same kernel launches, for callers that fuse many objects at once
 * (octrees of different depths and view counts).
 *
 * A batch borrows its member contexts: each keeps its own octree,
 * observations and split/join parameters, and a batch iteration performs one
 * iteration of every member, with results bit-identical to otf_fuse on each
 * member alone. Members must have been created with the batch's device and
 * stream and hold a built or imported octree. While a context is a member,
 * otf_fuse, otf_fuse_gd, otf_build_octree and otf_import_state on it return
 * OTF_E_STATE (the batch holds its store pointers); destroying a member
 * removes it from its batches, and destroying a batch releases its members.
 * Inspection calls (otf_extract, otf_energy, ...) on members are allowed
 * between batch calls.
 *
 * The first iterations of a batch double as an autotuner: each runs the
 * sweeps with another launch shape (threads per block and persistent grid
 * size) and the fastest per leaf is kept (otf_batch_config). When no member
 * restructures (restructure_every == 0), whole chunks of 16 iterations are
 * captured once in a HIP graph and replayed.
 * ------------------------------------------------------------------------- */
typedef struct otf_batch otf_batch;

/* Create an empty batch on `device` and `hip_stream` (borrowed; may be null,
 * the default stream). Errors: OTF_E_INVALID (bad device or null out). */
otf_status otf_batch_create(int device, void *hip_stream, otf_batch **out);

/* Destroy the batch (not its members). */
otf_status otf_batch_destroy(otf_batch *batch);

/* Add a member. Errors: OTF_E_INVALID (another device or stream, or already a
 * member), OTF_E_STATE (no octree in the context). */
otf_status otf_batch_add(otf_batch *batch, otf_ctx *ctx);

/* `iterations` primal-dual iterations of every member, arguments as
 * otf_fuse. An empty batch or zero iterations does nothing. Errors:
 * OTF_E_INVALID (arguments; nothing ran), OTF_E_STATE (a member has no valid
 * state), OTF_E_CAPACITY / OTF_E_NOMEM / OTF_E_DEVICE (a member's split/join
 * or the device failed; every member's state is then unspecified, as after a
 * failed otf_fuse). */
otf_status otf_batch_fuse(otf_batch *batch, int32_t iterations, float lambda, float tau, float sigma);

/* The sweep launch shape in use: threads per block (leaves per tile), grid
 * blocks (0: one per tile), whether the autotuner has finished, and how many
 * iterations of the last otf_batch_fuse were graph replays. Any output may be
 * null. */
otf_status otf_batch_config(const otf_batch *batch, int32_t *block, int32_t *grid, int32_t *tuned,
                            int32_t *graph_iterations);

/* Message of the batch's last failed call. */
const char *otf_batch_last_error(const otf_batch *batch);

#ifdef __cplusplus
}
#endif

#endif /* OTF_H */
