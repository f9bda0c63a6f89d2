/* Drives the CPU oracle through its whole C interface on small synthetic
 * volumes, for a build under AddressSanitizer and UndefinedBehaviorSanitizer:
 * build, primal-dual iterations with split and join, gradient-descent
 * iterations, energies, extraction, adjacency, the state round trip, a
 * corrupt blob and invalid arguments. Exits non-zero on an unexpected status;
 * the sanitizers report any memory or undefined-behaviour error. Test
 * infrastructure only. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

typedef struct orc orc;
typedef struct {
    int32_t max_depth;
    float delta, eta, spread_tau, gamma, split_tau, join_tau;
    int32_t restructure_every;
    int64_t max_leaves;
} params_t;

orc *orc_create(void);
void orc_destroy(orc *o);
int orc_build_volumes(orc *o, const float *f, const uint8_t *w, int n_views, const params_t *prm);
int orc_fuse(orc *o, int iterations, float lam, float tau, float sigma);
int orc_fuse_gd(orc *o, int iterations, float lam, float xi, float eps);
int64_t orc_num_leaves(const orc *o);
int orc_extract(const orc *o, int64_t cap, uint32_t *keys, uint8_t *levels, double *u, double *ubar, double *p);
int orc_energy(const orc *o, double *tv, double *data);
int orc_energy_eps(const orc *o, double eps, double *tv, double *data);
int64_t orc_neighbours(const orc *o, int32_t *counts, int64_t cap, int64_t *idx);
int orc_export_state(const orc *o, void *buf, int64_t cap, int64_t *n_bytes);
int orc_import_state(orc *o, const void *buf, int64_t n_bytes);
double orc_prox(int M, const double *F, const double *W, double gamma, double uprime, double tl);

#define CHECK(x)                                                         \
    do {                                                                 \
        if (!(x)) {                                                      \
            fprintf(stderr, "check failed line %d: %s\n", __LINE__, #x); \
            return 1;                                                    \
        }                                                                \
    } while (0)

/* xorshift64*, for the synthetic volumes */
static uint64_t rng = 88172645463325252ull;
static double urand(void) {
    rng ^= rng >> 12;
    rng ^= rng << 25;
    rng ^= rng >> 27;
    return (double)((rng * 2685821657736338717ull) >> 11) * (1.0 / 9007199254740992.0);
}

int main(void) {
    const int D = 4, G = 16, V = 3;
    const size_t n = (size_t)V * G * G * G;
    float *f = malloc(n * sizeof(float));
    uint8_t *w = malloc(n);
    for (int v = 0; v < V; ++v)
        for (int z = 0; z < G; ++z)
            for (int y = 0; y < G; ++y)
                for (int x = 0; x < G; ++x) {
                    size_t i = (((size_t)v * G + z) * G + y) * G + x;
                    double d = sqrt((x - 7.5) * (x - 7.5) + (y - 8.0) * (y - 8.0) + (z - 7.0) * (z - 7.0)) - 4.5;
                    double val = d / 1.5 + 0.05 * (urand() - 0.5);
                    f[i] = (float)(val > 1 ? 1 : val < -1 ? -1 : val);
                    w[i] = urand() > 0.2;
                }
    params_t prm = {D, 0.1f, 1.0f, 0.1f, 0.01f, 0.5f, 0.9f, 1, 0};
    const float tau = 0.28867513f;
    orc *o = orc_create();
    CHECK(o);
    CHECK(orc_fuse(o, 1, 0.5f, tau, tau) != 0); /* no state yet */
    CHECK(orc_build_volumes(o, f, w, V, &prm) == 0);
    CHECK(orc_fuse(o, 12, 0.5f, tau, tau) == 0);
    CHECK(orc_fuse(o, 1, NAN, tau, tau) != 0);
    CHECK(orc_fuse(o, -1, 0.5f, tau, tau) != 0);
    int64_t L = orc_num_leaves(o);
    CHECK(L > 8);
    uint32_t *keys = malloc((size_t)L * 4);
    uint8_t *levels = malloc((size_t)L);
    double *u = malloc((size_t)L * 8), *ub = malloc((size_t)L * 8), *p = malloc((size_t)L * 24);
    CHECK(orc_extract(o, L, keys, levels, u, ub, p) == 0);
    CHECK(orc_extract(o, L - 1, keys, levels, u, ub, p) != 0);
    double tv, da;
    CHECK(orc_energy(o, &tv, &da) == 0 && tv >= 0 && da >= 0);
    int32_t *counts = malloc((size_t)L * 6 * 4);
    int64_t ne = orc_neighbours(o, counts, 0, NULL);
    int64_t *idx = malloc((size_t)(ne > 0 ? ne : 1) * 8);
    CHECK(orc_neighbours(o, counts, ne, idx) == ne);
    int64_t nb = 0;
    CHECK(orc_export_state(o, NULL, 0, &nb) != 0 || nb > 0);
    uint8_t *blob = malloc((size_t)nb);
    CHECK(orc_export_state(o, blob, nb, &nb) == 0);
    orc *b = orc_create();
    CHECK(orc_import_state(b, blob, nb) == 0);
    CHECK(orc_fuse_gd(b, 6, 0.5f, 0.05f, 0.3f) == 0);
    CHECK(orc_energy_eps(b, 0.3, &tv, &da) == 0);
    CHECK(orc_fuse_gd(b, 1, 0.5f, -1.0f, 0.3f) != 0);
    blob[0] ^= 0xFF; /* corrupt magic */
    CHECK(orc_import_state(b, blob, nb) != 0);
    blob[0] ^= 0xFF;
    CHECK(orc_import_state(b, blob, nb / 2) != 0); /* truncated */
    CHECK(orc_import_state(b, blob, nb) == 0);
    prm.split_tau = 0.95f; /* split_tau > join_tau */
    CHECK(orc_build_volumes(b, f, w, V, &prm) != 0);
    const double F[3] = {-1.0, 0.25, 1.0}, W[3] = {1.0, 0.5, 0.75};
    double r = orc_prox(3, F, W, 0.01, 0.1, 0.5);
    CHECK(r >= -1.0 && r <= 1.0);
    CHECK(orc_prox(0, NULL, NULL, 0.01, 0.37, 1.0) == 0.37);
    orc_destroy(b);
    orc_destroy(o);
    free(f);
    free(w);
    free(keys);
    free(levels);
    free(u);
    free(ub);
    free(p);
    free(counts);
    free(idx);
    free(blob);
    printf("oracle driver ok: %lld leaves, %lld adjacency entries, %lld-byte state\n", (long long)L, (long long)ne,
           (long long)nb);
    return 0;
}
