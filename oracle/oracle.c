/*
 * oracle.c -- CPU oracle for octree-based TV-L1 range-data fusion.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing on the product path links, loads or calls
 * this file: only the test-suite, the smoke check and the CPU-baseline leg of
 * the benchmark do. It shares no code, header, table or helper with the HIP
 * library; it has its own declarations of the two plain records it reads (the
 * camera and the parameter block) and its own parser of the state blob.
 *
 * Plain, single-threaded C99. The octree is a pointer tree (each node owns an
 * array of 8 children, as the paper's own node does, Sec. 4.1) and neighbours
 * are found by walking up to the common ancestor and back down. Compiled twice:
 *   -DORC_FP32 : every value in float, following the canonical operation order
 *                the GPU path also follows (one IEEE op at a time, explicit fma),
 *                so that the two can be compared bit for bit;
 *   (default)  : the same steps in double, for the self-checks.
 *
 * What it computes (paper sections in brackets):
 *   - per-view TSDF at every finest voxel centre [Sec. 3.1, Eq. 1, eta rule];
 *   - per-view TSDF octrees by the spread rule, means kept at every node
 *     [Sec. 3.1, Eq. 2 and the construction paragraph];
 *   - the initial fused octree = union of the per-view structures [Fig. 1];
 *   - the data fetch at a node's level or from the subsuming leaf [Fig. 4];
 *   - the normalised TV-L1 energy with the weight normaliser [Eq. 3, Eq. 5];
 *   - one primal-dual iteration: forward-difference gradient across leaves of
 *     unequal size, dual ascent and unit-ball projection, divergence, and the
 *     generalised shrinkage (median) prox [Sec. 3.2; Sec. 5 names primal-dual];
 *   - split and join of leaves from the updated values [Sec. 3.2, the two
 *     restructuring rules];
 *   - the paper's own solver: gradient descent to the steady state of Eq. 6 on
 *     the smoothed (Eq. 4), normalised (Eq. 5) energy, lambda on TV.
 * Where the paper is silent the readings are: lambda weights the normalised
 * data term; leaves of unequal size couple through area-weighted differences
 * over centre distance (exactly adjoint to the divergence); a split cascades
 * with each child re-running the prox on its own data; a join collapses the
 * largest ancestor whose leaves are all joinable with one sign, taking
 * hierarchical means. Every pin of these functions is in the test-suite.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#ifdef ORC_FP32
typedef float real;
#define R_FMA fmaf
#define R_SQRT sqrtf
#define R_ABS fabsf
#define R_MIN fminf
#define R_MAX fmaxf
#define R_LDEXP ldexpf
#else
typedef double real;
#define R_FMA fma
#define R_SQRT sqrt
#define R_ABS fabs
#define R_MIN fmin
#define R_MAX fmax
#define R_LDEXP ldexp
#endif

#define ORC_OK 0
#define ORC_E_INVALID 1
#define ORC_E_NOMEM 2
#define ORC_E_STATE 5

/* Pinhole camera, OpenCV axes. 72 bytes. */
typedef struct {
    float fx, fy, cx, cy;
    int32_t width, height;
    float R_cw[9]; /* row-major camera->world rotation, columns = camera axes */
    float C[3];    /* projection centre in world coordinates */
} orc_camera;

/* Construction / restructuring parameters. 40 bytes. */
typedef struct {
    int32_t max_depth;
    float delta, eta, spread_tau, gamma, split_tau, join_tau;
    int32_t restructure_every;
    int64_t max_leaves;
} orc_params;

/* Node of a per-view TSDF octree f_i*. */
typedef struct vnode {
    struct vnode *kid; /* 8 children, or NULL for a leaf */
    real S;            /* sum of f over the observed finest voxels below */
    int64_t cnt;       /* number of observed finest voxels below */
} vnode;

/* Node of the fused iterate u*. */
typedef struct unode {
    struct unode *parent;
    struct unode *kid; /* 8 children, or NULL for a leaf */
    int level, octant;
    uint32_t x, y, z; /* min corner in finest-voxel units */
    /* leaf state */
    real u, ubar, p[3];
    real uprime, uold, uplus;
    int split_flag, join_sign, fresh_join;
    /* observations, sorted by (F, view) */
    int M;
    real *F, *W, *Sk; /* Sk has M+1 entries */
    real Wtot, inv;
} unode;

/* Solver of the running fuse call: the primal-dual iteration, or the paper's
 * own gradient descent (lambda on TV, step xi, smoothing eps^2). */
typedef struct {
    int gd;
    real lam, xi, eps2;
} solver_t;

typedef struct orc {
    orc_params prm;
    solver_t sol;
    int n_views;
    vnode *views; /* n_views roots */
    unode *root;
    int64_t iteration;
    int64_t last_splits, last_joins;
    char err[256];
} orc;

static void set_err(orc *o, const char *m) {
    if (o) snprintf(o->err, sizeof o->err, "%s", m);
}

static uint32_t side_of(const orc *o, int level) { return 1u << (o->prm.max_depth - level); }

/* Morton key of a min corner: x in bit 0, y in bit 1, z in bit 2 of every triple. */
static uint32_t morton(uint32_t x, uint32_t y, uint32_t z) {
    uint32_t k = 0;
    for (int b = 0; b < 10; ++b)
        k |= (((x >> b) & 1u) << (3 * b)) | (((y >> b) & 1u) << (3 * b + 1)) | (((z >> b) & 1u) << (3 * b + 2));
    return k;
}

static void demorton(uint32_t k, uint32_t *x, uint32_t *y, uint32_t *z) {
    *x = *y = *z = 0;
    for (int b = 0; b < 10; ++b) {
        *x |= ((k >> (3 * b)) & 1u) << b;
        *y |= ((k >> (3 * b + 1)) & 1u) << b;
        *z |= ((k >> (3 * b + 2)) & 1u) << b;
    }
}

/* ------------------------------------------------------------------------ */
/* Eq. 1: truncated signed distance of one view at one finest voxel centre.   */
/* ------------------------------------------------------------------------ */
typedef struct {
    const float *depth; /* n_views * H * W */
    const orc_camera *cams;
    const float *fvol;   /* alternative input: per-view finest-voxel values */
    const uint8_t *wvol; /* and observation masks, index ((v*G + z)*G + y)*G + x */
} src_t;

static int tsdf_voxel(const orc *o, const src_t *src, int v, uint32_t a, uint32_t b, uint32_t c, real *f) {
    if (src->fvol) {
        uint64_t G = 1ull << o->prm.max_depth;
        uint64_t i = (((uint64_t)v * G + c) * G + b) * G + a;
        if (!src->wvol[i]) return 0;
        *f = (real)src->fvol[i];
        return 1;
    }
    const orc_camera *cam = &src->cams[v];
    const real h = R_LDEXP((real)1, -o->prm.max_depth);
    /* voxel centre, exact: (index + 1/2) * 2^-Dmax */
    real dx = ((real)a + (real)0.5) * h - (real)cam->C[0];
    real dy = ((real)b + (real)0.5) * h - (real)cam->C[1];
    real dz = ((real)c + (real)0.5) * h - (real)cam->C[2];
    const float *R = cam->R_cw;
    /* camera coordinates: X_j = sum_r R[r][j] * d_r */
    real X = R_FMA((real)R[0], dx, R_FMA((real)R[3], dy, (real)R[6] * dz));
    real Y = R_FMA((real)R[1], dx, R_FMA((real)R[4], dy, (real)R[7] * dz));
    real Z = R_FMA((real)R[2], dx, R_FMA((real)R[5], dy, (real)R[8] * dz));
    if (!(Z > 0)) return 0; /* behind the camera */
    real pu = R_FMA((real)cam->fx, X / Z, (real)cam->cx);
    real pv = R_FMA((real)cam->fy, Y / Z, (real)cam->cy);
    if (!(pu >= 0 && pu < (real)cam->width && pv >= 0 && pv < (real)cam->height)) return 0;
    int pi = (int)pu, pj = (int)pv;
    float Dm = src->depth[((size_t)v * cam->height + pj) * cam->width + pi];
    if (!(Dm > 0.0f && Dm <= 3.4028234663852886e38f)) return 0; /* invalid pixel */
    real r = R_SQRT(R_FMA(dx, dx, R_FMA(dy, dy, dz * dz)));
    real phi = (real)Dm - r;
    if (phi < -(real)o->prm.eta) return 0; /* behind the eta band: unobserved */
    *f = R_MIN((real)1, R_MAX((real)-1, phi / (real)o->prm.delta));
    return 1;
}

/* ------------------------------------------------------------------------ */
/* Eq. 2 and the construction rule: post-order build of one view's octree.    */
/* A node keeps its children iff level < Dmax, some voxel below is observed   */
/* and the spread of the observed values exceeds spread_tau. Every stored     */
/* node keeps the sum and count of its observed voxels (the upward means).    */
/* ------------------------------------------------------------------------ */
static void free_vtree(vnode *n) {
    if (!n->kid) return;
    for (int c = 0; c < 8; ++c) free_vtree(&n->kid[c]);
    free(n->kid);
    n->kid = NULL;
}

static int build_vnode(const orc *o, const src_t *src, int v, vnode *n, int level, uint32_t x, uint32_t y,
                       uint32_t z, real *mn, real *mx) {
    n->kid = NULL;
    if (level == o->prm.max_depth) {
        real f = 0;
        if (tsdf_voxel(o, src, v, x, y, z, &f)) {
            n->S = f;
            n->cnt = 1;
            *mn = *mx = f;
        } else {
            n->S = 0;
            n->cnt = 0;
            *mn = (real)INFINITY;
            *mx = -(real)INFINITY;
        }
        return ORC_OK;
    }
    vnode *kid = (vnode *)calloc(8, sizeof(vnode));
    if (!kid) return ORC_E_NOMEM;
    uint32_t hs = side_of(o, level + 1);
    real S = 0, lo = (real)INFINITY, hi = -(real)INFINITY;
    int64_t cnt = 0;
    for (int c = 0; c < 8; ++c) {
        real cmn, cmx;
        int st = build_vnode(o, src, v, &kid[c], level + 1, x + (c & 1) * hs, y + ((c >> 1) & 1) * hs,
                             z + ((c >> 2) & 1) * hs, &cmn, &cmx);
        if (st) {
            for (int j = 0; j < c; ++j) free_vtree(&kid[j]);
            free(kid);
            return st;
        }
        S = S + kid[c].S;
        cnt += kid[c].cnt;
        lo = R_MIN(lo, cmn);
        hi = R_MAX(hi, cmx);
    }
    n->S = S;
    n->cnt = cnt;
    *mn = lo;
    *mx = hi;
    if (cnt > 0 && (hi - lo) > (real)o->prm.spread_tau) {
        n->kid = kid;
    } else {
        for (int c = 0; c < 8; ++c) free_vtree(&kid[c]);
        free(kid);
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Fig. 4: data fetch for a node of u* at level L: the view's node at the     */
/* same level if it is stored, else the deepest view leaf that contains it.   */
/* ------------------------------------------------------------------------ */
static const vnode *fetch_view(const orc *o, int v, int L, uint32_t x, uint32_t y, uint32_t z, int *lvl_out) {
    const vnode *n = &o->views[v];
    int l = 0;
    while (l < L && n->kid) {
        uint32_t hs = side_of(o, l + 1);
        int c = (int)((x / hs) & 1u) | (int)(((y / hs) & 1u) << 1) | (int)(((z / hs) & 1u) << 2);
        n = &n->kid[c];
        ++l;
    }
    *lvl_out = l;
    return n;
}

typedef struct {
    real F, W;
    int view;
} obs_t;

static int obs_cmp(const void *a, const void *b) {
    const obs_t *p = (const obs_t *)a, *q = (const obs_t *)b;
    if (p->F < q->F) return -1;
    if (p->F > q->F) return 1;
    return (p->view > q->view) - (p->view < q->view);
}

static void free_obs(unode *n) {
    free(n->F);
    free(n->W);
    free(n->Sk);
    n->F = n->W = n->Sk = NULL;
    n->M = 0;
}

/* Observations of node n sorted by (F, view), prefix weights, normaliser. */
static int gather_obs(const orc *o, unode *n) {
    free_obs(n);
    obs_t *tmp = (obs_t *)malloc(sizeof(obs_t) * (size_t)(o->n_views > 0 ? o->n_views : 1));
    if (!tmp) return ORC_E_NOMEM;
    int M = 0;
    for (int v = 0; v < o->n_views; ++v) {
        int lvl;
        const vnode *vn = fetch_view(o, v, n->level, n->x, n->y, n->z, &lvl);
        if (vn->cnt <= 0) continue; /* W = 0: dropped */
        tmp[M].F = vn->S / (real)vn->cnt;
        tmp[M].W = R_LDEXP((real)vn->cnt, -3 * (o->prm.max_depth - lvl)); /* cnt / vol */
        tmp[M].view = v;
        ++M;
    }
    qsort(tmp, (size_t)M, sizeof(obs_t), obs_cmp);
    n->F = (real *)malloc(sizeof(real) * (size_t)(M > 0 ? M : 1));
    n->W = (real *)malloc(sizeof(real) * (size_t)(M > 0 ? M : 1));
    n->Sk = (real *)malloc(sizeof(real) * (size_t)(M + 1));
    if (!n->F || !n->W || !n->Sk) {
        free(tmp);
        free_obs(n);
        return ORC_E_NOMEM;
    }
    real P = 0;
    for (int k = 0; k < M; ++k) {
        n->F[k] = tmp[k].F;
        n->W[k] = tmp[k].W;
        P = P + tmp[k].W;
    }
    n->M = M;
    n->Wtot = P;
    n->inv = (real)1 / (P + (real)o->prm.gamma);
    /* S_k = 2 P_k - W_tot: the derivative of the data term on (F_(k), F_(k+1)) */
    real Pk = 0;
    n->Sk[0] = R_FMA((real)2, Pk, -P);
    for (int k = 1; k <= M; ++k) {
        Pk = Pk + n->W[k - 1];
        n->Sk[k] = R_FMA((real)2, Pk, -P);
    }
    free(tmp);
    return ORC_OK;
}

/* Generalised shrinkage: argmin_v (v - u')^2 / (2 tau) + lambda_n sum_i W_i |v - F_i|
 * = the median of {F_(1..M)} and the M+1 stationary points u' - t S_k of the
 * quadratic pieces, with t = tau * lambda_n. Written as its definition: sort the
 * 2M+1 values and take the middle one. The result is returned as +0 for a zero. */
static int real_cmp(const void *a, const void *b) {
    real p = *(const real *)a, q = *(const real *)b;
    return (p > q) - (p < q);
}

static real prox_median(int M, const real *F, const real *Sk, real uprime, real t, real *scratch) {
    for (int k = 0; k < M; ++k) scratch[k] = F[k];
    for (int k = 0; k <= M; ++k) scratch[M + k] = R_FMA(-t, Sk[k], uprime);
    qsort(scratch, (size_t)(2 * M + 1), sizeof(real), real_cmp);
    return scratch[M] + (real)0;
}

/* ------------------------------------------------------------------------ */
/* Fused octree: union of the per-view structures [Fig. 1 caption].          */
/* ------------------------------------------------------------------------ */
static void free_utree(unode *n) {
    free_obs(n);
    if (!n->kid) return;
    for (int c = 0; c < 8; ++c) free_utree(&n->kid[c]);
    free(n->kid);
    n->kid = NULL;
}

static int make_kids(const orc *o, unode *n) {
    n->kid = (unode *)calloc(8, sizeof(unode));
    if (!n->kid) return ORC_E_NOMEM;
    uint32_t hs = side_of(o, n->level + 1);
    for (int c = 0; c < 8; ++c) {
        unode *k = &n->kid[c];
        k->parent = n;
        k->level = n->level + 1;
        k->octant = c;
        k->x = n->x + (c & 1) * hs;
        k->y = n->y + ((c >> 1) & 1) * hs;
        k->z = n->z + ((c >> 2) & 1) * hs;
    }
    return ORC_OK;
}

static int build_union(const orc *o, unode *n, const vnode **vv) {
    int split = 0;
    for (int v = 0; v < o->n_views; ++v)
        if (vv[v] && vv[v]->kid) split = 1;
    if (!split) return ORC_OK;
    int st = make_kids(o, n);
    if (st) return st;
    const vnode **cv = (const vnode **)malloc(sizeof(vnode *) * (size_t)o->n_views);
    if (!cv) return ORC_E_NOMEM;
    for (int c = 0; c < 8 && !st; ++c) {
        for (int v = 0; v < o->n_views; ++v) cv[v] = (vv[v] && vv[v]->kid) ? &vv[v]->kid[c] : NULL;
        st = build_union(o, &n->kid[c], cv);
    }
    free(cv);
    return st;
}

/* Leaves in Morton (depth-first, child 0..7) order. */
typedef struct {
    unode **a;
    int64_t n, cap;
} leafvec;

static int lv_push(leafvec *v, unode *n) {
    if (v->n == v->cap) {
        int64_t nc = v->cap ? 2 * v->cap : 1024;
        unode **na = (unode **)realloc(v->a, sizeof(unode *) * (size_t)nc);
        if (!na) return ORC_E_NOMEM;
        v->a = na;
        v->cap = nc;
    }
    v->a[v->n++] = n;
    return ORC_OK;
}

static int collect(unode *n, leafvec *v) {
    if (!n->kid) return lv_push(v, n);
    for (int c = 0; c < 8; ++c) {
        int st = collect(&n->kid[c], v);
        if (st) return st;
    }
    return ORC_OK;
}

/* Initial value: normalised weighted mean of the observations, p = 0. */
static void init_leaf(unode *n) {
    real acc = 0;
    for (int k = 0; k < n->M; ++k) acc = R_FMA(n->W[k], n->F[k], acc);
    n->u = acc * n->inv;
    n->ubar = n->u;
    n->p[0] = n->p[1] = n->p[2] = 0;
}

/* ------------------------------------------------------------------------ */
/* Face neighbours (walk up to the common ancestor, mirror back down).       */
/* ------------------------------------------------------------------------ */
/* The neighbour of n across its face (d, s) that is at least as large as n;
 * NULL on the domain boundary. s = +1 looks toward increasing coordinate d. */
static unode *nb_ge(unode *n, int d, int s) {
    if (!n->parent) return NULL;
    int bit = (n->octant >> d) & 1;
    if (s > 0 && bit == 0) return &n->parent->kid[n->octant | (1 << d)];
    if (s < 0 && bit == 1) return &n->parent->kid[n->octant & ~(1 << d)];
    unode *m = nb_ge(n->parent, d, s);
    if (!m || !m->kid) return m;
    return &m->kid[n->octant ^ (1 << d)];
}

/* Leaves of m's subtree that touch the face shared with the node on the other
 * side, in ascending key order. For s = +1 (m lies on the + side) that is m's
 * low face in d, i.e. children with bit d clear. */
static int face_leaves(unode *m, int d, int s, leafvec *out) {
    if (!m->kid) return lv_push(out, m);
    for (int c = 0; c < 8; ++c) {
        if (((c >> d) & 1) != (s > 0 ? 0 : 1)) continue;
        int st = face_leaves(&m->kid[c], d, s, out);
        if (st) return st;
    }
    return ORC_OK;
}

static int neighbours(unode *n, int d, int s, leafvec *out) {
    out->n = 0;
    unode *m = nb_ge(n, d, s);
    if (!m) return ORC_OK;
    return face_leaves(m, d, s, out);
}

/* The neighbour list of one side (s = +1 or -1) of n: the x neighbours, then
 * y, then z, each in ascending key; b[d] .. b[d+1] are direction d's entries. */
static int side_list(unode *n, int s, leafvec *out, int64_t b[4]) {
    out->n = 0;
    for (int d = 0; d < 3; ++d) {
        b[d] = out->n;
        unode *m = nb_ge(n, d, s);
        if (!m) continue;
        int st = face_leaves(m, d, s, out);
        if (st) return st;
    }
    b[3] = out->n;
    return ORC_OK;
}

/* Coupling coefficients between face-adjacent leaves (sides in voxel units).
 * Gradient: (Gu)_{n,d} = sum_{k in N+_d(n)} c_nk (u_k - u_n),
 *   c_nk = (min(s_n,s_k)/s_n)^2 / h_nk, h_nk = (s_n + s_k)/2:
 *   the fraction of n's face the contact covers, over the centre distance.
 * Divergence: div = -G^T under volume-weighted inner products,
 *   (div p)_n = sum_d [ C+_{n,d} p_{n,d} - sum_{m in N-_d(n)} c'_mn p_{m,d} ],
 *   C+_{n,d} = sum_k c_nk, c'_mn = vol_m c_mn / vol_n. */
static real coef_grad(const orc *o, const unode *n, const unode *k) {
    real sn = (real)side_of(o, n->level), sk = (real)side_of(o, k->level);
    real a = sn < sk ? sn : sk;
    real r = (a / sn) * (a / sn);
    real h = (sn + sk) * (real)0.5;
    return r / h;
}

static real coef_div(const orc *o, const unode *m, const unode *n) {
    real sm = (real)side_of(o, m->level), sn = (real)side_of(o, n->level);
    real a = sm < sn ? sm : sn;
    real h = (sm + sn) * (real)0.5;
    return (sm * a * a) / (h * sn * sn * sn);
}

/* Gradient sums of n over its + list (b: direction bounds): g[d] = sum of
 * c_nk (v_k - v_n), C[d] = sum of c_nk over direction d's entries, with v the
 * ubar (field 0) or u (field 1) values. Every sum is one sequential chain in
 * list order (ascending neighbour key), however long the list. */
static void grad_sums(const orc *o, const unode *n, const leafvec *nb, const int64_t b[4], int field, real g[3],
                      real C[3]) {
    const real vn = field ? n->u : n->ubar;
    for (int d = 0; d < 3; ++d) {
        g[d] = 0;
        C[d] = 0;
        for (int64_t q = b[d]; q < b[d + 1]; ++q) {
            const unode *k = nb->a[q];
            const real c = coef_grad(o, n, k);
            g[d] = R_FMA(c, (field ? k->u : k->ubar) - vn, g[d]);
            C[d] = C[d] + c;
        }
    }
}

/* ------------------------------------------------------------------------ */
/* One primal-dual iteration (Jacobi phases).                                */
/* ------------------------------------------------------------------------ */
static int dual_leaf(const orc *o, unode *n, real sigma, leafvec *nb) {
    real q[3], g[3], C[3];
    int64_t b[4];
    int st = side_list(n, +1, nb, b);
    if (st) return st;
    grad_sums(o, n, nb, b, 0, g, C);
    for (int d = 0; d < 3; ++d) q[d] = R_FMA(sigma, g[d], n->p[d]);
    real r2 = R_FMA(q[0], q[0], R_FMA(q[1], q[1], q[2] * q[2]));
    if (r2 > (real)1) {
        real nrm = R_SQRT(r2);
        for (int d = 0; d < 3; ++d) n->p[d] = q[d] / nrm;
    } else {
        for (int d = 0; d < 3; ++d) n->p[d] = q[d];
    }
    return ORC_OK;
}

static int div_leaf(const orc *o, unode *n, leafvec *nb, real *out) {
    /* own (outgoing) terms first, x, y, z; then the incoming terms of the -
     * list (x, y, z, each in ascending neighbour key) */
    real g[3], C[3];
    int64_t b[4];
    int st = side_list(n, +1, nb, b);
    if (st) return st;
    grad_sums(o, n, nb, b, 0, g, C);
    real acc = 0;
    for (int d = 0; d < 3; ++d) acc = R_FMA(C[d], n->p[d], acc);
    st = side_list(n, -1, nb, b);
    if (st) return st;
    for (int d = 0; d < 3; ++d)
        for (int64_t q = b[d]; q < b[d + 1]; ++q) {
            unode *m = nb->a[q];
            acc = R_FMA(-coef_div(o, m, n), m->p[d], acc);
        }
    *out = acc;
    return ORC_OK;
}

static real *g_scratch = NULL;
static int64_t g_scratch_n = 0;

static real *scratch_for(int M) {
    if (2 * (int64_t)M + 1 > g_scratch_n) {
        free(g_scratch);
        g_scratch_n = 2 * (int64_t)M + 1 + 64;
        g_scratch = (real *)malloc(sizeof(real) * (size_t)g_scratch_n);
        if (!g_scratch) g_scratch_n = 0;
    }
    return g_scratch;
}

static int primal_leaf(const orc *o, unode *n, real tau, real tl, leafvec *nb) {
    real dv;
    int st = div_leaf(o, n, nb, &dv);
    if (st) return st;
    real *scr = scratch_for(n->M);
    if (!scr) return ORC_E_NOMEM;
    n->uprime = R_FMA(tau, dv, n->u);
    n->uold = n->u;
    n->uplus = prox_median(n->M, n->F, n->Sk, n->uprime, tl * n->inv, scr);
    n->ubar = R_FMA((real)2, n->uplus, -n->uold);
    n->u = n->uplus;
    /* restructuring flags from the updated value */
    n->split_flag = (R_ABS(n->uplus) < (real)o->prm.split_tau) && (n->level < o->prm.max_depth);
    n->join_sign = 0;
    if (!(o->prm.join_tau > 1.0f) && R_ABS(n->uplus) > (real)o->prm.join_tau) n->join_sign = n->uplus > 0 ? 1 : -1;
    n->fresh_join = 0;
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* The paper's own solver: explicit gradient descent to the steady state of   */
/* the PDE of Eq. 6 for the energy of Eq. 5 with both terms smoothed as in    */
/* Eq. 4, Gamma(x^2) = sqrt(x^2 + eps^2), and lambda on the TV term:          */
/*   E(u) = sum_n vol_n [ sum_i W_i Gamma((u_n - F_i)^2) / (sum W + gamma)    */
/*                        + lambda Gamma(|(Gu)_n|^2) ]                        */
/*   u <- u + xi (lambda div(q) - d'(u)),   q = Gu / Gamma(|Gu|^2),           */
/*   d'(u) = sum_i W_i (u - F_i) / Gamma((u - F_i)^2) / (sum W + gamma).      */
/* q is kept in p; div is the same volume-weighted adjoint as above.          */
/* ------------------------------------------------------------------------ */
static int gd_flux_leaf(const orc *o, unode *n, real eps2, leafvec *nb) {
    real g[3], C[3];
    int64_t b[4];
    int st = side_list(n, +1, nb, b);
    if (st) return st;
    grad_sums(o, n, nb, b, 1, g, C);
    real r2 = R_FMA(g[0], g[0], R_FMA(g[1], g[1], g[2] * g[2]));
    real den = R_SQRT(r2 + eps2);
    for (int d = 0; d < 3; ++d) n->p[d] = g[d] / den;
    return ORC_OK;
}

/* d'(u) for leaf n's observations: the terms W_k (r_k / sqrt(r_k^2 + eps^2)),
 * r_k = u - F_k, summed in one sequential chain in (F, view) order, times the
 * normaliser 1 / (sum W + gamma). */
static real gd_data_grad(const unode *n, real u, real eps2) {
    real acc = 0;
    for (int k = 0; k < n->M; ++k) {
        real r = u - n->F[k];
        real den = R_SQRT(R_FMA(r, r, eps2));
        acc = acc + n->W[k] * (r / den);
    }
    return acc * n->inv;
}

static void set_flags(const orc *o, unode *n) {
    n->split_flag = (R_ABS(n->uplus) < (real)o->prm.split_tau) && (n->level < o->prm.max_depth);
    n->join_sign = 0;
    if (!(o->prm.join_tau > 1.0f) && R_ABS(n->uplus) > (real)o->prm.join_tau) n->join_sign = n->uplus > 0 ? 1 : -1;
    n->fresh_join = 0;
}

/* One descent step of leaf n; the divergence is kept (uprime) so that split
 * children can take the same step with their own data term. */
static int gd_update_leaf(const orc *o, unode *n, leafvec *nb) {
    const solver_t *s = &o->sol;
    real dv;
    int st = div_leaf(o, n, nb, &dv);
    if (st) return st;
    n->uprime = dv;
    n->uold = n->u;
    n->uplus = R_FMA(s->xi, R_FMA(s->lam, dv, -gd_data_grad(n, n->u, s->eps2)), n->u);
    n->u = n->uplus;
    n->ubar = n->uplus;
    set_flags(o, n);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* Restructuring [Sec. 3.2, split and join rules].                           */
/* ------------------------------------------------------------------------ */
/* +1 / -1 if every leaf below n is joinable with that sign, else 0. */
static int all_join_sign(const unode *n) {
    if (!n->kid) return n->join_sign;
    int s = all_join_sign(&n->kid[0]);
    if (!s) return 0;
    for (int c = 1; c < 8; ++c)
        if (all_join_sign(&n->kid[c]) != s) return 0;
    return s;
}

/* Hierarchical mean: a leaf's value, else 1/8 of the sum of the children's
 * hierarchical means in child order. which: 0 u, 1 ubar, 2..4 p. */
static real hmean(const unode *n, int which) {
    if (!n->kid) return which == 0 ? n->u : which == 1 ? n->ubar : n->p[which - 2];
    real acc = 0;
    for (int c = 0; c < 8; ++c) acc = acc + hmean(&n->kid[c], which);
    return (real)0.125 * acc;
}

static int collapse(orc *o, unode *n) {
    if (!n->kid) return ORC_OK;
    if (all_join_sign(n)) {
        real v[5];
        for (int w = 0; w < 5; ++w) v[w] = hmean(n, w);
        for (int c = 0; c < 8; ++c) free_utree(&n->kid[c]);
        free(n->kid);
        n->kid = NULL;
        n->u = v[0];
        n->ubar = v[1];
        n->p[0] = v[2];
        n->p[1] = v[3];
        n->p[2] = v[4];
        n->split_flag = 0;
        n->join_sign = 0;
        n->fresh_join = 1;
        o->last_joins++;
        return gather_obs(o, n);
    }
    for (int c = 0; c < 8; ++c) {
        int st = collapse(o, &n->kid[c]);
        if (st) return st;
    }
    return ORC_OK;
}

/* Split n into 8 children that inherit u', u_old and p; each child runs the
 * prox (gradient descent: the descent step) on its own observations and
 * splits again while it is still flagged. */
static int cascade(orc *o, unode *n, real tl) {
    int st = make_kids(o, n);
    if (st) return st;
    o->last_splits++;
    for (int c = 0; c < 8; ++c) {
        unode *k = &n->kid[c];
        k->uprime = n->uprime;
        k->uold = n->uold;
        k->p[0] = n->p[0];
        k->p[1] = n->p[1];
        k->p[2] = n->p[2];
        st = gather_obs(o, k);
        if (st) return st;
        if (o->sol.gd) {
            /* the parent's step with the child's own data term */
            const solver_t *s = &o->sol;
            k->uplus = R_FMA(s->xi, R_FMA(s->lam, k->uprime, -gd_data_grad(k, k->uold, s->eps2)), k->uold);
            k->u = k->uplus;
            k->ubar = k->uplus;
        } else {
            real *scr = scratch_for(k->M);
            if (!scr) return ORC_E_NOMEM;
            k->uplus = prox_median(k->M, k->F, k->Sk, k->uprime, tl * k->inv, scr);
            k->u = k->uplus;
            k->ubar = R_FMA((real)2, k->uplus, -k->uold);
        }
        k->join_sign = 0;
        k->split_flag = (R_ABS(k->uplus) < (real)o->prm.split_tau) && (k->level < o->prm.max_depth);
    }
    free_obs(n);
    for (int c = 0; c < 8; ++c) {
        if (n->kid[c].split_flag) {
            st = cascade(o, &n->kid[c], tl);
            if (st) return st;
        }
    }
    return ORC_OK;
}

static int restructure(orc *o, real tl) {
    o->last_splits = o->last_joins = 0;
    int st = collapse(o, o->root);
    if (st) return st;
    leafvec lv = {0};
    st = collect(o->root, &lv);
    for (int64_t i = 0; i < lv.n && !st; ++i) {
        unode *n = lv.a[i];
        if (n->split_flag && !n->fresh_join) st = cascade(o, n, tl);
    }
    free(lv.a);
    return st;
}

/* ------------------------------------------------------------------------ */
/* Public API (ctypes).                                                      */
/* ------------------------------------------------------------------------ */
static int check_params(orc *o, const orc_params *p, int n_views) {
    if (!p || n_views < 1 || n_views > 64) return set_err(o, "bad params / n_views (1..64)"), ORC_E_INVALID;
    if (p->max_depth < 1 || p->max_depth > 10) return set_err(o, "max_depth out of 1..10"), ORC_E_INVALID;
    if (!(p->delta > 0) || !(p->eta >= p->delta)) return set_err(o, "need eta >= delta > 0"), ORC_E_INVALID;
    if (!(p->gamma > 0)) return set_err(o, "need gamma > 0"), ORC_E_INVALID;
    if (!(p->split_tau <= p->join_tau)) return set_err(o, "need split_tau <= join_tau"), ORC_E_INVALID;
    if (p->restructure_every < 0) return set_err(o, "restructure_every < 0"), ORC_E_INVALID;
    return ORC_OK;
}

orc *orc_create(void) { return (orc *)calloc(1, sizeof(orc)); }

static void clear(orc *o) {
    if (o->views) {
        for (int v = 0; v < o->n_views; ++v) free_vtree(&o->views[v]);
        free(o->views);
        o->views = NULL;
    }
    if (o->root) {
        free_utree(o->root);
        free(o->root);
        o->root = NULL;
    }
    o->n_views = 0;
    o->iteration = 0;
}

void orc_destroy(orc *o) {
    if (!o) return;
    clear(o);
    free(o);
}

const char *orc_last_error(const orc *o) { return o ? o->err : "null oracle"; }

static int init_all_leaves(orc *o) {
    leafvec lv = {0};
    int st = collect(o->root, &lv);
    for (int64_t i = 0; i < lv.n && !st; ++i) {
        st = gather_obs(o, lv.a[i]);
        if (!st) init_leaf(lv.a[i]);
    }
    free(lv.a);
    return st;
}

static int build_common(orc *o, const src_t *src, int n_views, const orc_params *prm) {
    int st = check_params(o, prm, n_views);
    if (st) return st;
    clear(o);
    o->prm = *prm;
    o->n_views = n_views;
    o->views = (vnode *)calloc((size_t)n_views, sizeof(vnode));
    if (!o->views) return ORC_E_NOMEM;
    for (int v = 0; v < n_views; ++v) {
        real mn, mx;
        st = build_vnode(o, src, v, &o->views[v], 0, 0, 0, 0, &mn, &mx);
        if (st) return st;
    }
    o->root = (unode *)calloc(1, sizeof(unode));
    if (!o->root) return ORC_E_NOMEM;
    const vnode **vv = (const vnode **)malloc(sizeof(vnode *) * (size_t)n_views);
    if (!vv) return ORC_E_NOMEM;
    for (int v = 0; v < n_views; ++v) vv[v] = &o->views[v];
    st = build_union(o, o->root, vv);
    free(vv);
    if (st) return st;
    return init_all_leaves(o);
}

/* Build from depth maps (n_views * H * W radial ranges, 0 / NaN invalid). */
int orc_build(orc *o, const float *depth, int n_views, const orc_camera *cams, const orc_params *prm) {
    if (!o || !depth || !cams) return ORC_E_INVALID;
    for (int v = 0; v < n_views; ++v)
        if (cams[v].width <= 0 || cams[v].height <= 0 || cams[v].width != cams[0].width ||
            cams[v].height != cams[0].height)
            return set_err(o, "bad camera size"), ORC_E_INVALID;
    src_t src = {depth, cams, NULL, NULL};
    return build_common(o, &src, n_views, prm);
}

/* Build from per-view finest-voxel values f and masks w, each of size
 * n_views * G^3 with index ((v*G + z)*G + y)*G + x, G = 2^max_depth. This
 * bypasses Eq. 1 so that tests can feed chosen TSDF volumes. */
int orc_build_volumes(orc *o, const float *f, const uint8_t *w, int n_views, const orc_params *prm) {
    if (!o || !f || !w) return ORC_E_INVALID;
    src_t src = {NULL, NULL, f, w};
    return build_common(o, &src, n_views, prm);
}

/* Dense Eq. 1 evaluation of one view at every finest voxel (test hook). */
int orc_tsdf_volume(const float *depth, int n_views, const orc_camera *cams, const orc_params *prm, int view,
                    double *f_out, uint8_t *w_out) {
    orc tmp;
    memset(&tmp, 0, sizeof tmp);
    if (check_params(&tmp, prm, n_views) || view < 0 || view >= n_views) return ORC_E_INVALID;
    tmp.prm = *prm;
    tmp.n_views = n_views;
    src_t src = {depth, cams, NULL, NULL};
    uint32_t G = 1u << prm->max_depth;
    for (uint32_t c = 0; c < G; ++c)
        for (uint32_t b = 0; b < G; ++b)
            for (uint32_t a = 0; a < G; ++a) {
                real f = 0;
                int ob = tsdf_voxel(&tmp, &src, view, a, b, c, &f);
                size_t i = ((size_t)c * G + b) * G + a;
                f_out[i] = ob ? (double)f : 0.0;
                w_out[i] = (uint8_t)ob;
            }
    return ORC_OK;
}

int orc_fuse(orc *o, int iterations, float lam, float tau, float sigma) {
    if (!o || !o->root) return ORC_E_STATE;
    if (iterations < 0 || !isfinite(lam) || !isfinite(tau) || !isfinite(sigma) || lam < 0 || !(tau > 0) ||
        !(sigma > 0))
        return set_err(o, "bad fuse arguments"), ORC_E_INVALID;
    const real rt = (real)tau, rs = (real)sigma;
    const real tl = rt * (real)lam;
    o->sol.gd = 0;
    leafvec lv = {0}, nb = {0};
    int st = ORC_OK;
    for (int it = 0; it < iterations && !st; ++it) {
        o->iteration++;
        lv.n = 0;
        st = collect(o->root, &lv);
        for (int64_t i = 0; i < lv.n && !st; ++i) st = dual_leaf(o, lv.a[i], rs, &nb);
        for (int64_t i = 0; i < lv.n && !st; ++i) st = primal_leaf(o, lv.a[i], rt, tl, &nb);
        o->last_splits = o->last_joins = 0;
        if (!st && o->prm.restructure_every > 0 && o->iteration % o->prm.restructure_every == 0)
            st = restructure(o, tl);
    }
    free(lv.a);
    free(nb.a);
    return st;
}

/* `iterations` steps of the paper's gradient descent (see gd_update_leaf)
 * with step xi, TV weight lam and smoothing eps, split/join as for orc_fuse
 * with the descent step in place of the prox. Jacobi phases: every flux from
 * the current u, then every update. */
int orc_fuse_gd(orc *o, int iterations, float lam, float xi, float eps) {
    if (!o || !o->root) return ORC_E_STATE;
    if (iterations < 0 || !isfinite(lam) || !isfinite(xi) || !isfinite(eps) || lam < 0 || !(xi > 0) || !(eps > 0))
        return set_err(o, "bad fuse arguments"), ORC_E_INVALID;
    o->sol.gd = 1;
    o->sol.lam = (real)lam;
    o->sol.xi = (real)xi;
    o->sol.eps2 = (real)eps * (real)eps;
    leafvec lv = {0}, nb = {0};
    int st = ORC_OK;
    for (int it = 0; it < iterations && !st; ++it) {
        o->iteration++;
        lv.n = 0;
        st = collect(o->root, &lv);
        for (int64_t i = 0; i < lv.n && !st; ++i) st = gd_flux_leaf(o, lv.a[i], o->sol.eps2, &nb);
        for (int64_t i = 0; i < lv.n && !st; ++i) st = gd_update_leaf(o, lv.a[i], &nb);
        o->last_splits = o->last_joins = 0;
        if (!st && o->prm.restructure_every > 0 && o->iteration % o->prm.restructure_every == 0)
            st = restructure(o, 0);
    }
    o->sol.gd = 0;
    free(lv.a);
    free(nb.a);
    return st;
}

/* Test hook: the restructure of the current state, as the fuse loop runs it
 * after an iteration's primal phase (split/join flags, u', u_old and u+ from
 * that phase). Valid only right after an orc_fuse call whose last iteration
 * did not restructure (restructure_every = 0). */
int orc_restructure_now(orc *o, float lam, float tau) {
    if (!o || !o->root) return ORC_E_STATE;
    const real tl = (real)tau * (real)lam;
    o->sol.gd = 0;
    return restructure(o, tl);
}

/* Test hook: per leaf in key order, u' (the primal step's argument of the
 * prox; for the gradient descent its divergence), u_old (u before the step)
 * and the split flag, as the last primal phase or split cascade left them. */
int orc_extract_aux(const orc *o, int64_t cap, double *uprime, double *uold, int32_t *split) {
    if (!o || !o->root) return ORC_E_STATE;
    leafvec lv = {0};
    int st = collect(o->root, &lv);
    if (!st && lv.n > cap) st = ORC_E_INVALID;
    for (int64_t i = 0; i < lv.n && !st; ++i) {
        unode *n = lv.a[i];
        if (uprime) uprime[i] = (double)n->uprime;
        if (uold) uold[i] = (double)n->uold;
        if (split) split[i] = n->split_flag;
    }
    free(lv.a);
    return st;
}

int64_t orc_num_leaves(const orc *o) {
    if (!o || !o->root) return -1;
    leafvec lv = {0};
    collect(o->root, &lv);
    free(lv.a);
    return lv.n;
}

void orc_last_counts(const orc *o, int64_t *splits, int64_t *joins) {
    *splits = o->last_splits;
    *joins = o->last_joins;
}

/* Leaves in key order: key, level, u, ubar, p (3 per leaf). */
int orc_extract(const orc *o, int64_t cap, uint32_t *keys, uint8_t *levels, double *u, double *ubar, double *p) {
    if (!o || !o->root) return ORC_E_STATE;
    leafvec lv = {0};
    int st = collect(o->root, &lv);
    if (!st && lv.n > cap) st = ORC_E_INVALID;
    for (int64_t i = 0; i < lv.n && !st; ++i) {
        unode *n = lv.a[i];
        if (keys) keys[i] = morton(n->x, n->y, n->z);
        if (levels) levels[i] = (uint8_t)n->level;
        if (u) u[i] = (double)n->u;
        if (ubar) ubar[i] = (double)n->ubar;
        if (p)
            for (int d = 0; d < 3; ++d) p[3 * i + d] = (double)n->p[d];
    }
    free(lv.a);
    return st;
}

/* Observations of every leaf: M (per leaf), Wtot and inv (per leaf), and the
 * sorted F and W concatenated in leaf order. */
int64_t orc_num_obs(const orc *o) {
    leafvec lv = {0};
    collect(o->root, &lv);
    int64_t s = 0;
    for (int64_t i = 0; i < lv.n; ++i) s += lv.a[i]->M;
    free(lv.a);
    return s;
}

int orc_leaf_obs(const orc *o, int32_t *M, double *wtot, double *inv, double *F, double *W) {
    if (!o || !o->root) return ORC_E_STATE;
    leafvec lv = {0};
    int st = collect(o->root, &lv);
    int64_t j = 0;
    for (int64_t i = 0; i < lv.n && !st; ++i) {
        unode *n = lv.a[i];
        M[i] = n->M;
        wtot[i] = (double)n->Wtot;
        inv[i] = (double)n->inv;
        for (int k = 0; k < n->M; ++k, ++j) {
            F[j] = (double)n->F[k];
            W[j] = (double)n->W[k];
        }
    }
    free(lv.a);
    return st;
}

/* Face adjacency: for every leaf and each of the 6 faces (+x,+y,+z,-x,-y,-z)
 * the count of neighbours, and their leaf indices concatenated in that order. */
int64_t orc_neighbours(const orc *o, int32_t *counts, int64_t cap, int64_t *idx) {
    if (!o || !o->root) return -1;
    leafvec lv = {0}, nb = {0};
    collect(o->root, &lv);
    int64_t j = 0;
    for (int64_t i = 0; i < lv.n; ++i) {
        unode *n = lv.a[i];
        for (int f = 0; f < 6; ++f) {
            neighbours(n, f % 3, f < 3 ? +1 : -1, &nb);
            if (counts) counts[6 * i + f] = (int32_t)nb.n;
            for (int64_t q = 0; q < nb.n; ++q, ++j) {
                if (idx && j < cap) {
                    /* index of the neighbour: binary search by key */
                    uint32_t kk = morton(nb.a[q]->x, nb.a[q]->y, nb.a[q]->z);
                    int64_t lo = 0, hi = lv.n - 1;
                    while (lo < hi) {
                        int64_t mid = (lo + hi) / 2;
                        unode *mm = lv.a[mid];
                        if (morton(mm->x, mm->y, mm->z) < kk) lo = mid + 1;
                        else hi = mid;
                    }
                    idx[j] = lo;
                }
            }
        }
    }
    free(lv.a);
    free(nb.a);
    return j;
}

/* G applied to per-leaf values u (in leaf order): g[3i+d]. */
int orc_apply_grad(const orc *o, const double *u, double *g) {
    leafvec lv = {0}, nb = {0};
    collect(o->root, &lv);
    real *saved = (real *)malloc(sizeof(real) * (size_t)lv.n);
    for (int64_t i = 0; i < lv.n; ++i) {
        saved[i] = lv.a[i]->ubar;
        lv.a[i]->ubar = (real)u[i];
    }
    for (int64_t i = 0; i < lv.n; ++i) {
        unode *n = lv.a[i];
        for (int d = 0; d < 3; ++d) {
            neighbours(n, d, +1, &nb);
            real acc = 0;
            for (int64_t j = 0; j < nb.n; ++j)
                acc = R_FMA(coef_grad(o, n, nb.a[j]), nb.a[j]->ubar - n->ubar, acc);
            g[3 * i + d] = (double)acc;
        }
    }
    for (int64_t i = 0; i < lv.n; ++i) lv.a[i]->ubar = saved[i];
    free(saved);
    free(lv.a);
    free(nb.a);
    return ORC_OK;
}

/* div applied to per-leaf vectors p (3 per leaf, leaf order). */
int orc_apply_div(const orc *o, const double *p, double *out) {
    leafvec lv = {0}, nb = {0};
    collect(o->root, &lv);
    real *saved = (real *)malloc(sizeof(real) * 3 * (size_t)lv.n);
    for (int64_t i = 0; i < lv.n; ++i)
        for (int d = 0; d < 3; ++d) {
            saved[3 * i + d] = lv.a[i]->p[d];
            lv.a[i]->p[d] = (real)p[3 * i + d];
        }
    for (int64_t i = 0; i < lv.n; ++i) {
        real v;
        div_leaf(o, lv.a[i], &nb, &v);
        out[i] = (double)v;
    }
    for (int64_t i = 0; i < lv.n; ++i)
        for (int d = 0; d < 3; ++d) lv.a[i]->p[d] = saved[3 * i + d];
    free(saved);
    free(lv.a);
    free(nb.a);
    return ORC_OK;
}

/* Energy [Eq. 3 with the normaliser of Eq. 5, lambda on the data term]:
 * tv = sum_n vol_n |(G u)_n|, data = sum_n vol_n inv_n sum_i W_i |u_n - F_i|;
 * E = tv + lambda * data. Accumulated in double. */
/* Smoothed energy terms of Eq. 4-5 (eps > 0): tv = sum vol sqrt(|Gu|^2 + eps^2),
 * data = sum vol inv sum W sqrt((u - F)^2 + eps^2); in double. With eps = 0
 * these are the exact terms of orc_energy. */
int orc_energy_eps(const orc *o, double eps, double *tv, double *data) {
    if (!o || !o->root) return ORC_E_STATE;
    const double e2 = eps * eps;
    leafvec lv = {0}, nb = {0};
    collect(o->root, &lv);
    double t = 0, dt = 0;
    for (int64_t i = 0; i < lv.n; ++i) {
        unode *n = lv.a[i];
        double vol = (double)side_of(o, n->level);
        vol = vol * vol * vol;
        double g2 = 0;
        for (int d = 0; d < 3; ++d) {
            neighbours(n, d, +1, &nb);
            double g = 0;
            for (int64_t j = 0; j < nb.n; ++j)
                g += (double)coef_grad(o, n, nb.a[j]) * ((double)nb.a[j]->u - (double)n->u);
            g2 += g * g;
        }
        t += vol * sqrt(g2 + e2);
        double s = 0;
        for (int k = 0; k < n->M; ++k) {
            double r = (double)n->u - (double)n->F[k];
            s += (double)n->W[k] * sqrt(r * r + e2);
        }
        dt += vol * (double)n->inv * s;
    }
    free(lv.a);
    free(nb.a);
    *tv = t;
    *data = dt;
    return ORC_OK;
}

int orc_energy(const orc *o, double *tv, double *data) {
    if (!o || !o->root) return ORC_E_STATE;
    leafvec lv = {0}, nb = {0};
    collect(o->root, &lv);
    double t = 0, dt = 0;
    for (int64_t i = 0; i < lv.n; ++i) {
        unode *n = lv.a[i];
        double vol = (double)side_of(o, n->level);
        vol = vol * vol * vol;
        double g2 = 0;
        for (int d = 0; d < 3; ++d) {
            neighbours(n, d, +1, &nb);
            double g = 0;
            for (int64_t j = 0; j < nb.n; ++j)
                g += (double)coef_grad(o, n, nb.a[j]) * ((double)nb.a[j]->u - (double)n->u);
            g2 += g * g;
        }
        t += vol * sqrt(g2);
        double s = 0;
        for (int k = 0; k < n->M; ++k) s += (double)n->W[k] * fabs((double)n->u - (double)n->F[k]);
        dt += vol * (double)n->inv * s;
    }
    free(lv.a);
    free(nb.a);
    *tv = t;
    *data = dt;
    return ORC_OK;
}

/* Standalone prox on unsorted observations (F_i, W_i > 0): sorts by (F, index),
 * forms prefix weights, normaliser 1/(sum W + gamma), and returns the median
 * with t = tl * normaliser. Test hook. */
double orc_prox(int M, const double *F, const double *W, double gamma, double uprime, double tl) {
    obs_t *o = (obs_t *)malloc(sizeof(obs_t) * (size_t)(M > 0 ? M : 1));
    for (int k = 0; k < M; ++k) {
        o[k].F = (real)F[k];
        o[k].W = (real)W[k];
        o[k].view = k;
    }
    qsort(o, (size_t)M, sizeof(obs_t), obs_cmp);
    real *Fs = (real *)malloc(sizeof(real) * (size_t)(M > 0 ? M : 1));
    real *Sk = (real *)malloc(sizeof(real) * (size_t)(M + 1));
    real *scr = (real *)malloc(sizeof(real) * (size_t)(2 * M + 1));
    real P = 0;
    for (int k = 0; k < M; ++k) {
        Fs[k] = o[k].F;
        P = P + o[k].W;
    }
    real inv = (real)1 / (P + (real)gamma);
    real Pk = 0;
    Sk[0] = R_FMA((real)2, Pk, -P);
    for (int k = 1; k <= M; ++k) {
        Pk = Pk + o[k - 1].W;
        Sk[k] = R_FMA((real)2, Pk, -P);
    }
    real r = prox_median(M, Fs, Sk, (real)uprime, (real)tl * inv, scr);
    free(o);
    free(Fs);
    free(Sk);
    free(scr);
    return (double)r;
}

/* ------------------------------------------------------------------------ */
/* State blob (little-endian).                                               */
/*   "OTF1" | u32 version=1 | params (40 B) | i64 iteration | i32 n_views |    */
/*   i32 0 | per view: i64 n_nodes, n_nodes x {u32 key, u8 level, u8 leaf,   */
/*   u16 0, f32 S, u32 cnt} sorted by (level, key) | i64 n_leaves,            */
/*   n_leaves x {u32 key, u8 level, u8[3] 0, f32 u, ubar, px, py, pz}        */
/*   sorted by key.                                                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    uint8_t *p;
    int64_t n, cap;
    int ovf;
} wbuf;

static void put(wbuf *b, const void *src, int64_t n) {
    if (b->p && b->n + n <= b->cap) memcpy(b->p + b->n, src, (size_t)n);
    else if (b->p) b->ovf = 1;
    b->n += n;
}

typedef struct {
    const vnode *n;
    uint32_t key;
    int level;
} vq_t;

int orc_export_state(const orc *o, void *buf, int64_t cap, int64_t *n_bytes) {
    if (!o || !o->root) return ORC_E_STATE;
    wbuf b = {(uint8_t *)buf, 0, cap, 0};
    put(&b, "OTF1", 4);
    uint32_t ver = 1;
    put(&b, &ver, 4);
    put(&b, &o->prm, sizeof(orc_params));
    put(&b, &o->iteration, 8);
    int32_t nv = o->n_views, zero = 0;
    put(&b, &nv, 4);
    put(&b, &zero, 4);
    for (int v = 0; v < o->n_views; ++v) {
        /* breadth-first = (level, key) order */
        int64_t cap_q = 1024, head = 0, tail = 0;
        vq_t *q = (vq_t *)malloc(sizeof(vq_t) * (size_t)cap_q);
        q[tail++] = (vq_t){&o->views[v], 0u, 0};
        while (head < tail) {
            vq_t e = q[head++];
            if (e.n->kid) {
                if (tail + 8 > cap_q) {
                    cap_q *= 2;
                    q = (vq_t *)realloc(q, sizeof(vq_t) * (size_t)cap_q);
                }
                int sh = 3 * (o->prm.max_depth - e.level - 1);
                for (int c = 0; c < 8; ++c) q[tail++] = (vq_t){&e.n->kid[c], e.key | ((uint32_t)c << sh), e.level + 1};
            }
        }
        int64_t nn = tail;
        put(&b, &nn, 8);
        for (int64_t i = 0; i < nn; ++i) {
            uint8_t lv = (uint8_t)q[i].level, lf = q[i].n->kid ? 0 : 1;
            uint16_t z16 = 0;
            float S = (float)q[i].n->S;
            uint32_t cnt = (uint32_t)q[i].n->cnt;
            put(&b, &q[i].key, 4);
            put(&b, &lv, 1);
            put(&b, &lf, 1);
            put(&b, &z16, 2);
            put(&b, &S, 4);
            put(&b, &cnt, 4);
        }
        free(q);
    }
    leafvec lv = {0};
    collect(o->root, &lv);
    put(&b, &lv.n, 8);
    for (int64_t i = 0; i < lv.n; ++i) {
        unode *n = lv.a[i];
        uint32_t key = morton(n->x, n->y, n->z);
        uint8_t l[4] = {(uint8_t)n->level, 0, 0, 0};
        float vals[5] = {(float)n->u, (float)n->ubar, (float)n->p[0], (float)n->p[1], (float)n->p[2]};
        put(&b, &key, 4);
        put(&b, l, 4);
        put(&b, vals, 20);
    }
    free(lv.a);
    *n_bytes = b.n;
    if (b.ovf || (buf && b.n > cap)) return set_err((orc *)o, "buffer too small"), ORC_E_INVALID;
    return ORC_OK;
}

typedef struct {
    const uint8_t *p;
    int64_t n, at;
    int bad;
} rbuf;

static void get(rbuf *b, void *dst, int64_t n) {
    if (b->bad || b->at + n > b->n) {
        b->bad = 1;
        memset(dst, 0, (size_t)n);
        return;
    }
    memcpy(dst, b->p + b->at, (size_t)n);
    b->at += n;
}

int orc_import_state(orc *o, const void *buf, int64_t n_bytes) {
    if (!o || !buf) return ORC_E_INVALID;
    rbuf b = {(const uint8_t *)buf, n_bytes, 0, 0};
    char magic[4];
    uint32_t ver;
    orc_params prm;
    int64_t iter;
    int32_t nv, zero;
    get(&b, magic, 4);
    get(&b, &ver, 4);
    get(&b, &prm, sizeof prm);
    get(&b, &iter, 8);
    get(&b, &nv, 4);
    get(&b, &zero, 4);
    if (b.bad || memcmp(magic, "OTF1", 4) || ver != 1) return set_err(o, "bad blob header"), ORC_E_INVALID;
    int st = check_params(o, &prm, nv);
    if (st) return st;
    clear(o);
    o->prm = prm;
    o->iteration = iter;
    o->n_views = nv;
    o->views = (vnode *)calloc((size_t)nv, sizeof(vnode));
    for (int v = 0; v < nv; ++v) {
        int64_t nn;
        get(&b, &nn, 8);
        if (b.bad || nn < 1) return set_err(o, "bad view tree"), ORC_E_INVALID;
        /* nodes arrive in (level, key) order: the j-th group of 8 at level l+1
         * are the children of the j-th inner node at level l */
        vnode **inner = (vnode **)malloc(sizeof(vnode *) * (size_t)nn);
        uint32_t *ikey = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)nn);
        int *ilev = (int *)malloc(sizeof(int) * (size_t)nn);
        int64_t ni = 0, used = 0;
        for (int64_t i = 0; i < nn; ++i) {
            uint32_t key, cnt;
            uint8_t lv, lf;
            uint16_t z16;
            float S;
            get(&b, &key, 4);
            get(&b, &lv, 1);
            get(&b, &lf, 1);
            get(&b, &z16, 2);
            get(&b, &S, 4);
            get(&b, &cnt, 4);
            vnode *n;
            if (i == 0) {
                if (lv != 0 || key != 0) b.bad = 1;
                n = &o->views[v];
            } else {
                int64_t par = (i - 1) / 8, c = (i - 1) % 8;
                if (par >= ni) {
                    b.bad = 1;
                    break;
                }
                int sh = 3 * (prm.max_depth - ilev[par] - 1);
                if (lv != ilev[par] + 1 || key != (ikey[par] | ((uint32_t)c << sh))) b.bad = 1;
                n = &inner[par]->kid[c];
                used = par + 1;
            }
            n->S = (real)S;
            n->cnt = cnt;
            n->kid = NULL;
            if (!lf) {
                n->kid = (vnode *)calloc(8, sizeof(vnode));
                inner[ni] = n;
                ikey[ni] = key;
                ilev[ni] = lv;
                ++ni;
            }
            if (b.bad) break;
        }
        if (!b.bad && (nn - 1) != 8 * ni) b.bad = 1;
        (void)used;
        free(inner);
        free(ikey);
        free(ilev);
        if (b.bad) return set_err(o, "inconsistent view tree"), ORC_E_INVALID;
    }
    int64_t nl;
    get(&b, &nl, 8);
    if (b.bad || nl < 1) return set_err(o, "bad leaf count"), ORC_E_INVALID;
    o->root = (unode *)calloc(1, sizeof(unode));
    double vol = 0, full = ldexp(1.0, 3 * prm.max_depth);
    uint32_t prev = 0;
    for (int64_t i = 0; i < nl; ++i) {
        uint32_t key;
        uint8_t l[4];
        float vals[5];
        get(&b, &key, 4);
        get(&b, l, 4);
        get(&b, vals, 20);
        if (b.bad || l[0] > prm.max_depth || (i > 0 && key <= prev)) return set_err(o, "bad leaf"), ORC_E_INVALID;
        prev = key;
        uint32_t x, y, z;
        demorton(key, &x, &y, &z);
        unode *n = o->root;
        for (int lv = 0; lv < l[0]; ++lv) {
            if (!n->kid) {
                if (n->M < 0) return set_err(o, "overlapping leaves"), ORC_E_INVALID;
                if (make_kids(o, n)) return ORC_E_NOMEM;
            }
            uint32_t hs = side_of(o, lv + 1);
            int c = (int)((x / hs) & 1u) | (int)(((y / hs) & 1u) << 1) | (int)(((z / hs) & 1u) << 2);
            n = &n->kid[c];
        }
        if (n->kid || n->M < 0 || n->x != x || n->y != y || n->z != z)
            return set_err(o, "overlapping or misaligned leaves"), ORC_E_INVALID;
        n->M = -1; /* marks an assigned leaf until observations are gathered */
        n->u = (real)vals[0];
        n->ubar = (real)vals[1];
        n->p[0] = (real)vals[2];
        n->p[1] = (real)vals[3];
        n->p[2] = (real)vals[4];
        double s = ldexp(1.0, prm.max_depth - l[0]);
        vol += s * s * s;
    }
    if (vol != full) return set_err(o, "leaves do not tile the domain"), ORC_E_INVALID;
    leafvec lv = {0};
    collect(o->root, &lv);
    st = ORC_OK;
    for (int64_t i = 0; i < lv.n && !st; ++i) {
        lv.a[i]->M = 0;
        st = gather_obs(o, lv.a[i]);
    }
    free(lv.a);
    return st;
}
