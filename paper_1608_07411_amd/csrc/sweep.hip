// The two leaf sweeps of one primal-dual iteration and the energy reduction.
//
// Dual sweep (gradient + ascent + unit-ball projection):
//   g_d = sum_{k in N+_d(n)} c_nk (ubar_k - ubar_n)   ascending key, fma chain
//   q   = p + sigma g,  p = q / max(1, |q|)
//   ds  = C+_x p_x + C+_y p_y + C+_z p_z              C+_d = sum_k c_nk
// Primal sweep (divergence + generalised shrinkage + extrapolation + flags):
//   div = ds - sum_d sum_{m in N-_d(n)} c'_mn p_{m,d}
//   u'  = u + tau div
//   u+  = median of {F_(1..M)} and {u' - t S_k}, t = tau lambda / (sum W + gamma),
//         S_k = 2 P_k - W_tot: the smallest k with u' - t S_k <= F_(k+1) selects
//         max(u' - t S_k, F_(k)) (the median of the 2M+1 values)
//   ubar = 2 u+ - u,  u = u+
//   flags: split if |u+| < tau_s below max depth, joinable if |u+| > tau_j.
// Every floating-point operation is a single IEEE operation in a fixed order.
#include "otf_internal.h"

namespace otf {
namespace {

constexpr int kBlk = 256;

struct DualArgs {
    int64_t L, cap;
    const uint8_t *level;
    const float *ubar;
    const uint32_t *off;
    const uint32_t *ent;
    float *p;
    float *ds;
    float sigma;
};

__global__ void __launch_bounds__(kBlk) k_dual(DualArgs a, Coef cf) {
    const int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    if (i >= a.L) return;
    const int ln = a.level[i];
    const float ub = a.ubar[i];
    float gx = 0.0f, gy = 0.0f, gz = 0.0f, Cx = 0.0f, Cy = 0.0f, Cz = 0.0f;
    const uint32_t e1 = a.off[i + 1];
    for (uint32_t e = a.off[i]; e < e1; ++e) {
        const uint32_t v = a.ent[e];
        const uint32_t k = v & kIdxMask;
        const int d = (v >> kIdxBits) & 3;
        const int lk = v >> (kIdxBits + 2);
        const float c = cf.c[ln][lk];
        const float diff = a.ubar[k] - ub;
        if (d == 0) {
            gx = __fmaf_rn(c, diff, gx);
            Cx = Cx + c;
        } else if (d == 1) {
            gy = __fmaf_rn(c, diff, gy);
            Cy = Cy + c;
        } else {
            gz = __fmaf_rn(c, diff, gz);
            Cz = Cz + c;
        }
    }
    float qx = __fmaf_rn(a.sigma, gx, a.p[i]);
    float qy = __fmaf_rn(a.sigma, gy, a.p[a.cap + i]);
    float qz = __fmaf_rn(a.sigma, gz, a.p[2 * a.cap + i]);
    const float r2 = __fmaf_rn(qx, qx, __fmaf_rn(qy, qy, qz * qz));
    if (r2 > 1.0f) {
        const float nrm = sqrtf(r2);
        qx = qx / nrm;
        qy = qy / nrm;
        qz = qz / nrm;
    }
    a.p[i] = qx;
    a.p[a.cap + i] = qy;
    a.p[2 * a.cap + i] = qz;
    a.ds[i] = __fmaf_rn(Cz, qz, __fmaf_rn(Cy, qy, __fmaf_rn(Cx, qx, 0.0f)));
}

struct PrimalArgs {
    int64_t L, cap;
    const uint8_t *level;
    const float *ds;
    const float *p;
    const uint32_t *off;
    const uint32_t *ent;
    const uint32_t *obs_off;
    const uint8_t *obs_m, *obs_unit;
    const float *inv, *wtot;
    const float *F, *W;
    float *u, *ubar;
    uint8_t *flag;
    float *uprime, *uold;
    uint32_t *counters;  // [0] split flags, [1] join flags
    float tau, tl, split_tau, join_tau;
    int join_enabled, max_depth;
};

__global__ void __launch_bounds__(kBlk) k_primal(PrimalArgs a, Coef cf) {
    const int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    bool split = false, join = false;
    if (i < a.L) {
        const int ln = a.level[i];
        float acc = a.ds[i];
        const uint32_t e1 = a.off[i + 1];
        for (uint32_t e = a.off[i]; e < e1; ++e) {
            const uint32_t v = a.ent[e];
            const uint32_t m = v & kIdxMask;
            const int d = (v >> kIdxBits) & 3;
            const int lm = v >> (kIdxBits + 2);
            acc = __fmaf_rn(-cf.cp[lm][ln], a.p[(int64_t)d * a.cap + m], acc);
        }
        const float un = a.u[i];
        const float up = __fmaf_rn(a.tau, acc, un);
        const int M = a.obs_m[i];
        const uint32_t oo = a.obs_off[i];
        const float val = prox_select(up, a.tl * a.inv[i], M, a.obs_unit[i] != 0, a.F + oo, a.W + oo, a.wtot[i]);
        a.ubar[i] = __fmaf_rn(2.0f, val, -un);
        a.u[i] = val;
        const float av = fabsf(val);
        split = av < a.split_tau && ln < a.max_depth;
        join = a.join_enabled && av > a.join_tau;
        uint8_t fl = split ? 1 : (join ? (val > 0.0f ? 2 : 4) : 0);
        a.flag[i] = fl;
        if (split) {
            a.uprime[i] = up;
            a.uold[i] = un;
        }
    }
    const uint64_t bs = __ballot(split), bj = __ballot(join);
    if ((threadIdx.x & 63) == 0) {
        if (bs) atomicAdd(&a.counters[0], (uint32_t)__popcll(bs));
        if (bj) atomicAdd(&a.counters[1], (uint32_t)__popcll(bj));
    }
}

// Energy: per-leaf terms in double, block partial sums in a fixed tree order.
__global__ void __launch_bounds__(kBlk) k_energy(int64_t L, int D, const uint8_t *level, const float *u,
                                                 const uint32_t *off, const uint32_t *ent, const uint32_t *obs_off,
                                                 const uint8_t *obs_m, const float *inv, const float *F,
                                                 const float *W, Coef cf, double *partial) {
    __shared__ double s_tv[kBlk], s_da[kBlk];
    const int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    double tv = 0.0, da = 0.0;
    if (i < L) {
        const int ln = level[i];
        const double un = u[i];
        double g[3] = {0.0, 0.0, 0.0};
        for (uint32_t e = off[i]; e < off[i + 1]; ++e) {
            const uint32_t v = ent[e];
            const int d = (v >> kIdxBits) & 3;
            const int lk = v >> (kIdxBits + 2);
            const double c = cf.c[ln][lk];
            const double dif = (double)u[v & kIdxMask] - un;
            if (d == 0) g[0] += c * dif;
            else if (d == 1) g[1] += c * dif;
            else g[2] += c * dif;
        }
        const double s = ldexp(1.0, D - ln);
        const double vol = s * s * s;
        tv = vol * sqrt(g[0] * g[0] + g[1] * g[1] + g[2] * g[2]);
        double acc = 0.0;
        const uint32_t o = obs_off[i];
        for (int k = 0; k < obs_m[i]; ++k) acc += (double)W[o + k] * fabs(un - (double)F[o + k]);
        da = vol * (double)inv[i] * acc;
    }
    s_tv[threadIdx.x] = tv;
    s_da[threadIdx.x] = da;
    __syncthreads();
    for (int st = kBlk / 2; st > 0; st >>= 1) {
        if ((int)threadIdx.x < st) {
            s_tv[threadIdx.x] += s_tv[threadIdx.x + st];
            s_da[threadIdx.x] += s_da[threadIdx.x + st];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partial[2 * blockIdx.x] = s_tv[0];
        partial[2 * blockIdx.x + 1] = s_da[0];
    }
}

}  // namespace

void launch_dual(Ctx &c, float sigma) {
    LeafStore &s = c.lv();
    DualArgs a{c.L, s.cap, s.level.p, s.ubar.p, s.nbp_off.p, s.nbp.p, s.p.p, s.ds.p, sigma};
    hipLaunchKernelGGL(k_dual, dim3((unsigned)cdiv(c.L, kBlk)), dim3(kBlk), 0, c.stream, a, c.coef);
    OTF_LAUNCH_CHECK("k_dual");
}

void launch_primal(Ctx &c, float tau, float tl) {
    LeafStore &s = c.lv();
    PrimalArgs a;
    a.L = c.L;
    a.cap = s.cap;
    a.level = s.level.p;
    a.ds = s.ds.p;
    a.p = s.p.p;
    a.off = s.nbm_off.p;
    a.ent = s.nbm.p;
    a.obs_off = s.obs_off.p;
    a.obs_m = s.obs_m.p;
    a.obs_unit = s.obs_unit.p;
    a.inv = s.inv.p;
    a.wtot = s.wtot.p;
    a.F = c.op().F.p;
    a.W = c.op().W.p;
    a.u = s.u.p;
    a.ubar = s.ubar.p;
    a.flag = s.flag.p;
    a.uprime = s.uprime.p;
    a.uold = s.uold.p;
    a.counters = c.counters.p;
    a.tau = tau;
    a.tl = tl;
    a.split_tau = c.prm.split_tau;
    a.join_tau = c.prm.join_tau;
    a.join_enabled = !(c.prm.join_tau > 1.0f);
    a.max_depth = c.prm.max_depth;
    hipLaunchKernelGGL(k_primal, dim3((unsigned)cdiv(c.L, kBlk)), dim3(kBlk), 0, c.stream, a, c.coef);
    OTF_LAUNCH_CHECK("k_primal");
}

void energy(Ctx &c, double *tv, double *data) {
    LeafStore &s = c.lv();
    const int64_t blocks = cdiv(c.L, kBlk);
    c.s.dred.reserve(2 * blocks);
    hipLaunchKernelGGL(k_energy, dim3((unsigned)blocks), dim3(kBlk), 0, c.stream, c.L, c.prm.max_depth, s.level.p,
                       s.u.p, s.nbp_off.p, s.nbp.p, s.obs_off.p, s.obs_m.p, s.inv.p, c.op().F.p, c.op().W.p, c.coef,
                       c.s.dred.p);
    OTF_LAUNCH_CHECK("k_energy");
    std::vector<double> h(2 * blocks);
    OTF_HIP(hipMemcpyAsync(h.data(), c.s.dred.p, h.size() * sizeof(double), hipMemcpyDeviceToHost, c.stream));
    OTF_HIP(hipStreamSynchronize(c.stream));
    double t = 0.0, d = 0.0;
    for (int64_t b = 0; b < blocks; ++b) {
        t += h[2 * b];
        d += h[2 * b + 1];
    }
    *tv = t;
    *data = d;
}

}  // namespace otf
