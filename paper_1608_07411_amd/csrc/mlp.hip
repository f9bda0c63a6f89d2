// Learned warm start: a per-leaf network predicts how far the converged fused
// value u of every leaf lies from its start, and its converged dual p, from
// the leaf's sorted observations and its neighbourhood, so that the
// primal-dual iteration (Sec. 3.2) starts closer to its solution.
//
// Network: 32 features -> 128 -> 128 -> 128 -> 4 (change of u, px, py, pz), ReLU on the
// hidden layers. Weights and activations are bfloat16, products accumulate in
// fp32 on the matrix cores (v_mfma_f32_16x16x32 bf16), biases and the master
// weights (Adam) are fp32. Parameter vector: per layer W (in x out,
// row-major) then b.
//
// Features of a leaf: 16 quantiles of its observations (they are stored
// sorted by F), the mean u of its neighbours across each of the 6 faces, its
// u, its normalised weight sum W/(W + gamma), M/64, level/max_depth, zeros.
#include <algorithm>
#include <cmath>
#include <new>
#include <vector>

#include "otf_internal.h"

namespace otf {
namespace {

constexpr int kBlk = 256;
constexpr int kIn = 32, kHid = 128, kOut = 4, kLayers = 4;
constexpr int kSizes[kLayers + 1] = {kIn, kHid, kHid, kHid, kOut};

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// 8 consecutive bf16 values (16 bytes, 16-byte aligned) as an MFMA operand
__device__ inline bf16x8 ld8(const uint16_t *p) {
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const uint4 *>(p));
}

__device__ inline uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);  // nearest, ties to even
    return (uint16_t)(u >> 16);
}
__device__ inline float bf2f(uint16_t b) { return __uint_as_float((uint32_t)b << 16); }

// C(m, n) = sum_k A(m, k) B(k, n); A(m, k) = A[m sam + k sak], B(k, n) =
// B[k sbk + n sbn] (the strides express transposes). A block computes a
// 64 x 64 tile of C: per step of 32 over k it stages the 64 x 32 slices of A
// and of B^T in LDS (coalesced: along k when k is the contiguous index,
// else along the rows), and each of its 4 waves multiplies a 32 x 32 quarter
// as 2 x 2 v_mfma_f32_16x16x32 bf16 steps (lane l: row or column l % 16,
// k = 8 (l / 16) .. + 7). With gridDim.z > 1 the k range is split: block z
// writes its partial sum to C + z M N and k_sum_splits adds them. Epilogue
// (one split): + bias[n], then ReLU, or the ReLU mask of a stored activation
// (v = mask(m, n) > 0 ? v : 0); fp32 to C and/or bf16 to Cb (row-major M x N).
constexpr int kTM = 64, kTN = 64, kTK = 32;
constexpr int kTP = kTK + 8;  // LDS row pitch (bf16 elements): 16-byte aligned rows

// Rows [r0, r0 + 64) x k [k0, k0 + 32) of X(r, k) = X[r sr + k sk] into
// t[r][k] (zeros outside R x [k0, ke)).
__device__ inline void stage_slice(const uint16_t *X, int R, int64_t ke, int64_t sr, int64_t sk, int r0, int64_t k0,
                                   uint16_t *t) {
    const int tid = threadIdx.x;
    uint16_t v[8];
    if (sk == 1) {  // k contiguous: 8 consecutive k of one row per thread
        const int r = tid >> 2, kc = (tid & 3) * 8;
        const int64_t row = r0 + r, k = k0 + kc;
        const uint16_t *src = X + row * sr + k;
        if (row < R && k + 8 <= ke && ((uintptr_t)src & 15) == 0) {
            *reinterpret_cast<uint4 *>(t + r * kTP + kc) = *reinterpret_cast<const uint4 *>(src);
            return;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) v[j] = (row < R && k + j < ke) ? src[j] : (uint16_t)0;
#pragma unroll
        for (int j = 0; j < 8; ++j) t[r * kTP + kc + j] = v[j];
    } else {  // rows contiguous: 8 consecutive rows of one k per thread
        const int kk = tid >> 3, rc = (tid & 7) * 8;
        const int64_t k = k0 + kk;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
            const int64_t row = r0 + rc + j;
            v[j] = (row < R && k < ke) ? X[row * sr + k * sk] : (uint16_t)0;
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) t[(rc + j) * kTP + kk] = v[j];
    }
}

__global__ void __launch_bounds__(kBlk) k_gemm(int M, int N, int64_t K, const uint16_t *A, int64_t sam, int64_t sak,
                                               const uint16_t *B, int64_t sbk, int64_t sbn, float *C, uint16_t *Cb,
                                               int64_t kchunk, const float *bias, int relu, const uint16_t *mask) {
    __shared__ __align__(16) uint16_t ta[kTM * kTP];
    __shared__ __align__(16) uint16_t tb[kTN * kTP];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int m0 = blockIdx.x * kTM, n0 = blockIdx.y * kTN;
    const int wm = (w >> 1) * 32, wn = (w & 1) * 32;
    const int64_t kb = (int64_t)blockIdx.z * kchunk, ke = min(K, kb + kchunk);
    const int r16 = lane & 15, kq = 8 * (lane >> 4);
    f32x4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
    for (int64_t k0 = kb; k0 < ke; k0 += kTK) {
        stage_slice(A, M, ke, sam, sak, m0, k0, ta);
        stage_slice(B, N, ke, sbn, sbk, n0, k0, tb);  // B^T(n, k) = B(k, n)
        __syncthreads();
        bf16x8 a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = ld8(ta + (wm + 16 * i + r16) * kTP + kq);
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = ld8(tb + (wn + 16 * j + r16) * kTP + kq);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
        __syncthreads();
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) {
            const int nc = n0 + wn + 16 * j + r16;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int row = m0 + wm + 16 * i + 4 * (lane >> 4) + r;
                if (row >= M || nc >= N) continue;
                float v = acc[i][j][r];
                if (gridDim.z > 1) {
                    C[(int64_t)blockIdx.z * M * N + (int64_t)row * N + nc] = v;
                    continue;
                }
                if (bias) v = v + bias[nc];
                if (relu) v = fmaxf(v, 0.0f);
                if (mask && !(bf2f(mask[(int64_t)row * N + nc]) > 0.0f)) v = 0.0f;
                if (C) C[(int64_t)row * N + nc] = v;
                if (Cb) Cb[(int64_t)row * N + nc] = f2bf(v);
            }
        }
}

// out[e] = sum over z < splits of part[z n + e]: one wave per element, lane
// l adding partials l, l + 64, ... in order, then a fixed shuffle tree (a
// deterministic order; the split partials of a long reduction are many, so
// they are spread over the lanes rather than walked by one thread)
__global__ void k_sum_splits(const float *part, int splits, int64_t n, float *out) {
    const int64_t e = (int64_t)blockIdx.x * (kBlk / 64) + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (e >= n) return;  // the whole wave
    float s = 0.0f;
    for (int z = lane; z < splits; z += 64) s = s + part[(int64_t)z * n + e];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) s = s + __shfl_down(s, o, 64);
    if (lane == 0) out[e] = s;
}

// Per-block column sums of a bf16 matrix (rows x N, N <= kBlk) over `chunk`
// rows: with G = kBlk / N row phases, thread t sums column t % N over rows
// r0 + t / N, r0 + t / N + G, ... (a wave's loads cover whole rows), then
// the G phase sums of each column are added in phase order.
constexpr int kColRows = 16;  // rows per thread and block
__global__ void __launch_bounds__(kBlk) k_colsum(const uint16_t *Z, int64_t rows, int N, int64_t chunk,
                                                 float *part) {
    __shared__ float sh[kBlk];
    const int t = threadIdx.x, G = kBlk / N, c = t % N, g = t / N;
    const int64_t r0 = (int64_t)blockIdx.x * chunk, r1 = min(rows, r0 + chunk);
    float s = 0.0f;
    if (g < G) {
        float v[kColRows];
#pragma unroll
        for (int k = 0; k < kColRows; ++k) {
            const int64_t r = r0 + g + (int64_t)k * G;
            v[k] = r < r1 ? bf2f(Z[r * N + c]) : 0.0f;
        }
#pragma unroll
        for (int k = 0; k < kColRows; ++k) s = s + v[k];
        for (int64_t r = r0 + g + (int64_t)kColRows * G; r < r1; r += G) s = s + bf2f(Z[r * N + c]);
    }
    sh[t] = s;
    __syncthreads();
    if (t < N) {
        float acc = 0.0f;
        for (int k = 0; k < G; ++k) acc = acc + sh[k * N + t];
        part[(int64_t)blockIdx.x * N + t] = acc;
    }
}

__global__ void k_to_bf16(const float *x, int64_t n, uint16_t *y) {
    const int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    if (i < n) y[i] = f2bf(x[i]);
}

// dZ = bf16(2 (Y - T) / (rows * kOut)); per-block sums of (Y - T)^2 in double
__global__ void k_mse(const float *Y, const float *T, int64_t n, float scale, uint16_t *dZ, double *part) {
    __shared__ double red[kBlk];
    const int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    double sq = 0.0;
    if (i < n) {
        const float d = Y[i] - T[i];
        dZ[i] = f2bf(scale * d);
        sq = (double)d * (double)d;
    }
    red[threadIdx.x] = sq;
    __syncthreads();
    for (int s = kBlk / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

__global__ void k_adam(float *w, float *m, float *v, const float *g, int64_t n, float lr, float b1, float b2,
                       float c1, float c2, float eps) {
    const int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] = w[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// features of leaf i (row i of X, 32 floats)
__global__ void k_features(int64_t L, int D, float gamma, const uint8_t *level, const float *u,
                           const uint32_t *obs_off, const uint8_t *obs_m, const float *wtot, const float *F,
                           const uint32_t *offp, const uint32_t *entp, const uint32_t *offm, const uint32_t *entm,
                           float *X) {
    const int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    if (i >= L) return;
    float *x = X + i * kIn;
    const int M = obs_m[i];
    const uint32_t oo = obs_off[i];
    for (int k = 0; k < 16; ++k) x[k] = M > 0 ? F[oo + (uint32_t)(((2 * k + 1) * M) / 32)] : 0.0f;
    for (int side = 0; side < 2; ++side) {
        const uint32_t *off = side ? offm : offp, *ent = side ? entm : entp;
        float s[3] = {0.0f, 0.0f, 0.0f};
        int n[3] = {0, 0, 0};
        for (uint32_t e = off[i]; e < off[i + 1]; ++e) {
            const uint32_t v = ent[e];
            const int d = (v >> kIdxBits) & 3;
            s[d] = s[d] + u[v & kIdxMask];
            n[d] += 1;
        }
        for (int d = 0; d < 3; ++d) x[16 + 3 * side + d] = n[d] ? s[d] / (float)n[d] : 0.0f;
    }
    x[22] = u[i];
    x[23] = wtot[i] / (wtot[i] + gamma);
    x[24] = (float)M / 64.0f;
    x[25] = (float)level[i] / (float)D;
    for (int k = 26; k < kIn; ++k) x[k] = 0.0f;
}

// leaf targets / warm start: rows (u, px, py, pz)
__global__ void k_targets(int64_t L, int64_t cap, const float *u, const float *p, float *T) {
    const int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    if (i >= L) return;
    T[4 * i] = u[i];
    T[4 * i + 1] = p[i];
    T[4 * i + 2] = p[cap + i];
    T[4 * i + 3] = p[2 * cap + i];
}

// the prediction applied: output 0 is the change of u (u <- u + y0, kept in
// the TSDF range [-1, 1]; ubar = u), outputs 1..3 are p, projected onto the
// unit ball as the dual constraint requires
__global__ void k_apply_warm(int64_t L, int64_t cap, const float *Y, float *u, float *ubar, float *p) {
    const int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    if (i >= L) return;
    const float v = fminf(1.0f, fmaxf(-1.0f, u[i] + Y[4 * i]));
    u[i] = v;
    ubar[i] = v;
    float q[3] = {Y[4 * i + 1], Y[4 * i + 2], Y[4 * i + 3]};
    const float r2 = __fmaf_rn(q[0], q[0], __fmaf_rn(q[1], q[1], q[2] * q[2]));
    if (r2 > 1.0f) {
        const float nrm = sqrtf(r2);
        for (int d = 0; d < 3; ++d) q[d] = q[d] / nrm;
    }
    for (int d = 0; d < 3; ++d) p[(int64_t)d * cap + i] = q[d];
}

// The prediction applied at step alpha from the start (u0, p0): u = u0 +
// alpha y0 (one rounding) kept in [-1, 1], ubar = u, p = (1 - alpha) p0 +
// alpha q with q the projected prediction (a point of the unit ball again).
// alpha = 1 gives k_apply_warm's values.
__global__ void k_apply_warm_alpha(int64_t L, int64_t cap, const float *Y, const float *u0, const float *p0,
                                   float alpha, float *u, float *ubar, float *p) {
    const int64_t i = (int64_t)blockIdx.x * kBlk + threadIdx.x;
    if (i >= L) return;
    const float v = fminf(1.0f, fmaxf(-1.0f, __fmaf_rn(alpha, Y[4 * i], u0[i])));
    u[i] = v;
    ubar[i] = v;
    float q[3] = {Y[4 * i + 1], Y[4 * i + 2], Y[4 * i + 3]};
    const float r2 = __fmaf_rn(q[0], q[0], __fmaf_rn(q[1], q[1], q[2] * q[2]));
    if (r2 > 1.0f) {
        const float nrm = sqrtf(r2);
        for (int d = 0; d < 3; ++d) q[d] = q[d] / nrm;
    }
    for (int d = 0; d < 3; ++d) {
        const int64_t k = (int64_t)d * cap + i;
        p[k] = __fmaf_rn(alpha, q[d], (1.0f - alpha) * p0[k]);
    }
}

// Inference forward in one launch. A block holds every layer's weights
// (transposed, bf16: row n of W^T is column n of W) and biases in LDS; each
// wave takes a tile of 16 rows through the four layers, its activations
// staged in LDS between layers as bf16 (the values the layered forward
// stores). Operands, the order of the MFMA steps over k and the epilogue
// (+ bias, ReLU, bf16 rounding) are k_gemm's, so the outputs equal the
// layered forward's bit for bit; only the features are read and the 4
// outputs written. Row pitches of 8 extra elements keep the 16-byte operand
// reads aligned.
constexpr int kFusedWaves = 4;
constexpr int kPitchIn = kIn + 8, kPitchHid = kHid + 8;  // 16-byte aligned rows
struct __align__(16) FusedLds {
    uint16_t w0[kHid * kPitchIn];
    uint16_t w1[kHid * kPitchHid];
    uint16_t w2[kHid * kPitchHid];
    uint16_t w3[16 * kPitchHid];  // 4 outputs padded to 16 columns of zeros
    float b[3 * kHid + 16];
    uint16_t x[kFusedWaves][16 * kPitchIn];
    uint16_t h[kFusedWaves][2][16 * kPitchHid];
};

// W (K x N, row-major bf16) into W^T rows of pitch `pitch`
__device__ inline void stage_wt(const uint16_t *W, int K, int N, uint16_t *wt, int pitch) {
    for (int idx = threadIdx.x; idx < K * N; idx += blockDim.x) wt[(idx % N) * pitch + idx / N] = W[idx];
}

// One layer of the wave's tile: out(16 x 16 NT) = in(16 x K) W + b, as k_gemm
// computes each 16 x 16 output tile.
template <int K, int NT>
__device__ inline void fused_layer(const uint16_t *in, int pin, const uint16_t *wt, int pw, const float *bias,
                                   uint16_t *out, int pout, int lane) {
    const int r16 = lane & 15, kq = 8 * (lane >> 4), rq = 4 * (lane >> 4);
    for (int t = 0; t < NT; ++t) {
        f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int k0 = 0; k0 < K; k0 += 32) {
            const bf16x8 a = ld8(in + r16 * pin + k0 + kq);
            const bf16x8 b = ld8(wt + (t * 16 + r16) * pw + k0 + kq);
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const float v = fmaxf(acc[r] + bias[t * 16 + r16], 0.0f);
            out[(rq + r) * pout + t * 16 + r16] = f2bf(v);
        }
    }
}

__global__ void __launch_bounds__(64 * kFusedWaves) k_mlp_forward(const float *X, int64_t rows,
                                                                  const uint16_t *wbf, const float *theta,
                                                                  int64_t ow0, int64_t ow1, int64_t ow2, int64_t ow3,
                                                                  int64_t ob0, int64_t ob1, int64_t ob2, int64_t ob3,
                                                                  float *Y) {
    __shared__ FusedLds s;
    stage_wt(wbf + ow0, kIn, kHid, s.w0, kPitchIn);
    stage_wt(wbf + ow1, kHid, kHid, s.w1, kPitchHid);
    stage_wt(wbf + ow2, kHid, kHid, s.w2, kPitchHid);
    for (int i = threadIdx.x; i < 16 * kPitchHid; i += blockDim.x) s.w3[i] = 0;
    __syncthreads();
    stage_wt(wbf + ow3, kHid, kOut, s.w3, kPitchHid);
    for (int i = threadIdx.x; i < kHid; i += blockDim.x) {
        s.b[i] = theta[ob0 + i];
        s.b[kHid + i] = theta[ob1 + i];
        s.b[2 * kHid + i] = theta[ob2 + i];
    }
    if (threadIdx.x < 16) s.b[3 * kHid + threadIdx.x] = threadIdx.x < kOut ? theta[ob3 + threadIdx.x] : 0.0f;
    __syncthreads();
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int64_t ntiles = (rows + 15) / 16;
    // block-uniform loop: every wave of the block takes one tile per round
    for (int64_t g = blockIdx.x; g * kFusedWaves < ntiles; g += gridDim.x) {
        const int64_t m0 = (g * kFusedWaves + wv) * 16;
        {  // the tile's features to bf16: lane takes 8 of row lane / 4
            const int r = lane >> 2, k = (lane & 3) * 8;
            const int64_t row = m0 + r;
            for (int j = 0; j < 8; ++j)
                s.x[wv][r * kPitchIn + k + j] = row < rows ? f2bf(X[row * kIn + k + j]) : (uint16_t)0;
        }
        __syncthreads();
        fused_layer<kIn, kHid / 16>(s.x[wv], kPitchIn, s.w0, kPitchIn, s.b, s.h[wv][0], kPitchHid, lane);
        __syncthreads();
        fused_layer<kHid, kHid / 16>(s.h[wv][0], kPitchHid, s.w1, kPitchHid, s.b + kHid, s.h[wv][1], kPitchHid, lane);
        __syncthreads();
        fused_layer<kHid, kHid / 16>(s.h[wv][1], kPitchHid, s.w2, kPitchHid, s.b + 2 * kHid, s.h[wv][0], kPitchHid,
                                     lane);
        __syncthreads();
        {  // output layer: fp32, no ReLU; lane holds column r16 of rows rq..rq+3
            const int r16 = lane & 15, kq = 8 * (lane >> 4), rq = 4 * (lane >> 4);
            f32x4 acc = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int k0 = 0; k0 < kHid; k0 += 32) {
                const bf16x8 a = ld8(s.h[wv][0] + r16 * kPitchHid + k0 + kq);
                const bf16x8 b = ld8(s.w3 + r16 * kPitchHid + k0 + kq);
                acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc, 0, 0, 0);
            }
            if (r16 < kOut)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int64_t row = m0 + rq + r;
                    if (row < rows) Y[row * kOut + r16] = acc[r] + s.b[3 * kHid + r16];
                }
        }
        __syncthreads();
    }
}

unsigned g1(int64_t n) { return (unsigned)cdiv(n > 0 ? n : 1, kBlk); }

}  // namespace

struct Mlp {
    int device = 0;
    hipStream_t stream = nullptr;
    int64_t n_params = 0;
    int64_t off_w[kLayers], off_b[kLayers];
    DBuf<float> theta, m, v, grad, Y, part;
    DBuf<double> lpart;
    DBuf<uint16_t> wbf, X, H[kLayers], dZ, dZ2;
    DBuf<float> dH;
    int64_t step = 0;
    std::string err;

    Mlp() {
        int64_t at = 0;
        for (int l = 0; l < kLayers; ++l) {
            off_w[l] = at;
            at += (int64_t)kSizes[l] * kSizes[l + 1];
            off_b[l] = at;
            at += kSizes[l + 1];
        }
        n_params = at;
    }

    void sync_bf16() {
        hipLaunchKernelGGL(k_to_bf16, dim3(g1(n_params)), dim3(kBlk), 0, stream, theta.p, n_params, wbf.p);
        OTF_LAUNCH_CHECK("k_to_bf16");
    }

    // C = A B with the epilogue of k_gemm; split over k when K is long
    void gemm(int M, int N, int64_t K, const uint16_t *A, int64_t sam, int64_t sak, const uint16_t *B, int64_t sbk,
              int64_t sbn, float *C, uint16_t *Cb, const float *bias, int relu, const uint16_t *mask) {
        const unsigned gx = (unsigned)cdiv(M, kTM), gy = (unsigned)cdiv(N, kTN);
        int splits = 1;
        if ((int64_t)gx * gy < 256 && K > 4096) splits = (int)std::min<int64_t>(512, cdiv(K, 256));
        if (splits == 1) {
            hipLaunchKernelGGL(k_gemm, dim3(gx, gy, 1), dim3(kBlk), 0, stream, M, N, K, A, sam, sak, B, sbk, sbn, C, Cb,
                               K, bias, relu, mask);
            OTF_LAUNCH_CHECK("k_gemm");
            return;
        }
        const int64_t chunk = ((cdiv(K, splits) + kTK - 1) / kTK) * kTK;
        splits = (int)cdiv(K, chunk);
        part.reserve((size_t)splits * M * N);
        hipLaunchKernelGGL(k_gemm, dim3(gx, gy, (unsigned)splits), dim3(kBlk), 0, stream, M, N, K, A, sam, sak, B, sbk,
                           sbn, part.p, (uint16_t *)nullptr, chunk, (const float *)nullptr, 0,
                           (const uint16_t *)nullptr);
        OTF_LAUNCH_CHECK("k_gemm split");
        hipLaunchKernelGGL(k_sum_splits, dim3(g1((int64_t)M * N * 64)), dim3(kBlk), 0, stream, part.p, splits,
                           (int64_t)M * N, C);
        OTF_LAUNCH_CHECK("k_sum_splits");
    }

    // forward of `rows` feature rows (device fp32, rows x 32) to Y (rows x 4)
    void forward(const float *Xf, int64_t rows, float *Yout) {
        X.reserve((size_t)rows * kIn);
        hipLaunchKernelGGL(k_to_bf16, dim3(g1(rows * kIn)), dim3(kBlk), 0, stream, Xf, rows * kIn, X.p);
        OTF_LAUNCH_CHECK("features to bf16");
        const uint16_t *h = X.p;
        for (int l = 0; l < kLayers; ++l) {
            const int in = kSizes[l], out = kSizes[l + 1];
            const bool last = l == kLayers - 1;
            if (!last) H[l].reserve((size_t)rows * out);
            gemm((int)rows, out, in, h, in, 1, wbf.p + off_w[l], out, 1, last ? Yout : nullptr,
                 last ? nullptr : H[l].p, theta.p + off_b[l], last ? 0 : 1, nullptr);
            if (!last) h = H[l].p;
        }
    }

    // the same outputs in one launch (k_mlp_forward), for inference
    void forward_fused(const float *Xf, int64_t rows, float *Yout) {
        const int64_t groups = cdiv(cdiv(rows, 16), kFusedWaves);
        if (groups == 0) return;
        hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)std::min<int64_t>(groups, 1024)), dim3(64 * kFusedWaves), 0,
                           stream, Xf, rows, (const uint16_t *)wbf.p, (const float *)theta.p, off_w[0], off_w[1],
                           off_w[2], off_w[3], off_b[0], off_b[1], off_b[2], off_b[3], Yout);
        OTF_LAUNCH_CHECK("k_mlp_forward");
    }

    // loss and gradient (grad) of the mean squared error against T (rows x 4)
    double backward(const float *Xf, const float *T, int64_t rows) {
        Y.reserve((size_t)rows * kOut);
        forward(Xf, rows, Y.p);
        grad.reserve((size_t)n_params);
        dZ.reserve((size_t)rows * kHid);
        dZ2.reserve((size_t)rows * kHid);
        dH.reserve((size_t)rows * kHid);
        const int64_t n = rows * kOut;
        const int64_t nb = (int64_t)g1(n);
        lpart.reserve((size_t)nb);
        hipLaunchKernelGGL(k_mse, dim3((unsigned)nb), dim3(kBlk), 0, stream, Y.p, T, n, 2.0f / (float)n, dZ.p, lpart.p);
        OTF_LAUNCH_CHECK("k_mse");
        uint16_t *dz = dZ.p, *dzn = dZ2.p;
        for (int l = kLayers - 1; l >= 0; --l) {
            const int in = kSizes[l], out = kSizes[l + 1];
            const uint16_t *hin = l == 0 ? X.p : H[l - 1].p;
            // dW = H_in^T dZ (in x out), reduced over the rows
            gemm(in, out, rows, hin, 1, in, dz, out, 1, grad.p + off_w[l], nullptr, nullptr, 0, nullptr);
            // db = column sums of dZ
            const int64_t chunk = (int64_t)kColRows * (kBlk / out), nbk = cdiv(rows, chunk);
            part.reserve((size_t)std::max<int64_t>(nbk * out, 1));
            hipLaunchKernelGGL(k_colsum, dim3((unsigned)nbk), dim3(kBlk), 0, stream, dz, rows, out, chunk, part.p);
            OTF_LAUNCH_CHECK("k_colsum");
            hipLaunchKernelGGL(k_sum_splits, dim3(g1((int64_t)out * 64)), dim3(kBlk), 0, stream, part.p, (int)nbk,
                               (int64_t)out,
                               grad.p + off_b[l]);
            OTF_LAUNCH_CHECK("bias gradient");
            if (l > 0) {
                // dZ_prev = mask(H_in) (dZ W^T), rows x in
                gemm((int)rows, in, out, dz, out, 1, wbf.p + off_w[l], 1, out, nullptr, dzn, nullptr, 0, hin);
                std::swap(dz, dzn);
            }
        }
        std::vector<double> h((size_t)nb);
        OTF_HIP(hipMemcpyAsync(h.data(), lpart.p, sizeof(double) * nb, hipMemcpyDeviceToHost, stream));
        OTF_HIP(hipStreamSynchronize(stream));
        double s = 0.0;
        for (double x : h) s += x;
        return s / (double)n;
    }
};

}  // namespace otf

struct otf_mlp {
    otf::Mlp m;
};

using namespace otf;

namespace {
template <class F>
otf_status mguard(otf_mlp *nn, F &&f) {
    if (hipSetDevice(nn->m.device) != hipSuccess) {
        (void)hipGetLastError();
        nn->m.err = "hipSetDevice failed";
        return OTF_E_DEVICE;
    }
    try {
        f();
        nn->m.err.clear();
        return OTF_OK;
    } catch (const Failure &e) {
        nn->m.err = e.msg;
        return e.st;
    } catch (...) {
        nn->m.err = "unexpected failure";
        return OTF_E_DEVICE;
    }
}
}  // namespace

extern "C" {

otf_status otf_mlp_create(int device, void *hip_stream, otf_mlp **out) {
    if (!out) return OTF_E_INVALID;
    *out = nullptr;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) {
        (void)hipGetLastError();
        return OTF_E_INVALID;
    }
    otf_mlp *nn = new (std::nothrow) otf_mlp();
    if (!nn) return OTF_E_NOMEM;
    nn->m.device = device;
    nn->m.stream = (hipStream_t)hip_stream;
    otf_status st = mguard(nn, [&] {
        Mlp &m = nn->m;
        m.theta.reserve(m.n_params);
        m.m.reserve(m.n_params);
        m.v.reserve(m.n_params);
        m.wbf.reserve(m.n_params);
        OTF_HIP(hipMemsetAsync(m.theta.p, 0, sizeof(float) * m.n_params, m.stream));
        OTF_HIP(hipMemsetAsync(m.m.p, 0, sizeof(float) * m.n_params, m.stream));
        OTF_HIP(hipMemsetAsync(m.v.p, 0, sizeof(float) * m.n_params, m.stream));
        m.sync_bf16();
        OTF_HIP(hipStreamSynchronize(m.stream));
    });
    if (st != OTF_OK) {
        delete nn;
        return st;
    }
    *out = nn;
    return OTF_OK;
}

otf_status otf_mlp_destroy(otf_mlp *nn) {
    if (!nn) return OTF_E_INVALID;
    (void)hipSetDevice(nn->m.device);
    (void)hipStreamSynchronize(nn->m.stream);
    delete nn;
    return OTF_OK;
}

int64_t otf_mlp_num_params(void) { return Mlp().n_params; }

otf_status otf_mlp_set_params(otf_mlp *nn, const float *params, int64_t n) {
    if (!nn || !params || n != nn->m.n_params) return OTF_E_INVALID;
    return mguard(nn, [&] {
        Mlp &m = nn->m;
        OTF_HIP(hipMemcpyAsync(m.theta.p, params, sizeof(float) * n, hipMemcpyHostToDevice, m.stream));
        OTF_HIP(hipMemsetAsync(m.m.p, 0, sizeof(float) * n, m.stream));
        OTF_HIP(hipMemsetAsync(m.v.p, 0, sizeof(float) * n, m.stream));
        m.step = 0;
        m.sync_bf16();
        OTF_HIP(hipStreamSynchronize(m.stream));
    });
}

otf_status otf_mlp_get_params(otf_mlp *nn, float *params, int64_t n) {
    if (!nn || !params || n != nn->m.n_params) return OTF_E_INVALID;
    return mguard(nn, [&] {
        Mlp &m = nn->m;
        OTF_HIP(hipMemcpyAsync(params, m.theta.p, sizeof(float) * n, hipMemcpyDeviceToHost, m.stream));
        OTF_HIP(hipStreamSynchronize(m.stream));
    });
}

otf_status otf_mlp_forward(otf_mlp *nn, const float *X, int64_t rows, float *Y) {
    if (!nn || !X || !Y || rows < 1) return OTF_E_INVALID;
    return mguard(nn, [&] {
        nn->m.forward(X, rows, Y);
        OTF_HIP(hipStreamSynchronize(nn->m.stream));
    });
}

otf_status otf_mlp_gradient(otf_mlp *nn, const float *X, const float *T, int64_t rows, float *grad, double *loss) {
    if (!nn || !X || !T || rows < 1) return OTF_E_INVALID;
    return mguard(nn, [&] {
        Mlp &m = nn->m;
        const double l = m.backward(X, T, rows);
        if (loss) *loss = l;
        if (grad) {
            OTF_HIP(hipMemcpyAsync(grad, m.grad.p, sizeof(float) * m.n_params, hipMemcpyDeviceToHost, m.stream));
            OTF_HIP(hipStreamSynchronize(m.stream));
        }
    });
}

otf_status otf_mlp_train_step(otf_mlp *nn, const float *X, const float *T, int64_t rows, float lr, double *loss) {
    if (!nn || !X || !T || rows < 1 || !std::isfinite(lr) || !(lr > 0.0f)) return OTF_E_INVALID;
    return mguard(nn, [&] {
        Mlp &m = nn->m;
        const double l = m.backward(X, T, rows);
        if (loss) *loss = l;
        m.step += 1;
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.0f - std::pow(b1, (float)m.step), c2 = 1.0f - std::pow(b2, (float)m.step);
        hipLaunchKernelGGL(k_adam, dim3(g1(m.n_params)), dim3(kBlk), 0, m.stream, m.theta.p, m.m.p, m.v.p, m.grad.p,
                           m.n_params, lr, b1, b2, c1, c2, 1e-8f);
        OTF_LAUNCH_CHECK("k_adam");
        m.sync_bf16();
    });
}

const char *otf_mlp_last_error(const otf_mlp *nn) { return nn ? nn->m.err.c_str() : "null network"; }

otf_status otf_features(otf_ctx *ctx, float *X, int64_t cap_rows) {
    if (!ctx || !X) return OTF_E_INVALID;
    if (!ctx->c.valid) return OTF_E_STATE;
    if (cap_rows < ctx->c.L) return OTF_E_CAPACITY;
    Ctx &c = ctx->c;
    try {
        OTF_HIP(hipSetDevice(c.device));
        LeafStore &s = c.lv();
        hipLaunchKernelGGL(k_features, dim3(g1(c.L)), dim3(kBlk), 0, c.stream, c.L, c.prm.max_depth, c.prm.gamma,
                           s.level.p, s.u.p, s.obs_off.p, s.obs_m.p, s.wtot.p, c.op().F.p, s.nbp_off.p, s.nbp.p,
                           s.nbm_off.p, s.nbm.p, X);
        OTF_LAUNCH_CHECK("k_features");
        OTF_HIP(hipStreamSynchronize(c.stream));
    } catch (const Failure &e) {
        c.err = e.msg;
        return e.st;
    }
    return OTF_OK;
}

otf_status otf_leaf_targets(otf_ctx *ctx, float *T, int64_t cap_rows) {
    if (!ctx || !T) return OTF_E_INVALID;
    if (!ctx->c.valid) return OTF_E_STATE;
    if (cap_rows < ctx->c.L) return OTF_E_CAPACITY;
    Ctx &c = ctx->c;
    try {
        OTF_HIP(hipSetDevice(c.device));
        LeafStore &s = c.lv();
        hipLaunchKernelGGL(k_targets, dim3(g1(c.L)), dim3(kBlk), 0, c.stream, c.L, s.cap, s.u.p, s.p.p, T);
        OTF_LAUNCH_CHECK("k_targets");
        OTF_HIP(hipStreamSynchronize(c.stream));
    } catch (const Failure &e) {
        c.err = e.msg;
        return e.st;
    }
    return OTF_OK;
}

otf_status otf_warm_start_guarded(otf_ctx *ctx, otf_mlp *nn, float lambda, int32_t n_alpha, const float *alphas,
                                 float *alpha_used, double *energy_used) {
    if (!ctx || !nn || !alphas || !alpha_used || !energy_used) return OTF_E_INVALID;
    if (n_alpha < 1 || n_alpha > 8 || !std::isfinite(lambda) || lambda < 0.0f) return OTF_E_INVALID;
    for (int k = 0; k < n_alpha; ++k)
        if (!(alphas[k] > 0.0f && alphas[k] <= 1.0f)) return OTF_E_INVALID;
    if (!ctx->c.valid) return OTF_E_STATE;
    if (ctx->c.device != nn->m.device || ctx->c.stream != nn->m.stream) return OTF_E_INVALID;
    Ctx &c = ctx->c;
    try {
        OTF_HIP(hipSetDevice(c.device));
        LeafStore &s = c.lv();
        const int64_t L = c.L;
        auto E = [&] {
            double tv = 0.0, data = 0.0;
            energy(c, &tv, &data);
            return tv + (double)lambda * data;
        };
        // the plain start, kept for the candidates and as the fallback (the
        // context's grow-only scratch: no allocation once it is large enough)
        DBuf<float> &X = c.s.fa, &Y = c.s.fb, &u0 = c.s.fc, &ub0 = c.s.fd, &p0 = c.s.fe;
        X.reserve((size_t)L * kIn);
        Y.reserve((size_t)L * kOut);
        u0.reserve((size_t)L);
        ub0.reserve((size_t)L);
        p0.reserve((size_t)3 * s.cap);
        OTF_HIP(hipMemcpyAsync(u0.p, s.u.p, (size_t)L * sizeof(float), hipMemcpyDeviceToDevice, c.stream));
        OTF_HIP(hipMemcpyAsync(ub0.p, s.ubar.p, (size_t)L * sizeof(float), hipMemcpyDeviceToDevice, c.stream));
        OTF_HIP(hipMemcpyAsync(p0.p, s.p.p, (size_t)3 * s.cap * sizeof(float), hipMemcpyDeviceToDevice, c.stream));
        const double e_plain = E();
        hipLaunchKernelGGL(k_features, dim3(g1(L)), dim3(kBlk), 0, c.stream, L, c.prm.max_depth, c.prm.gamma,
                           s.level.p, s.u.p, s.obs_off.p, s.obs_m.p, s.wtot.p, c.op().F.p, s.nbp_off.p, s.nbp.p,
                           s.nbm_off.p, s.nbm.p, X.p);
        OTF_LAUNCH_CHECK("k_features");
        nn->m.forward_fused(X.p, L, Y.p);
        float best_a = 0.0f;
        double best_e = e_plain;
        for (int k = 0; k < n_alpha; ++k) {
            hipLaunchKernelGGL(k_apply_warm_alpha, dim3(g1(L)), dim3(kBlk), 0, c.stream, L, s.cap, Y.p, u0.p, p0.p,
                               alphas[k], s.u.p, s.ubar.p, s.p.p);
            OTF_LAUNCH_CHECK("k_apply_warm_alpha");
            const double e = E();
            if (e < best_e) {
                best_e = e;
                best_a = alphas[k];
            }
        }
        if (best_a == 0.0f) {  // the plain start
            OTF_HIP(hipMemcpyAsync(s.u.p, u0.p, (size_t)L * sizeof(float), hipMemcpyDeviceToDevice, c.stream));
            OTF_HIP(hipMemcpyAsync(s.ubar.p, ub0.p, (size_t)L * sizeof(float), hipMemcpyDeviceToDevice, c.stream));
            OTF_HIP(hipMemcpyAsync(s.p.p, p0.p, (size_t)3 * s.cap * sizeof(float), hipMemcpyDeviceToDevice,
                                   c.stream));
        } else if (best_a != alphas[n_alpha - 1]) {
            hipLaunchKernelGGL(k_apply_warm_alpha, dim3(g1(L)), dim3(kBlk), 0, c.stream, L, s.cap, Y.p, u0.p, p0.p,
                               best_a, s.u.p, s.ubar.p, s.p.p);
            OTF_LAUNCH_CHECK("k_apply_warm_alpha");
        }
        OTF_HIP(hipStreamSynchronize(c.stream));
        *alpha_used = best_a;
        *energy_used = best_e;
    } catch (const Failure &e) {
        c.err = e.msg;
        return e.st;
    }
    return OTF_OK;
}

otf_status otf_warm_start(otf_ctx *ctx, otf_mlp *nn) {
    if (!ctx || !nn) return OTF_E_INVALID;
    if (!ctx->c.valid) return OTF_E_STATE;
    if (ctx->c.device != nn->m.device || ctx->c.stream != nn->m.stream) return OTF_E_INVALID;
    Ctx &c = ctx->c;
    try {
        OTF_HIP(hipSetDevice(c.device));
        DBuf<float> &X = c.s.fa, &Y = c.s.fb;  // the context's grow-only scratch
        X.reserve((size_t)c.L * kIn);
        Y.reserve((size_t)c.L * kOut);
        LeafStore &s = c.lv();
        hipLaunchKernelGGL(k_features, dim3(g1(c.L)), dim3(kBlk), 0, c.stream, c.L, c.prm.max_depth, c.prm.gamma,
                           s.level.p, s.u.p, s.obs_off.p, s.obs_m.p, s.wtot.p, c.op().F.p, s.nbp_off.p, s.nbp.p,
                           s.nbm_off.p, s.nbm.p, X.p);
        OTF_LAUNCH_CHECK("k_features");
        nn->m.forward_fused(X.p, c.L, Y.p);
        hipLaunchKernelGGL(k_apply_warm, dim3(g1(c.L)), dim3(kBlk), 0, c.stream, c.L, s.cap, Y.p, s.u.p, s.ubar.p,
                           s.p.p);
        OTF_LAUNCH_CHECK("k_apply_warm");
        OTF_HIP(hipStreamSynchronize(c.stream));
    } catch (const Failure &e) {
        c.err = e.msg;
        return e.st;
    }
    return OTF_OK;
}

}  // extern "C"
