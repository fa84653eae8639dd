// k_mlp.hip -- the per-object step network: features, BF16 inference, FP32
// training (forward, backward, Adam) and the per-object record counts that the
// training targets are built from.
//
// The paper keeps a time interval per object so that objects far from all
// others take long intervals (Sec. Collision Detection with 4D AABB Trees;
// Procedure advanceTime) but leaves the choice of step open.  This network
// predicts log2(step in seconds) from five orbital features:
//   x = (a / 42164, e, i / pi, r_p / 42164, vmax / 8),  r_p = a (1 - e),
//   h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2), y = w3 . h2 + b3,
//   step = clamp(floor(2^y / tick), 1, max(T, 1)) ticks.
// Any step keeps the boxes conservative, so the network changes cost only.
//
// Inference runs one object per lane: BF16 weights staged in LDS (read as
// wave-uniform broadcasts), BF16 inputs and hidden activations packed two to a
// register, FP32 accumulation through v_dot2c_f32_bf16.  Training keeps FP32
// master weights: one kernel runs the forward and backward pass per sample and
// writes the activations and their gradients feature-major; a second forms the
// per-parameter outer-product sums over a block of samples in LDS; a third adds
// the block partials in a fixed order, so gradients are deterministic.
#include "cd_internal.h"

namespace cd {

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// FP32 -> bfloat16 bits, round to nearest, ties to even.
__device__ inline uint32_t bf16_bits(float f)
{
    uint32_t u = __float_as_uint(f);
    if (f != f)
        return (u >> 16) | 0x40u;
    return (u + 0x7FFFu + ((u >> 16) & 1u)) >> 16;
}

__device__ inline float bf16_value(uint32_t h) { return __uint_as_float(h << 16); }

__device__ inline float dot2_bf16(uint32_t a, uint32_t b, float c)
{
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2, a),
                                           __builtin_bit_cast(bf16x2, b), c, false);
}

__device__ inline void mlp_features(double a, double e, double inc, double mu, double x[5],
                                    double &vmax)
{
    double rp = a * (1.0 - e);
    vmax = sqrt(mu * (1.0 + e) / rp);
    x[0] = a / 42164.0;
    x[1] = e;
    x[2] = inc / 3.141592653589793;
    x[3] = rp / 42164.0;
    x[4] = vmax / 8.0;
}

__global__ void k_mlp_features(cd_elements el, double mu, float *xo)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= el.n)
        return;
    double x[5], vmax;
    mlp_features(el.a[i], el.e[i], el.inc[i], mu, x, vmax);
    for (int f = 0; f < kMlpIn; ++f)
        xo[i * kMlpIn + f] = (float)x[f];
}

// ---- BF16 inference -----------------------------------------------------------------

__global__ __launch_bounds__(256) void k_dt_mlp(cd_elements el, const uint16_t *__restrict__ w,
                                                double mu, double tick_s, double fallback,
                                                uint32_t T, uint32_t *dt, float *yout)
{
    __shared__ uint4 sW2[kMlpHid][8];     // row r: bf16 pairs (2k, 2k+1), k < 32
    __shared__ uint32_t sW1[kMlpHid][3];  // row r: pairs (x0 x1), (x2 x3), (x4 0)
    __shared__ float sB1[kMlpHid], sB2[kMlpHid], sW3[kMlpHid];
    __shared__ float sB3;
    uint32_t *w2 = (uint32_t *)&sW2[0][0];
    for (int t = threadIdx.x; t < kMlpHid * 32; t += blockDim.x) {
        int r = t >> 5, k = t & 31;
        const uint16_t *row = w + kMlpW2 + r * kMlpHid;
        w2[t] = (uint32_t)row[2 * k] | ((uint32_t)row[2 * k + 1] << 16);
    }
    for (int t = threadIdx.x; t < kMlpHid * 3; t += blockDim.x) {
        int r = t / 3, q = t % 3;
        const uint16_t *row = w + kMlpW1 + r * kMlpIn;
        uint32_t lo = row[2 * q];
        uint32_t hi = (2 * q + 1 < kMlpIn) ? (uint32_t)row[2 * q + 1] : 0u;
        sW1[r][q] = lo | (hi << 16);
    }
    for (int t = threadIdx.x; t < kMlpHid; t += blockDim.x) {
        sB1[t] = bf16_value(w[kMlpB1 + t]);
        sB2[t] = bf16_value(w[kMlpB2 + t]);
        sW3[t] = bf16_value(w[kMlpW3 + t]);
    }
    if (threadIdx.x == 0)
        sB3 = bf16_value(w[kMlpB3]);
    __syncthreads();

    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= el.n)
        return;
    double xd[5], vmax;
    mlp_features(el.a[i], el.e[i], el.inc[i], mu, xd, vmax);
    uint32_t xb[5];
    for (int f = 0; f < 5; ++f)
        xb[f] = bf16_bits((float)xd[f]);
    uint32_t x01 = xb[0] | (xb[1] << 16), x23 = xb[2] | (xb[3] << 16), x4 = xb[4];

    uint32_t h1[32];
#pragma unroll
    for (int k = 0; k < 32; ++k) {
        uint32_t hb[2];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            int r = 2 * k + q;
            float acc = sB1[r];
            acc = dot2_bf16(sW1[r][0], x01, acc);
            acc = dot2_bf16(sW1[r][1], x23, acc);
            acc = dot2_bf16(sW1[r][2], x4, acc);
            hb[q] = bf16_bits(fmaxf(acc, 0.0f));
        }
        h1[k] = hb[0] | (hb[1] << 16);
    }
    float y = 0.0f;
    for (int r = 0; r < kMlpHid; ++r) {
        float acc = sB2[r];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            uint4 wv = sW2[r][q];
            acc = dot2_bf16(wv.x, h1[4 * q + 0], acc);
            acc = dot2_bf16(wv.y, h1[4 * q + 1], acc);
            acc = dot2_bf16(wv.z, h1[4 * q + 2], acc);
            acc = dot2_bf16(wv.w, h1[4 * q + 3], acc);
        }
        float h2 = bf16_value(bf16_bits(fmaxf(acc, 0.0f)));
        y = fmaf(sW3[r], h2, y);
    }
    y += sB3;
    if (yout)
        yout[i] = y;
    uint32_t d;
    if (isfinite(y)) {
        double v = floor(exp2((double)y) / tick_s);
        double cap = T > 0 ? (double)T : 1.0;
        v = v < 1.0 ? 1.0 : (v > cap ? cap : v);
        d = (uint32_t)v;
    } else {
        d = heuristic_step(vmax, tick_s, fallback, T);
    }
    dt[i] = d;
}

// ---- FP32 training ----------------------------------------------------------------------

struct MlpF32 {
    float W1[kMlpHid][kMlpIn];
    float b1[kMlpHid];
    float4 W2[kMlpHid][kMlpHid / 4];
    float b2[kMlpHid];
    float w3[kMlpHid];
    float b3;
};

__device__ inline void load_mlp_f32(MlpF32 &s, const float *__restrict__ w)
{
    float *W1 = &s.W1[0][0];
    float *W2 = (float *)&s.W2[0][0];
    for (int t = threadIdx.x; t < kMlpHid * kMlpHid; t += blockDim.x)
        W2[t] = w[kMlpW2 + t];
    for (int t = threadIdx.x; t < kMlpHid * kMlpIn; t += blockDim.x)
        W1[t] = w[kMlpW1 + t];
    for (int t = threadIdx.x; t < kMlpHid; t += blockDim.x) {
        s.b1[t] = w[kMlpB1 + t];
        s.b2[t] = w[kMlpB2 + t];
        s.w3[t] = w[kMlpW3 + t];
    }
    if (threadIdx.x == 0)
        s.b3 = w[kMlpB3];
    __syncthreads();
}

__device__ inline void mlp_layer1(const MlpF32 &s, const float x[5], float h1[kMlpHid])
{
#pragma unroll
    for (int r = 0; r < kMlpHid; ++r) {
        float acc = s.b1[r];
#pragma unroll
        for (int c = 0; c < kMlpIn; ++c)
            acc = fmaf(s.W1[r][c], x[c], acc);
        h1[r] = fmaxf(acc, 0.0f);
    }
}

__device__ inline float mlp_row2(const MlpF32 &s, int r, const float h1[kMlpHid])
{
    float acc = s.b2[r];
#pragma unroll
    for (int q = 0; q < kMlpHid / 4; ++q) {
        float4 wv = s.W2[r][q];
        acc = fmaf(wv.x, h1[4 * q + 0], acc);
        acc = fmaf(wv.y, h1[4 * q + 1], acc);
        acc = fmaf(wv.z, h1[4 * q + 2], acc);
        acc = fmaf(wv.w, h1[4 * q + 3], acc);
    }
    return acc;
}

__global__ __launch_bounds__(256) void k_mlp_forward(const float *__restrict__ w,
                                                     const float *__restrict__ x, uint32_t B,
                                                     float *__restrict__ y)
{
    __shared__ MlpF32 s;
    load_mlp_f32(s, w);
    uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B)
        return;
    float xv[kMlpIn], h1[kMlpHid];
    for (int c = 0; c < kMlpIn; ++c)
        xv[c] = x[(uint64_t)b * kMlpIn + c];
    mlp_layer1(s, xv, h1);
    float out = s.b3;
#pragma unroll 1
    for (int r = 0; r < kMlpHid; ++r)
        out = fmaf(s.w3[r], fmaxf(mlp_row2(s, r, h1), 0.0f), out);
    y[b] = out;
}

// Rows of the activation array (each B long).
constexpr int kActH1 = 0, kActDZ1 = 64, kActH2 = 128, kActDZ2 = 192, kActDY = 256,
              kActSQ = 257, kActRows = 258;

// Per sample: forward, loss term (y - t)^2 / B and the backward pass to the
// pre-activation gradients dz1, dz2 and dy.
__global__ __launch_bounds__(256) void k_mlp_backprop(const float *__restrict__ w,
                                                      const float *__restrict__ x,
                                                      const float *__restrict__ target,
                                                      uint32_t B, float *__restrict__ act)
{
    __shared__ MlpF32 s;
    load_mlp_f32(s, w);
    uint32_t b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= B)
        return;
    float xv[kMlpIn], h1[kMlpHid];
    for (int c = 0; c < kMlpIn; ++c)
        xv[c] = x[(uint64_t)b * kMlpIn + c];
    mlp_layer1(s, xv, h1);
    float y = s.b3;
#pragma unroll 1
    for (int r = 0; r < kMlpHid; ++r)
        y = fmaf(s.w3[r], fmaxf(mlp_row2(s, r, h1), 0.0f), y);
    float res = y - target[b];
    float dy = 2.0f * res / (float)B;
    act[(uint64_t)kActDY * B + b] = dy;
    act[(uint64_t)kActSQ * B + b] = res * res / (float)B;
    // second pass: recompute each h2 row (cheaper than holding 64 more
    // registers), then accumulate dh1 = W2^T dz2
    float dh1[kMlpHid];
#pragma unroll
    for (int k = 0; k < kMlpHid; ++k)
        dh1[k] = 0.0f;
#pragma unroll 1
    for (int r = 0; r < kMlpHid; ++r) {
        float h2 = fmaxf(mlp_row2(s, r, h1), 0.0f);
        float dz2 = h2 > 0.0f ? dy * s.w3[r] : 0.0f;
        act[(uint64_t)(kActH2 + r) * B + b] = h2;
        act[(uint64_t)(kActDZ2 + r) * B + b] = dz2;
#pragma unroll
        for (int q = 0; q < kMlpHid / 4; ++q) {
            float4 wv = s.W2[r][q];
            dh1[4 * q + 0] = fmaf(dz2, wv.x, dh1[4 * q + 0]);
            dh1[4 * q + 1] = fmaf(dz2, wv.y, dh1[4 * q + 1]);
            dh1[4 * q + 2] = fmaf(dz2, wv.z, dh1[4 * q + 2]);
            dh1[4 * q + 3] = fmaf(dz2, wv.w, dh1[4 * q + 3]);
        }
    }
#pragma unroll
    for (int k = 0; k < kMlpHid; ++k) {
        act[(uint64_t)(kActH1 + k) * B + b] = h1[k];
        act[(uint64_t)(kActDZ1 + k) * B + b] = h1[k] > 0.0f ? dh1[k] : 0.0f;
    }
}

// Block partial of every gradient entry (and of the loss, entry kMlpParams):
// sum over the block's samples of u[s] * v[s] for the entry's two rows.
constexpr int kOuterStage = 32;
constexpr int kOuterStride = kOuterStage + 1;   // row stride in LDS: no bank conflicts
// LDS rows: act rows 0..257, then x (5 rows), then a row of ones
constexpr int kOuterRowX = kActRows, kOuterRowOne = kActRows + kMlpIn,
              kOuterRows = kActRows + kMlpIn + 1;
constexpr int kOuterSlots = (kMlpParams + 1 + kMlpOuterThreads - 1) / kMlpOuterThreads;

__device__ inline void outer_rows(int p, int &u, int &v)
{
    if (p < kMlpB1) {   // W1[r][c] = sum dz1[r] x[c]
        u = kActDZ1 + p / kMlpIn;
        v = kOuterRowX + p % kMlpIn;
    } else if (p < kMlpW2) {
        u = kActDZ1 + (p - kMlpB1);
        v = kOuterRowOne;
    } else if (p < kMlpB2) {   // W2[r][c] = sum dz2[r] h1[c]
        int q = p - kMlpW2;
        u = kActDZ2 + q / kMlpHid;
        v = kActH1 + q % kMlpHid;
    } else if (p < kMlpW3) {
        u = kActDZ2 + (p - kMlpB2);
        v = kOuterRowOne;
    } else if (p < kMlpB3) {   // w3[c] = sum dy h2[c]
        u = kActDY;
        v = kActH2 + (p - kMlpW3);
    } else if (p == kMlpB3) {
        u = kActDY;
        v = kOuterRowOne;
    } else {   // loss
        u = kActSQ;
        v = kOuterRowOne;
    }
}

__global__ __launch_bounds__(kMlpOuterThreads) void k_mlp_outer(const float *__restrict__ act,
                                                                const float *__restrict__ x,
                                                                uint32_t B,
                                                                float *__restrict__ part)
{
    __shared__ float st[kOuterRows * kOuterStride];
    int uo[kOuterSlots], vo[kOuterSlots];
    float acc[kOuterSlots];
#pragma unroll
    for (int j = 0; j < kOuterSlots; ++j) {
        int p = threadIdx.x + j * kMlpOuterThreads;
        int u = kOuterRowOne, v = kOuterRowOne;
        if (p <= kMlpParams)
            outer_rows(p, u, v);
        uo[j] = u * kOuterStride;
        vo[j] = v * kOuterStride;
        acc[j] = 0.0f;
    }
    uint64_t b0 = (uint64_t)blockIdx.x * kMlpOuterSamples;
    uint64_t b1 = b0 + kMlpOuterSamples < B ? b0 + kMlpOuterSamples : B;
    for (uint64_t s0 = b0; s0 < b1; s0 += kOuterStage) {
        __syncthreads();
        for (int t = threadIdx.x; t < kOuterRows * kOuterStage; t += kMlpOuterThreads) {
            int row = t / kOuterStage, c = t % kOuterStage;
            uint64_t b = s0 + c;
            float val = 0.0f;
            if (b < b1) {
                if (row < kActRows)
                    val = act[(uint64_t)row * B + b];
                else if (row < kOuterRowOne)
                    val = x[b * kMlpIn + (row - kOuterRowX)];
                else
                    val = 1.0f;
            }
            st[row * kOuterStride + c] = val;
        }
        __syncthreads();
#pragma unroll
        for (int j = 0; j < kOuterSlots; ++j) {
            const float *u = st + uo[j];
            const float *v = st + vo[j];
            float a = acc[j];
#pragma unroll 8
            for (int c = 0; c < kOuterStage; ++c)
                a = fmaf(u[c], v[c], a);
            acc[j] = a;
        }
    }
#pragma unroll
    for (int j = 0; j < kOuterSlots; ++j) {
        int p = threadIdx.x + j * kMlpOuterThreads;
        if (p <= kMlpParams)
            part[(uint64_t)blockIdx.x * (kMlpParams + 1) + p] = acc[j];
    }
}

// Gradient entry p = sum of the block partials in block order.
__global__ void k_mlp_reduce(const float *__restrict__ part, uint32_t nblk,
                             float *__restrict__ grad, float *__restrict__ loss)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > kMlpParams)
        return;
    float sum = 0.0f;
    for (uint32_t k = 0; k < nblk; ++k)
        sum += part[(uint64_t)k * (kMlpParams + 1) + p];
    if (p < kMlpParams)
        grad[p] = sum;
    else if (loss)
        *loss = sum;
}

// Adam (Kingma & Ba) with bias-corrected moments; optional BF16 export.
__global__ void k_mlp_adam(float *w, float *m, float *v, const float *g, int64_t step, float lr,
                           float beta1, float beta2, float eps, uint16_t *wb)
{
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= kMlpParams)
        return;
    float gp = g[p];
    float mp = beta1 * m[p] + (1.0f - beta1) * gp;
    float vp = beta2 * v[p] + (1.0f - beta2) * gp * gp;
    m[p] = mp;
    v[p] = vp;
    float bc1 = (float)(1.0 - pow((double)beta1, (double)step));
    float bc2 = (float)(1.0 - pow((double)beta2, (double)step));
    float wp = w[p] - lr * (mp / bc1) / (sqrtf(vp / bc2) + eps);
    w[p] = wp;
    if (wb)
        wb[p] = (uint16_t)bf16_bits(wp);
}

// Records per object: each record counts once for i and once for j.
__global__ void k_pair_object_counts(const cd_pair *pairs, uint64_t count, uint32_t n,
                                     uint32_t *counts)
{
    uint64_t r = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= count)
        return;
    cd_pair p = pairs[r];
    if (p.i < n)
        atomicAdd(&counts[p.i], 1u);
    if (p.j < n)
        atomicAdd(&counts[p.j], 1u);
}

static inline unsigned blocks_for(uint64_t n, unsigned t) { return (unsigned)((n + t - 1) / t); }

hipError_t launch_mlp_features(const cd_elements &el, double mu, float *x, hipStream_t s)
{
    if (el.n == 0)
        return hipSuccess;
    k_mlp_features<<<blocks_for(el.n, 256), 256, 0, s>>>(el, mu, x);
    return hipGetLastError();
}

hipError_t launch_dt_mlp(const cd_elements &el, const uint16_t *w, double mu, double tick_s,
                         double fallback_disp, uint32_t T, uint32_t *dt, float *y,
                         hipStream_t s)
{
    if (el.n == 0)
        return hipSuccess;
    k_dt_mlp<<<blocks_for(el.n, 256), 256, 0, s>>>(el, w, mu, tick_s, fallback_disp, T, dt, y);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const float *w, const float *x, uint32_t B, float *y,
                              hipStream_t s)
{
    if (B == 0)
        return hipSuccess;
    k_mlp_forward<<<blocks_for(B, 256), 256, 0, s>>>(w, x, B, y);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const float *w, const float *x, const float *target, uint32_t B,
                           float *act, float *part, float *grad, float *loss, hipStream_t s)
{
    unsigned nblk = blocks_for(B, kMlpOuterSamples);
    k_mlp_backprop<<<blocks_for(B, 256), 256, 0, s>>>(w, x, target, B, act);
    k_mlp_outer<<<nblk, kMlpOuterThreads, 0, s>>>(act, x, B, part);
    k_mlp_reduce<<<blocks_for(kMlpParams + 1, 256), 256, 0, s>>>(part, nblk, grad, loss);
    return hipGetLastError();
}

hipError_t launch_mlp_adam(float *w, float *m, float *v, const float *g, int64_t step,
                           float lr, float beta1, float beta2, float eps, uint16_t *w_bf16,
                           hipStream_t s)
{
    k_mlp_adam<<<blocks_for(kMlpParams, 256), 256, 0, s>>>(w, m, v, g, step, lr, beta1, beta2,
                                                           eps, w_bf16);
    return hipGetLastError();
}

hipError_t launch_pair_object_counts(const cd_pair *pairs, uint64_t count, uint32_t n,
                                     uint32_t *counts, hipStream_t s)
{
    hipError_t e = launch_fill_u32(counts, 0u, n, s);
    if (e != hipSuccess || count == 0)
        return e;
    k_pair_object_counts<<<blocks_for(count, 256), 256, 0, s>>>(pairs, count, n, counts);
    return hipGetLastError();
}

} // namespace cd
