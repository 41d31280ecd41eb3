/*
 * Training, evaluation and target-generation kernels of the kernel surrogate
 * (4 -> 64 -> 64 -> 1 SiLU perceptron; see fspb_mlp.h).
 *
 *   k_mlp_targets  analytic K(d, u, v, a) = PDD(d) F(u, v; a, a, d) and the
 *                  features of each sample (one thread per sample)
 *   k_mlp_forward  surrogate outputs, 64 samples per wave
 *   k_mlp_grad     forward + backward of 64 samples per wave; BF16 matrix
 *                  cores for h1 W2^T, dz2^T h1 and dz2 W2; per-wave gradient
 *                  partials (deterministic, no atomics)
 *   k_mlp_reduce   sum of the partials, then Adam on the FP32 masters and
 *                  fresh BF16 copies of W2 (or the plain gradient)
 */
#include <hip/hip_runtime.h>
#include <math.h>
#include <stdint.h>

#include "fspb_mlp_device.h"

namespace fspb {

namespace {

using namespace mlp;

/* erfc(x / kScale), x = z * kScale >= 0, from a global piecewise-quadratic table. */
__device__ inline float erfc_tab(const float4 *__restrict__ tab, float x)
{
    const float xc = fminf(x, 511.999f);
    const int k = (int)xc;
    const float f = __builtin_amdgcn_fractf(xc);
    const float4 c = tab[k];
    return fmaf(fmaf(c.z, f, c.y), f, c.x);
}

__device__ inline float bracket(const float4 *__restrict__ tab, float ax, float h, float isk)
{
    const float hk = h * isk;
    const float ea = erfc_tab(tab, fabsf(fmaf(-ax, isk, hk)));
    const float eb = erfc_tab(tab, fmaf(ax, isk, hk));
    return (ax <= h ? 2.0f - ea : ea) - eb;
}

__global__ __launch_bounds__(256) void k_mlp_targets(MlpTargetDev K, const float *__restrict__ samples, int64_t n,
                                                     float *__restrict__ feats, float *__restrict__ targets)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float d = samples[4 * i], au = fabsf(samples[4 * i + 1]), av = fabsf(samples[4 * i + 2]);
    const float a = samples[4 * i + 3];
    float x[4];
    features(d, au, av, a, x);
#pragma unroll
    for (int k = 0; k < 4; ++k) feats[4 * i + k] = x[k];
    const float xp = fminf(fmaxf(d * K.pdd_inv_step, 0.0f), K.pdd_max);
    const int kp = min((int)xp, K.n_pdd - 2);
    const float fp = xp - (float)kp;
    const float pdd = fmaf(fp, K.pdd[kp + 1] - K.pdd[kp], K.pdd[kp]);
    constexpr float kIs = 0.70710678118654752f * 128.0f;
    float L = 0.0f;
    for (int t = 0; t < K.n_terms; ++t) {
        const float isk = kIs / fmaf(K.sig1[t], d, K.sig0[t]);
        const float h = 0.5f * K.c2[t] * a;
        L = fmaf(K.w4[t] * bracket(K.erfc_tab, au, h, isk), bracket(K.erfc_tab, av, h, isk), L);
    }
    targets[i] = pdd * L;
}

__global__ __launch_bounds__(256) void k_mlp_forward(MlpDev m, const float *__restrict__ feats, int64_t n,
                                                     float *__restrict__ out)
{
    __shared__ __align__(16) uint16_t h1[4][64 * kH1Stride];
    const int w = threadIdx.x >> 6, l = lane();
    const int64_t i = ((int64_t)blockIdx.x * 4 + w) * 64 + l;
    W2Frags wf;
    load_w2_frags(m.w2, wf);
    float x[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (i < n)
        for (int k = 0; k < 4; ++k) x[k] = feats[4 * i + k];
    const float y = forward_wave<false>(m.p, nullptr, wf, x, h1[w]);
    if (i < n) out[i] = y;
}

__global__ __launch_bounds__(64) void k_mlp_grad(MlpDev m, const float *__restrict__ feats,
                                                 const float *__restrict__ targets, int64_t n_total, int64_t base,
                                                 int64_t n_step, uint64_t stride, uint64_t offset, float inv_count,
                                                 float *__restrict__ partials)
{
    __shared__ float Xs[64][4];
    __shared__ float Z1s[64][65];
    __shared__ __align__(16) uint16_t H1[64 * kH1Stride];     // [sample][in]
    __shared__ __align__(16) uint16_t H1T[64 * kTStride];     // [in][sample]
    __shared__ __align__(16) uint16_t DZ2[64 * kH1Stride];    // [sample][out]
    __shared__ __align__(16) uint16_t DZ2T[64 * kTStride];    // [out][sample]
    const int l = lane(), n = l & 15, g = l >> 4;
    const int64_t mine = (int64_t)blockIdx.x * 64 + l;
    const bool valid = mine < n_step;
    const int64_t idx = valid ? (int64_t)((offset + (uint64_t)(base + mine) * stride) % (uint64_t)n_total) : 0;
    float x[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    float t = 0.0f;
    if (valid) {
        for (int k = 0; k < 4; ++k) x[k] = feats[4 * idx + k];
        t = targets[idx];
    }
    const float *p = m.p;
    for (int k = 0; k < 4; ++k) Xs[l][k] = x[k];
    // ---- layer 1
    for (int o = 0; o < kMlpH; ++o) {
        float z = p[kOffB1 + o];
#pragma unroll
        for (int k = 0; k < kMlpIn; ++k) z = fmaf(p[kOffW1 + o * kMlpIn + k], x[k], z);
        Z1s[l][o] = z;
        const uint16_t h = bf16_bits(z * sigmoid(z));
        H1[l * kH1Stride + o] = h;
        H1T[o * kTStride + l] = h;
    }
    __syncthreads();
    // ---- layer 2 (matrix cores), layer 3, loss and the backward of layers 3 and 2's activation
    W2Frags wf;
    load_w2_frags(m.w2, wf);
    float gb2[4] = {0, 0, 0, 0}, gw3[4] = {0, 0, 0, 0}, gb3 = 0.0f, loss = 0.0f;
    for (int rt = 0; rt < 4; ++rt) {
        f32x4 acc[4];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[ct] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const bf16x8 a = frag(H1 + (16 * rt + n) * kH1Stride + 32 * ks + 8 * g);
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) acc[ct] = mfma(a, wf.b[ct][ks], acc[ct]);
        }
        float z2[4][4], sg[4][4], part[4] = {0, 0, 0, 0};
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const float b2 = p[kOffB2 + 16 * ct + n], w3 = p[kOffW3 + 16 * ct + n];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                z2[ct][i] = acc[ct][i] + b2;
                sg[ct][i] = sigmoid(z2[ct][i]);
                part[i] = fmaf(z2[ct][i] * sg[ct][i], w3, part[i]);
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int mm = 1; mm < 16; mm <<= 1) part[i] += __shfl_xor(part[i], mm, 64);
        float dy[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = 16 * rt + 4 * g + i;
            const float trow = __shfl(t, row, 64);
            const bool vrow = (int64_t)blockIdx.x * 64 + row < n_step;
            const float r = part[i] + p[kOffB3] - trow;
            dy[i] = vrow ? 2.0f * r * inv_count : 0.0f;
            if (n == 0 && vrow) {
                loss = fmaf(r, r, loss);
                gb3 += dy[i];
            }
        }
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const int col = 16 * ct + n;
            const float w3 = p[kOffW3 + col];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * rt + 4 * g + i;
                const float z = z2[ct][i], s = sg[ct][i];
                const float dz = dy[i] * w3 * (s * (1.0f + z * (1.0f - s)));
                gb2[ct] += dz;
                gw3[ct] = fmaf(dy[i], z * s, gw3[ct]);
                const uint16_t q = bf16_bits(dz);
                DZ2[row * kH1Stride + col] = q;
                DZ2T[col * kTStride + row] = q;
            }
        }
    }
    __syncthreads();
    float *out = partials + (size_t)blockIdx.x * kPartialStride;
    // ---- dW2 = dz2^T h1 (K = the 64 samples)
    for (int mt = 0; mt < 4; ++mt)
        for (int nt = 0; nt < 4; ++nt) {
            f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
            for (int ks = 0; ks < 2; ++ks)
                acc = mfma(frag(DZ2T + (16 * mt + n) * kTStride + 32 * ks + 8 * g),
                           frag(H1T + (16 * nt + n) * kTStride + 32 * ks + 8 * g), acc);
#pragma unroll
            for (int i = 0; i < 4; ++i) out[kOffW2 + (16 * mt + 4 * g + i) * kMlpH + 16 * nt + n] = acc[i];
        }
    // ---- dh1 = dz2 W2, then dz1 = dh1 silu'(z1), dW1 and db1
    bf16x8 bt[4][2];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) bt[nt][ks] = frag(m.w2t + (16 * nt + n) * kMlpH + 32 * ks + 8 * g);
    float gb1[4] = {0, 0, 0, 0}, gw1[4][4] = {{0}};
    for (int rt = 0; rt < 4; ++rt) {
        f32x4 acc[4];
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) acc[nt] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const bf16x8 a = frag(DZ2 + (16 * rt + n) * kH1Stride + 32 * ks + 8 * g);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) acc[nt] = mfma(a, bt[nt][ks], acc[nt]);
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int row = 16 * rt + 4 * g + i, col = 16 * nt + n;
                const float z = Z1s[row][col], s = sigmoid(z);
                const float dz = acc[nt][i] * (s * (1.0f + z * (1.0f - s)));
                gb1[nt] += dz;
#pragma unroll
                for (int k = 0; k < 4; ++k) gw1[nt][k] = fmaf(dz, Xs[row][k], gw1[nt][k]);
            }
    }
    // ---- column partials: sum the four lane groups, lanes 0..15 write
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        gb2[c] += __shfl_xor(gb2[c], 16, 64);
        gb2[c] += __shfl_xor(gb2[c], 32, 64);
        gw3[c] += __shfl_xor(gw3[c], 16, 64);
        gw3[c] += __shfl_xor(gw3[c], 32, 64);
        gb1[c] += __shfl_xor(gb1[c], 16, 64);
        gb1[c] += __shfl_xor(gb1[c], 32, 64);
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            gw1[c][k] += __shfl_xor(gw1[c][k], 16, 64);
            gw1[c][k] += __shfl_xor(gw1[c][k], 32, 64);
        }
    }
    if (g == 0) {
#pragma unroll
        for (int c = 0; c < 4; ++c) {
            const int col = 16 * c + n;
            out[kOffB2 + col] = gb2[c];
            out[kOffW3 + col] = gw3[c];
            out[kOffB1 + col] = gb1[c];
#pragma unroll
            for (int k = 0; k < 4; ++k) out[kOffW1 + col * kMlpIn + k] = gw1[c][k];
        }
    }
    for (int mm = 1; mm < 64; mm <<= 1) {
        gb3 += __shfl_xor(gb3, mm, 64);
        loss += __shfl_xor(loss, mm, 64);
    }
    if (l == 0) {
        out[kOffB3] = gb3;
        out[kMlpParams] = loss;
    }
}

/*
 * Sum of the waves' gradient partials (in wave order, one thread per
 * parameter: a fixed summation order, so training stays deterministic) and
 * the Adam step.  The loads of 32 partials are issued before they are added.
 */
constexpr int kReduceBlock = 64;
constexpr int kReduceBatch = 32;
__global__ __launch_bounds__(kReduceBlock) void k_mlp_reduce(
    float *__restrict__ params, float *__restrict__ m1, float *__restrict__ m2, uint16_t *__restrict__ w2,
    uint16_t *__restrict__ w2t, const float *__restrict__ partials, int n_waves, int adam, float lr, float b1,
    float b2, float eps, float bc1, float bc2, float *__restrict__ grad_out)
{
    const int k = blockIdx.x * kReduceBlock + threadIdx.x;
    if (k > kMlpParams) return;
    float gsum = 0.0f;
    int w = 0;
    for (; w + kReduceBatch <= n_waves; w += kReduceBatch) {
        float v[kReduceBatch];
#pragma unroll
        for (int u = 0; u < kReduceBatch; ++u) v[u] = partials[(size_t)(w + u) * kPartialStride + k];
#pragma unroll
        for (int u = 0; u < kReduceBatch; ++u) gsum += v[u];
    }
    for (; w < n_waves; ++w) gsum += partials[(size_t)w * kPartialStride + k];
    if (grad_out) grad_out[k] = gsum;
    if (!adam || k == kMlpParams) return;
    const float mm = b1 * m1[k] + (1.0f - b1) * gsum;
    const float vv = b2 * m2[k] + (1.0f - b2) * gsum * gsum;
    m1[k] = mm;
    m2[k] = vv;
    const float pk = params[k] - lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
    params[k] = pk;
    if (k >= kOffW2 && k < kOffB2) {
        const int o = (k - kOffW2) / kMlpH, i = (k - kOffW2) % kMlpH;
        const uint16_t q = bf16_bits(pk);
        w2[o * kMlpH + i] = q;
        w2t[i * kMlpH + o] = q;
    }
}

__global__ __launch_bounds__(256) void k_mlp_bf16_copies(const float *__restrict__ params, uint16_t *__restrict__ w2,
                                                         uint16_t *__restrict__ w2t)
{
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= kMlpH * kMlpH) return;
    const int o = k / kMlpH, i = k % kMlpH;
    const uint16_t q = bf16_bits(params[kOffW2 + k]);
    w2[o * kMlpH + i] = q;
    w2t[i * kMlpH + o] = q;
}

}  // namespace

hipError_t launch_mlp_targets(const MlpTargetDev &k, const float *samples, int64_t n, float *features, float *targets,
                              hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_targets, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, k, samples, n, features,
                       targets);
    return hipGetLastError();
}

hipError_t launch_mlp_forward(const MlpDev &m, const float *features, int64_t n, float *out, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_forward, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, m, features, n, out);
    return hipGetLastError();
}

hipError_t launch_mlp_grad(const MlpDev &m, const float *features, const float *targets, int64_t n_total, int64_t base,
                           int64_t n_step, uint64_t stride, uint64_t offset, float inv_count, float *partials,
                           hipStream_t s)
{
    const unsigned waves = (unsigned)((n_step + 63) / 64);
    hipLaunchKernelGGL(k_mlp_grad, dim3(waves), dim3(64), 0, s, m, features, targets, n_total, base, n_step, stride,
                       offset, inv_count, partials);
    return hipGetLastError();
}

hipError_t launch_mlp_reduce(float *params, float *m1, float *m2, uint16_t *w2, uint16_t *w2t, const float *partials,
                             int n_waves, int adam, float lr, float b1, float b2, float eps, float bc1, float bc2,
                             float *grad_out, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_reduce, dim3((kMlpParams + 1 + kReduceBlock - 1) / kReduceBlock), dim3(kReduceBlock), 0,
                       s, params, m1, m2, w2, w2t, partials, n_waves, adam, lr, b1, b2, eps, bc1, bc2, grad_out);
    return hipGetLastError();
}

hipError_t launch_mlp_bf16_copies(const float *params, uint16_t *w2, uint16_t *w2t, hipStream_t s)
{
    hipLaunchKernelGGL(k_mlp_bf16_copies, dim3((kMlpH * kMlpH + 255) / 256), dim3(256), 0, s, params, w2, w2t);
    return hipGetLastError();
}

}  // namespace fspb
