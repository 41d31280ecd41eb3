/*
 * Wave-level building blocks of the kernel surrogate (see fspb_mlp.h):
 * BF16 rounding, SiLU, W2 fragments for v_mfma_f32_16x16x32_bf16, and the
 * forward pass of 64 samples (one per lane) used both by training and by the
 * fused fill.
 *
 * v_mfma_f32_16x16x32_bf16 operand layout (one wave): lane l supplies
 * A[m = l % 16][k = 8 (l / 16) + i] and B[k = 8 (l / 16) + i][n = l % 16],
 * i = 0..7, and receives D[m = 4 (l / 16) + i][n = l % 16], i = 0..3.
 */
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "fspb_mlp.h"

namespace fspb {
namespace mlp {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(4))) float f32x4;

constexpr int kH1Stride = 68;    // bf16 per row of a [64][64] tile read as A fragments (136 B rows)
constexpr int kTStride = 72;     // bf16 per row of a transposed tile read as A/B fragments (144 B rows)

__device__ inline int lane() { return threadIdx.x & 63; }

/* float -> bfloat16 bits, round to nearest even (finite inputs). */
__device__ inline uint16_t bf16_bits(float f)
{
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

__device__ inline float sigmoid(float z) { return __builtin_amdgcn_rcpf(1.0f + __expf(-z)); }

__device__ inline f32x4 mfma(const bf16x8 &a, const bf16x8 &b, const f32x4 &c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ inline bf16x8 frag(const uint16_t *p) { return *reinterpret_cast<const bf16x8 *>(p); }

/* B fragments of W2^T for the forward product h1 W2^T: b[ct][ks] covers outputs
 * 16 ct .. 16 ct + 15 and inputs 32 ks .. 32 ks + 31. */
struct W2Frags {
    bf16x8 b[4][2];
};

__device__ inline void load_w2_frags(const uint16_t *__restrict__ w2, W2Frags &f)
{
    const int n = lane() & 15, kq = (lane() >> 4) * 8;
#pragma unroll
    for (int ct = 0; ct < 4; ++ct)
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) f.b[ct][ks] = frag(w2 + (16 * ct + n) * kMlpH + 32 * ks + kq);
}

/* Features of the training box, [-1, 1]^4 (square-root stretch of d, |u|, |v|). */
__device__ inline float feature_a(float a) { return (a - 0.625f) * (1.0f / 0.375f); }
__device__ inline void features(float d, float au, float av, float a, float x[4])
{
    x[0] = 2.0f * __builtin_sqrtf(fmaxf(d, 0.0f) * (1.0f / 30.0f)) - 1.0f;
    x[1] = 2.0f * __builtin_sqrtf(au * (1.0f / 3.0f)) - 1.0f;
    x[2] = 2.0f * __builtin_sqrtf(av * (1.0f / 3.0f)) - 1.0f;
    x[3] = feature_a(a);
}

/*
 * Forward pass of 64 samples, sample = lane, features x.  h1s: this wave's
 * [64][kH1Stride] BF16 LDS tile.  p: FP32 parameters.  With FOLD the fourth
 * feature is the same for every sample and b1x (LDS) holds the layer-1 bias
 * with its term added, b1 + W1[:, 3] x[3]; x[3] is then not read.  Returns the
 * output for the lane's sample.  Every lane of the wave must call it.
 */
template <bool FOLD>
__device__ inline float forward_wave(const float *__restrict__ p, const float *b1x, const W2Frags &wf,
                                     const float x[4], uint16_t *h1s)
{
    const int l = lane();
    // layer 1 (FP32), h1 rounded to BF16 into the lane's row
#pragma unroll 4
    for (int o = 0; o < kMlpH; o += 2) {
        float z0 = FOLD ? b1x[o] : p[kOffB1 + o], z1 = FOLD ? b1x[o + 1] : p[kOffB1 + o + 1];
#pragma unroll
        for (int k = 0; k < (FOLD ? kMlpIn - 1 : kMlpIn); ++k) {
            z0 = fmaf(p[kOffW1 + o * kMlpIn + k], x[k], z0);
            z1 = fmaf(p[kOffW1 + (o + 1) * kMlpIn + k], x[k], z1);
        }
        const uint32_t pk = (uint32_t)bf16_bits(z0 * sigmoid(z0)) | ((uint32_t)bf16_bits(z1 * sigmoid(z1)) << 16);
        *reinterpret_cast<uint32_t *>(h1s + l * kH1Stride + o) = pk;
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // layer 2 on matrix cores, layer 3 as a dot over each lane's columns + 16-lane reduction
    const int n = l & 15, g = l >> 4;
    float y = 0.0f;
#pragma unroll
    for (int rt = 0; rt < 4; ++rt) {
        f32x4 acc[4];
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) acc[ct] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ks = 0; ks < 2; ++ks) {
            const bf16x8 a = frag(h1s + (16 * rt + n) * kH1Stride + 32 * ks + 8 * g);
#pragma unroll
            for (int ct = 0; ct < 4; ++ct) acc[ct] = mfma(a, wf.b[ct][ks], acc[ct]);
        }
        float part[4] = {0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int ct = 0; ct < 4; ++ct) {
            const float b2 = p[kOffB2 + 16 * ct + n], w3 = p[kOffW3 + 16 * ct + n];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float z = acc[ct][i] + b2;
                part[i] = fmaf(z * sigmoid(z), w3, part[i]);
            }
        }
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int m = 1; m < 16; m <<= 1) part[i] += __shfl_xor(part[i], m, 64);
        // row 16 rt + 4 g' + i is held by the lanes of group g'; lane 16 rt + q wants q = 4 g' + i
        const int src = 16 * ((l & 15) >> 2);
        const float v0 = __shfl(part[0], src, 64), v1 = __shfl(part[1], src, 64);
        const float v2 = __shfl(part[2], src, 64), v3 = __shfl(part[3], src, 64);
        const int q = l & 3;
        const float mine = q == 0 ? v0 : (q == 1 ? v1 : (q == 2 ? v2 : v3));
        if (g == rt) y = mine;
    }
    return y + p[kOffB3];
}

}  // namespace mlp
}  // namespace fspb
