/*
 * Kernel surrogate: a 4 -> 64 -> 64 -> 1 SiLU perceptron that approximates
 * K(d, u, v, a) = PDD(d) F(u, v; a, a, d) (Eq. 2-3 without the inverse
 * square), trained and evaluated by the gfx950 kernels of fspb_mlp.hip.
 * Internal header (not part of the public ABI).
 *
 * Parameter vector (FP32 masters, 4545 values): W1[64][4], b1[64],
 * W2[64][64], b2[64], W3[64], b3; W[o][i] maps input i to output o.
 * Features: x0 = 2 sqrt(d/30) - 1, x1 = 2 sqrt(|u|/3) - 1,
 * x2 = 2 sqrt(|v|/3) - 1, x3 = (a - 0.625)/0.375; the training box
 * d in [0, 30], |u|, |v| <= 3, a in [0.25, 1] maps onto [-1, 1]^4.
 *
 * Precision: layer 1, the activations and layer 3 are FP32; the 64 x 64
 * layer runs on BF16 matrix cores with FP32 accumulation: its inputs h1 and
 * its weights W2 are rounded to BF16 (round to nearest even), and in the
 * backward pass dz2, h1 and W2 are rounded the same way.
 */
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace fspb {

constexpr int kMlpH = 64;
constexpr int kMlpIn = 4;
constexpr int kOffW1 = 0;
constexpr int kOffB1 = kOffW1 + kMlpH * kMlpIn;
constexpr int kOffW2 = kOffB1 + kMlpH;
constexpr int kOffB2 = kOffW2 + kMlpH * kMlpH;
constexpr int kOffW3 = kOffB2 + kMlpH;
constexpr int kOffB3 = kOffW3 + kMlpH;
constexpr int kMlpParams = kOffB3 + 1;          // 4545
constexpr int kPartialStride = 4608;            // per-wave gradient partials (+ loss at kMlpParams)

// training-box limits of the surrogate's inputs
constexpr float kMlpDMax = 30.0f;
constexpr float kMlpUVMax = 3.0f;
constexpr float kMlpAMin = 0.25f, kMlpAMax = 1.0f;

/* Device view of a surrogate's parameters. */
struct MlpDev {
    const float *p;            // FP32 parameters
    const uint16_t *w2;        // BF16 W2 [out][in]
    const uint16_t *w2t;       // BF16 W2 transposed [in][out]
};

/* Kernel-parameter record used to generate training targets on the device. */
struct MlpTargetDev {
    int32_t n_terms, n_pdd;
    float w4[4], sig0[4], sig1[4], c2[4];
    float pdd_inv_step, pdd_max;
    const float *pdd;
    const float4 *erfc_tab;
};

hipError_t launch_mlp_targets(const MlpTargetDev &k, const float *samples, int64_t n, float *features,
                              float *targets, hipStream_t s);
hipError_t launch_mlp_forward(const MlpDev &m, const float *features, int64_t n, float *out, hipStream_t s);
/* One step's gradient partials: sample i of the step is permuted index
 * (offset + (base + i) * stride) mod n_total; n_step samples in 64-sample waves. */
hipError_t launch_mlp_grad(const MlpDev &m, const float *features, const float *targets, int64_t n_total,
                           int64_t base, int64_t n_step, uint64_t stride, uint64_t offset, float inv_count,
                           float *partials, hipStream_t s);
/* Reduce partials of n_waves waves; with adam != 0 update params/m/v and the
 * BF16 copies, else write the summed gradient and loss to grad_out. */
hipError_t launch_mlp_reduce(float *params, float *m1, float *m2, uint16_t *w2, uint16_t *w2t,
                             const float *partials, int n_waves, int adam, float lr, float b1, float b2,
                             float eps, float bc1, float bc2, float *grad_out, hipStream_t s);
hipError_t launch_mlp_bf16_copies(const float *params, uint16_t *w2, uint16_t *w2t, hipStream_t s);

}  // namespace fspb
