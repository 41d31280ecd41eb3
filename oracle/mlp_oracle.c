/*
 * Kernel surrogate MLP -- plain FP64 CPU oracle.
 *
 * TEST INFRASTRUCTURE ONLY (same rules as fspb_oracle.c: tests, the smoke
 * check and the CPU-baseline leg may load it; the library never does).
 *
 * The surrogate approximates the FSPB kernel value K(d, u, v, a) =
 * PDD(d) F(u, v; a, a, d) (Eq. 2-3 without the inverse-square factor) with a
 * 4 -> 64 -> 64 -> 1 multilayer perceptron, SiLU activations, trained by mean
 * squared error.  Feature map (part of the model's definition):
 *   x0 = 2 sqrt(d / 30) - 1,  x1 = 2 sqrt(|u| / 3) - 1,  x2 = 2 sqrt(|v| / 3) - 1,
 *   x3 = (a - 0.625) / 0.375,
 * so the training box d in [0, 30], |u|, |v| in [0, 3], a in [0.25, 1] maps to
 * [-1, 1]^4.  The square roots spread the steep parts of K -- the depth-dose
 * build-up near d = 0 and the beamlet edges near |u|, |v| = a/2 -- over more
 * of the feature range; K is even in u and v and linear in d near 0, so it
 * stays smooth in these coordinates.
 *
 * Parameter layout (4545 values): W1[64][4], b1[64], W2[64][64], b2[64],
 * W3[64], b3[1]; W[o][i] multiplies input i into output o.
 *
 * With bf16 != 0 the values that the GPU feeds to its BF16 matrix cores are
 * rounded to bfloat16 (round to nearest, ties to even) first:
 *   forward  z2 = W2 h1        : W2 and h1 rounded
 *   backward dW2 = dz2^T h1    : dz2 and h1 rounded
 *            dh1 = dz2 W2      : dz2 and W2 rounded
 * everything else stays FP64, so the two sides then differ only by
 * accumulation order and FP32 rounding.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define H 64
#define NIN 4
#define OFF_W1 0
#define OFF_B1 (OFF_W1 + H * NIN)
#define OFF_W2 (OFF_B1 + H)
#define OFF_B2 (OFF_W2 + H * H)
#define OFF_W3 (OFF_B2 + H)
#define OFF_B3 (OFF_W3 + H)
#define NPARAM (OFF_B3 + 1)

int32_t ofs_mlp_nparams(void) { return NPARAM; }

/* bfloat16 round-to-nearest-even of a value first rounded to float. */
double ofs_bf16_round(double v)
{
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return v;          /* inf / nan untouched */
    uint32_t lsb = (u >> 16) & 1u;
    u = (u + 0x7fffu + lsb) & 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

static double silu(double z) { return z / (1.0 + exp(-z)); }

static double silu_grad(double z)
{
    double s = 1.0 / (1.0 + exp(-z));
    return s * (1.0 + z * (1.0 - s));
}

void ofs_surrogate_features(const double *raw, int64_t n, double *feat)
{
    for (int64_t i = 0; i < n; ++i) {
        feat[4 * i + 0] = 2.0 * sqrt(fmax(raw[4 * i + 0], 0.0) / 30.0) - 1.0;
        feat[4 * i + 1] = 2.0 * sqrt(fabs(raw[4 * i + 1]) / 3.0) - 1.0;
        feat[4 * i + 2] = 2.0 * sqrt(fabs(raw[4 * i + 2]) / 3.0) - 1.0;
        feat[4 * i + 3] = (raw[4 * i + 3] - 0.625) / 0.375;
    }
}

typedef struct { double z1[H], h1[H], h1q[H], z2[H], h2[H], y; } act;

static void forward_one(const double *p, const double *W2q, const double *x, act *A, int bf16)
{
    for (int o = 0; o < H; ++o) {
        double s = p[OFF_B1 + o];
        for (int i = 0; i < NIN; ++i) s += p[OFF_W1 + o * NIN + i] * x[i];
        A->z1[o] = s;
        A->h1[o] = silu(s);
        A->h1q[o] = bf16 ? ofs_bf16_round(A->h1[o]) : A->h1[o];
    }
    for (int o = 0; o < H; ++o) {
        double s = 0.0;
        for (int i = 0; i < H; ++i) s += W2q[o * H + i] * A->h1q[i];
        A->z2[o] = s + p[OFF_B2 + o];
        A->h2[o] = silu(A->z2[o]);
    }
    double y = p[OFF_B3];
    for (int i = 0; i < H; ++i) y += p[OFF_W3 + i] * A->h2[i];
    A->y = y;
}

static double *quantised_w2(const double *p, int bf16)
{
    double *w = (double *)malloc(sizeof(double) * H * H);
    for (int k = 0; k < H * H; ++k) w[k] = bf16 ? ofs_bf16_round(p[OFF_W2 + k]) : p[OFF_W2 + k];
    return w;
}

void ofs_mlp_forward(const double *p, const double *x, int64_t n, double *y, int32_t bf16)
{
    double *W2q = quantised_w2(p, bf16);
    act A;
    for (int64_t s = 0; s < n; ++s) {
        forward_one(p, W2q, x + 4 * s, &A, bf16);
        y[s] = A.y;
    }
    free(W2q);
}

/*
 * Mean squared error over the batch and its gradient with respect to every
 * parameter (written to grad, NPARAM values).  Returns the loss.
 */
double ofs_mlp_loss_grad(const double *p, const double *x, const double *target, int64_t n,
                         double *grad, int32_t bf16)
{
    double *W2q = quantised_w2(p, bf16);
    memset(grad, 0, sizeof(double) * NPARAM);
    double loss = 0.0;
    act A;
    double dz2[H], dz2q[H], dz1[H];
    for (int64_t s = 0; s < n; ++s) {
        const double *xs = x + 4 * s;
        forward_one(p, W2q, xs, &A, bf16);
        double r = A.y - target[s];
        loss += r * r;
        double dy = 2.0 * r / (double)n;
        grad[OFF_B3] += dy;
        for (int i = 0; i < H; ++i) {
            grad[OFF_W3 + i] += dy * A.h2[i];
            dz2[i] = dy * p[OFF_W3 + i] * silu_grad(A.z2[i]);
            dz2q[i] = bf16 ? ofs_bf16_round(dz2[i]) : dz2[i];
            grad[OFF_B2 + i] += dz2[i];
        }
        for (int o = 0; o < H; ++o)
            for (int i = 0; i < H; ++i) grad[OFF_W2 + o * H + i] += dz2q[o] * A.h1q[i];
        for (int i = 0; i < H; ++i) {
            double dh = 0.0;
            for (int o = 0; o < H; ++o) dh += dz2q[o] * W2q[o * H + i];
            dz1[i] = dh * silu_grad(A.z1[i]);
            grad[OFF_B1 + i] += dz1[i];
            for (int k = 0; k < NIN; ++k) grad[OFF_W1 + i * NIN + k] += dz1[i] * xs[k];
        }
    }
    free(W2q);
    return loss / (double)n;
}
