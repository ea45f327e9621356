/*
 * mlp_oracle.c -- FP64 reference for the learned self-collision screen.
 * TEST INFRASTRUCTURE ONLY (see ezo_oracle.c).
 *
 * The screen is a multilayer perceptron D -> H -> H -> H -> 1 with SiLU
 * activations that predicts a configuration's minimum self-collision signed
 * distance from x = q / pi.  It is trained with a Huber loss on targets
 * clipped to [clip_lo, clip_hi].  Parameters are one flat vector in the order
 *   W1[H][D] b1[H] W2[H][H] b2[H] W3[H][H] b3[H] W4[H] b4[1]
 * (W[out][in], z = W a + b).  This file computes the plain definitions:
 * forward pass, mean loss over a batch, and its exact gradient by the chain
 * rule, one sample at a time.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

static double sigmoid(double z) { return 1.0 / (1.0 + exp(-z)); }
static double silu(double z) { return z * sigmoid(z); }
static double silu_grad(double z) {
    double s = sigmoid(z);
    return s * (1.0 + z * (1.0 - s));
}

int64_t orc_mlp_num_params(int32_t D, int32_t H) {
    return (int64_t)H * D + H + 2 * ((int64_t)H * H + H) + H + 1;
}

typedef struct {
    const double *W1, *b1, *W2, *b2, *W3, *b3, *W4, *b4;
} mlp_view;

static mlp_view view_of(const double *p, int D, int H) {
    mlp_view v;
    v.W1 = p; p += (size_t)H * D;
    v.b1 = p; p += H;
    v.W2 = p; p += (size_t)H * H;
    v.b2 = p; p += H;
    v.W3 = p; p += (size_t)H * H;
    v.b3 = p; p += H;
    v.W4 = p; p += H;
    v.b4 = p;
    return v;
}

static void dense(const double *W, const double *b, const double *a, int out, int in, double *z) {
    for (int i = 0; i < out; ++i) {
        double s = b[i];
        for (int j = 0; j < in; ++j) s += W[(size_t)i * in + j] * a[j];
        z[i] = s;
    }
}

/* One sample: pre-activations z1..z3, activations a1..a3, output y. */
static double forward_one(const mlp_view *v, int D, int H, const double *x, double *z1, double *a1, double *z2,
                          double *a2, double *z3, double *a3) {
    dense(v->W1, v->b1, x, H, D, z1);
    for (int i = 0; i < H; ++i) a1[i] = silu(z1[i]);
    dense(v->W2, v->b2, a1, H, H, z2);
    for (int i = 0; i < H; ++i) a2[i] = silu(z2[i]);
    dense(v->W3, v->b3, a2, H, H, z3);
    for (int i = 0; i < H; ++i) a3[i] = silu(z3[i]);
    double y = v->b4[0];
    for (int i = 0; i < H; ++i) y += v->W4[i] * a3[i];
    return y;
}

void orc_mlp_forward(int32_t D, int32_t H, const double *params, const double *x, int64_t n, double *y) {
    mlp_view v = view_of(params, D, H);
#pragma omp parallel
    {
        double *tmp = (double *)malloc(sizeof(double) * 6 * (size_t)H);
#pragma omp for schedule(static)
        for (int64_t r = 0; r < n; ++r)
            y[r] = forward_one(&v, D, H, x + (size_t)r * D, tmp, tmp + H, tmp + 2 * H, tmp + 3 * H, tmp + 4 * H,
                               tmp + 5 * H);
        free(tmp);
    }
}

static double clip(double t, double lo, double hi) { return t < lo ? lo : (t > hi ? hi : t); }

/* Huber loss with threshold d: r^2/2 for |r| <= d, else d (|r| - d/2). */
static double huber(double r, double d) { return fabs(r) <= d ? 0.5 * r * r : d * (fabs(r) - 0.5 * d); }
static double huber_grad(double r, double d) { return fabs(r) <= d ? r : (r > 0 ? d : -d); }

/* Mean Huber loss over n samples and its gradient w.r.t. every parameter
 * (grad has the parameter layout).  Targets are clipped first. */
double orc_mlp_loss_grad(int32_t D, int32_t H, const double *params, const double *x, const double *t, int64_t n,
                         double huber_delta, double clip_lo, double clip_hi, double *grad) {
    mlp_view v = view_of(params, D, H);
    const int64_t P = orc_mlp_num_params(D, H);
    memset(grad, 0, sizeof(double) * (size_t)P);
    mlp_view g = view_of(grad, D, H);
    double *z1 = (double *)malloc(sizeof(double) * 9 * (size_t)H);
    double *a1 = z1 + H, *z2 = z1 + 2 * H, *a2 = z1 + 3 * H, *z3 = z1 + 4 * H, *a3 = z1 + 5 * H;
    double *d3 = z1 + 6 * H, *d2 = z1 + 7 * H, *d1 = z1 + 8 * H;
    double loss = 0.0;
    for (int64_t r = 0; r < n; ++r) {
        const double *xr = x + (size_t)r * D;
        double y = forward_one(&v, D, H, xr, z1, a1, z2, a2, z3, a3);
        double res = y - clip(t[r], clip_lo, clip_hi);
        loss += huber(res, huber_delta);
        double dy = huber_grad(res, huber_delta) / (double)n;
        /* output layer */
        ((double *)g.b4)[0] += dy;
        for (int i = 0; i < H; ++i) {
            ((double *)g.W4)[i] += dy * a3[i];
            d3[i] = dy * v.W4[i] * silu_grad(z3[i]);
        }
        /* layer 3: z3 = W3 a2 + b3 */
        for (int i = 0; i < H; ++i) {
            ((double *)g.b3)[i] += d3[i];
            for (int j = 0; j < H; ++j) ((double *)g.W3)[(size_t)i * H + j] += d3[i] * a2[j];
        }
        for (int j = 0; j < H; ++j) {
            double s = 0.0;
            for (int i = 0; i < H; ++i) s += v.W3[(size_t)i * H + j] * d3[i];
            d2[j] = s * silu_grad(z2[j]);
        }
        /* layer 2 */
        for (int i = 0; i < H; ++i) {
            ((double *)g.b2)[i] += d2[i];
            for (int j = 0; j < H; ++j) ((double *)g.W2)[(size_t)i * H + j] += d2[i] * a1[j];
        }
        for (int j = 0; j < H; ++j) {
            double s = 0.0;
            for (int i = 0; i < H; ++i) s += v.W2[(size_t)i * H + j] * d2[i];
            d1[j] = s * silu_grad(z1[j]);
        }
        /* layer 1 */
        for (int i = 0; i < H; ++i) {
            ((double *)g.b1)[i] += d1[i];
            for (int j = 0; j < D; ++j) ((double *)g.W1)[(size_t)i * D + j] += d1[i] * xr[j];
        }
    }
    free(z1);
    return loss / (double)n;
}

/* Loss only (for finite differences). */
double orc_mlp_loss(int32_t D, int32_t H, const double *params, const double *x, const double *t, int64_t n,
                    double huber_delta, double clip_lo, double clip_hi) {
    mlp_view v = view_of(params, D, H);
    double *tmp = (double *)malloc(sizeof(double) * 6 * (size_t)H);
    double loss = 0.0;
    for (int64_t r = 0; r < n; ++r) {
        double y = forward_one(&v, D, H, x + (size_t)r * D, tmp, tmp + H, tmp + 2 * H, tmp + 3 * H, tmp + 4 * H,
                               tmp + 5 * H);
        loss += huber(y - clip(t[r], clip_lo, clip_hi), huber_delta);
    }
    free(tmp);
    return loss / (double)n;
}
