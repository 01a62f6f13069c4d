/*
 * Placement MLP oracle -- TEST INFRASTRUCTURE ONLY (see fsne_oracle.h).
 *
 * A multilayer perceptron D -> H1 -> H2 -> d with ReLU hidden layers that maps
 * HD coordinates to embedding coordinates, trained by mean squared error on
 * (x, y) pairs of a converged embedding, to place inserted or drifted points
 * (dynamic data, Sec. 3 on online use and Sec. 5).  The paper does not
 * describe this network; its architecture, loss and optimiser are readings:
 * ReLU, MSE on standardised y, Adam (Kingma and Ba 2015), He-uniform init.
 *
 * Parameters are one flat float32 array:
 *   W1 (H1 x D), b1 (H1), W2 (H2 x H1), b2 (H2), W3 (d x H2), b3 (d).
 *
 * Arithmetic is double.  With bf16_ops = 1 the operands of the three large
 * products (x W1^T, h1 W2^T, and the backward products that involve W2, h1, x
 * and the hidden gradients) are first rounded to bfloat16 (through float,
 * round to nearest even), which is what the matrix cores are fed; the
 * 2-wide output layer stays unrounded.  With bf16_ops = 0 the network is
 * plain double (used for finite-difference pins).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int32_t D, H1, H2, d;
} fsneo_mlp_dims;

void fsneo_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);

int64_t fsneo_mlp_nparams(const fsneo_mlp_dims *m)
{
    return (int64_t)m->H1 * m->D + m->H1 + (int64_t)m->H2 * m->H1 + m->H2 +
           (int64_t)m->d * m->H2 + m->d;
}

/* He-uniform: w = (2u - 1) sqrt(6 / fan_in), u = (draw >> 8) 2^-24 from the */
/* Philox block (index, layer, 8, 0); biases 0.  Single precision, each     */
/* operation rounded (no fused multiply-add).                                */
void fsneo_mlp_init(const fsneo_mlp_dims *m, uint64_t seed, float *p)
{
    const int32_t fan_in[3] = {m->D, m->H1, m->H2};
    const int64_t n_w[3] = {(int64_t)m->H1 * m->D, (int64_t)m->H2 * m->H1, (int64_t)m->d * m->H2};
    const int64_t n_b[3] = {m->H1, m->H2, m->d};
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    int64_t o = 0;
    for (int layer = 0; layer < 3; ++layer) {
        volatile float six = 6.0f;
        volatile float ratio = six / (float)fan_in[layer];
        float bound = sqrtf(ratio);
        for (int64_t k = 0; k < n_w[layer]; ++k) {
            uint32_t ctr[4] = {(uint32_t)k, (uint32_t)layer, 8u, 0u}, u[4];
            fsneo_philox4x32_10(ctr, key, u);
            volatile float unit = (float)(u[0] >> 8) * 5.9604644775390625e-08f; /* 2^-24 */
            volatile float two_u = 2.0f * unit;
            volatile float centred = two_u - 1.0f;
            volatile float w = centred * bound;
            p[o + k] = w;
        }
        o += n_w[layer];
        for (int64_t k = 0; k < n_b[layer]; ++k) p[o + k] = 0.0f;
        o += n_b[layer];
    }
}

static double bf16_round(double v)
{
    float f = (float)v;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7F800000u) == 0x7F800000u) return (double)f;
    u = (u + 0x7FFFu + ((u >> 16) & 1u)) & 0xFFFF0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

static double op(double v, int bf) { return bf ? bf16_round(v) : v; }

static double xin(const void *X, int32_t xdtype, int64_t k)
{
    if (xdtype == 0) return (double)((const float *)X)[k];
    uint32_t u = (uint32_t)((const uint16_t *)X)[k] << 16;
    float f;
    memcpy(&f, &u, 4);
    return (double)f;
}

typedef struct {
    const float *W1, *b1, *W2, *b2, *W3, *b3;
} params_view;

static params_view view(const fsneo_mlp_dims *m, const float *p)
{
    params_view v;
    v.W1 = p;
    v.b1 = v.W1 + (int64_t)m->H1 * m->D;
    v.W2 = v.b1 + m->H1;
    v.b2 = v.W2 + (int64_t)m->H2 * m->H1;
    v.W3 = v.b2 + m->H2;
    v.b3 = v.W3 + (int64_t)m->d * m->H2;
    return v;
}

/* Forward pass of one row: h1, h2 (post-ReLU) and out. */
static void forward_row(const fsneo_mlp_dims *m, const params_view *P, const void *X,
                        int32_t xdtype, int64_t r, int bf, double *h1, double *h2, double *out)
{
    for (int32_t j = 0; j < m->H1; ++j) {
        double s = 0.0;
        for (int32_t k = 0; k < m->D; ++k)
            s += op(xin(X, xdtype, r * m->D + k), bf) * op(P->W1[(int64_t)j * m->D + k], bf);
        s += P->b1[j];
        h1[j] = s > 0.0 ? s : 0.0;
    }
    for (int32_t j = 0; j < m->H2; ++j) {
        double s = 0.0;
        for (int32_t k = 0; k < m->H1; ++k)
            s += op(h1[k], bf) * op(P->W2[(int64_t)j * m->H1 + k], bf);
        s += P->b2[j];
        h2[j] = s > 0.0 ? s : 0.0;
    }
    for (int32_t j = 0; j < m->d; ++j) {
        double s = 0.0;
        for (int32_t k = 0; k < m->H2; ++k) s += h2[k] * P->W3[(int64_t)j * m->H2 + k];
        out[j] = s + P->b3[j];
    }
}

void fsneo_mlp_forward(const fsneo_mlp_dims *m, const float *p, const void *X, int32_t xdtype,
                       int64_t n, int32_t bf, double *out)
{
    params_view P = view(m, p);
#pragma omp parallel
    {
        double *h1 = malloc(sizeof(double) * m->H1), *h2 = malloc(sizeof(double) * m->H2);
#pragma omp for schedule(static)
        for (int64_t r = 0; r < n; ++r) forward_row(m, &P, X, xdtype, r, bf, h1, h2, out + r * m->d);
        free(h1);
        free(h2);
    }
}

/* Loss L = 1/(n d) sum (out - t)^2 over the n rows, and its gradient with  */
/* respect to every parameter (flat, same layout as p).                      */
double fsneo_mlp_loss_grad(const fsneo_mlp_dims *m, const float *p, const void *X,
                           int32_t xdtype, const float *T, int64_t n, int32_t bf, double *g)
{
    params_view P = view(m, p);
    const int32_t D = m->D, H1 = m->H1, H2 = m->H2, d = m->d;
    double *h1 = malloc(sizeof(double) * n * H1), *h2 = malloc(sizeof(double) * n * H2);
    double *out = malloc(sizeof(double) * n * d), *dh2 = malloc(sizeof(double) * n * H2);
    double *dh1 = malloc(sizeof(double) * n * H1);
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r)
        forward_row(m, &P, X, xdtype, r, bf, h1 + r * H1, h2 + r * H2, out + r * d);
    double loss = 0.0;
    for (int64_t r = 0; r < n; ++r)
        for (int32_t j = 0; j < d; ++j) {
            double e = out[r * d + j] - (double)T[r * d + j];
            loss += e * e;
        }
    loss /= (double)(n * d);
    /* output layer */
    double *gW1 = g, *gb1 = gW1 + (int64_t)H1 * D, *gW2 = gb1 + H1, *gb2 = gW2 + (int64_t)H2 * H1;
    double *gW3 = gb2 + H2, *gb3 = gW3 + (int64_t)d * H2;
    memset(g, 0, sizeof(double) * (size_t)fsneo_mlp_nparams(m));
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
        for (int32_t k = 0; k < H2; ++k) {
            double s = 0.0;
            for (int32_t j = 0; j < d; ++j)
                s += 2.0 * (out[r * d + j] - (double)T[r * d + j]) / (double)(n * d) *
                     P.W3[(int64_t)j * H2 + k];
            dh2[r * H2 + k] = h2[r * H2 + k] > 0.0 ? s : 0.0;
        }
    }
    for (int32_t j = 0; j < d; ++j) {
        for (int64_t r = 0; r < n; ++r) {
            double go = 2.0 * (out[r * d + j] - (double)T[r * d + j]) / (double)(n * d);
            gb3[j] += go;
            for (int32_t k = 0; k < H2; ++k) gW3[(int64_t)j * H2 + k] += go * h2[r * H2 + k];
        }
    }
    /* second hidden layer */
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < H2; ++j) {
        for (int64_t r = 0; r < n; ++r) {
            double gz = op(dh2[r * H2 + j], bf);
            gb2[j] += dh2[r * H2 + j];
            for (int32_t k = 0; k < H1; ++k) gW2[(int64_t)j * H1 + k] += gz * op(h1[r * H1 + k], bf);
        }
    }
#pragma omp parallel for schedule(static)
    for (int64_t r = 0; r < n; ++r) {
        for (int32_t k = 0; k < H1; ++k) {
            double s = 0.0;
            for (int32_t j = 0; j < H2; ++j)
                s += op(dh2[r * H2 + j], bf) * op(P.W2[(int64_t)j * H1 + k], bf);
            dh1[r * H1 + k] = h1[r * H1 + k] > 0.0 ? s : 0.0;
        }
    }
    /* first hidden layer */
#pragma omp parallel for schedule(static)
    for (int32_t j = 0; j < H1; ++j) {
        for (int64_t r = 0; r < n; ++r) {
            double gz = op(dh1[r * H1 + j], bf);
            gb1[j] += dh1[r * H1 + j];
            for (int32_t k = 0; k < D; ++k)
                gW1[(int64_t)j * D + k] += gz * op(xin(X, xdtype, r * D + k), bf);
        }
    }
    free(h1);
    free(h2);
    free(out);
    free(dh2);
    free(dh1);
    return loss;
}

/* One Adam step (Kingma and Ba 2015) at step number t >= 1:                 */
/* m <- b1 m + (1-b1) g;  v <- b2 v + (1-b2) g^2;                            */
/* p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).              */
void fsneo_mlp_adam(int64_t np, float *p, double *mo, double *vo, const double *g, int64_t t,
                    double lr, double b1, double b2, double eps)
{
    double c1 = 1.0 - pow(b1, (double)t), c2 = 1.0 - pow(b2, (double)t);
    for (int64_t k = 0; k < np; ++k) {
        mo[k] = b1 * mo[k] + (1.0 - b1) * g[k];
        vo[k] = b2 * vo[k] + (1.0 - b2) * g[k] * g[k];
        double step = lr * (mo[k] / c1) / (sqrt(vo[k] / c2) + eps);
        p[k] = (float)((double)p[k] - step);
    }
}
