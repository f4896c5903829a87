/*
 * mlp_oracle.c -- TEST INFRASTRUCTURE ONLY (the oracle of the learned
 * Riemann initial guess).
 *
 * A plain FP64 implementation of the small network that proposes the starting
 * point of the interface Riemann solver's Newton iteration: a fully connected
 * network 14 -> 64 -> 64 -> 2 with the tanh form of the GELU activation
 * (Hendrycks & Gimpel 2016: gelu(x) = x/2 (1 + tanh(sqrt(2/pi)(x + 0.044715 x^3)))),
 * mean-squared-error loss, its gradient by the chain rule, and one Adam step
 * (Kingma & Ba 2015).  Only the test suite may load this library; it shares
 * no code with the GPU kernels.
 *
 * Layout (row-major, one sample per row):
 *   X [n][14], W1 [14][64], b1 [64], W2 [64][64], b2 [64], W3 [64][2], b3 [2]
 *   parameters packed in that order into one vector theta (5250 values).
 * Pins: central finite differences of the loss (tests), gelu special values.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NIN 14
#define NH 64
#define NOUT 2
#define NPAR (NIN * NH + NH + NH * NH + NH + NH * NOUT + NOUT)

static const double kC = 0.7978845608028654;   /* sqrt(2/pi) */
static const double kA = 0.044715;

double mlp_gelu(double x)
{
    return 0.5 * x * (1.0 + tanh(kC * (x + kA * x * x * x)));
}

/* derivative of the tanh-form GELU */
double mlp_gelu_grad(double x)
{
    double u = kC * (x + kA * x * x * x);
    double t = tanh(u);
    double du = kC * (1.0 + 3.0 * kA * x * x);
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * du;
}

int mlp_num_params(void) { return NPAR; }

static void unpack(const double *th, const double **W1, const double **b1, const double **W2,
                   const double **b2, const double **W3, const double **b3)
{
    *W1 = th;
    *b1 = *W1 + NIN * NH;
    *W2 = *b1 + NH;
    *b2 = *W2 + NH * NH;
    *W3 = *b2 + NH;
    *b3 = *W3 + NH * NOUT;
}

/* Forward pass for n samples: out [n][2]; optional caches of the hidden
 * pre-activations z1, z2 [n][64]. */
void mlp_forward(const double *theta, int n, const double *X, double *out, double *z1c, double *z2c)
{
    const double *W1, *b1, *W2, *b2, *W3, *b3;
    unpack(theta, &W1, &b1, &W2, &b2, &W3, &b3);
    double z1[NH], h1[NH], z2[NH], h2[NH];
    for (int s = 0; s < n; ++s) {
        const double *x = X + (size_t)s * NIN;
        for (int j = 0; j < NH; ++j) {
            double a = b1[j];
            for (int i = 0; i < NIN; ++i) a += x[i] * W1[i * NH + j];
            z1[j] = a;
            h1[j] = mlp_gelu(a);
        }
        for (int j = 0; j < NH; ++j) {
            double a = b2[j];
            for (int i = 0; i < NH; ++i) a += h1[i] * W2[i * NH + j];
            z2[j] = a;
            h2[j] = mlp_gelu(a);
        }
        for (int k = 0; k < NOUT; ++k) {
            double a = b3[k];
            for (int i = 0; i < NH; ++i) a += h2[i] * W3[i * NOUT + k];
            out[(size_t)s * NOUT + k] = a;
        }
        if (z1c) memcpy(z1c + (size_t)s * NH, z1, sizeof(z1));
        if (z2c) memcpy(z2c + (size_t)s * NH, z2, sizeof(z2));
    }
}

/* Loss L = (1 / (2 n)) sum_s sum_k (out_sk - Y_sk)^2 over n samples and its
 * gradient with respect to every parameter (grad, NPAR values; NULL = loss
 * only).  Returns L. */
double mlp_loss_grad(const double *theta, int n, const double *X, const double *Y, double *grad)
{
    const double *W1, *b1, *W2, *b2, *W3, *b3;
    unpack(theta, &W1, &b1, &W2, &b2, &W3, &b3);
    double *g = grad;
    double *gW1 = g, *gb1 = gW1 + NIN * NH, *gW2 = gb1 + NH, *gb2 = gW2 + NH * NH;
    double *gW3 = gb2 + NH, *gb3 = gW3 + NH * NOUT;
    if (g) memset(g, 0, sizeof(double) * NPAR);
    double loss = 0.0;
    double z1[NH], h1[NH], z2[NH], h2[NH], o[NOUT];
    double d3[NOUT], d2[NH], d1[NH];
    for (int s = 0; s < n; ++s) {
        const double *x = X + (size_t)s * NIN;
        for (int j = 0; j < NH; ++j) {
            double a = b1[j];
            for (int i = 0; i < NIN; ++i) a += x[i] * W1[i * NH + j];
            z1[j] = a;
            h1[j] = mlp_gelu(a);
        }
        for (int j = 0; j < NH; ++j) {
            double a = b2[j];
            for (int i = 0; i < NH; ++i) a += h1[i] * W2[i * NH + j];
            z2[j] = a;
            h2[j] = mlp_gelu(a);
        }
        for (int k = 0; k < NOUT; ++k) {
            double a = b3[k];
            for (int i = 0; i < NH; ++i) a += h2[i] * W3[i * NOUT + k];
            o[k] = a;
            double r = a - Y[(size_t)s * NOUT + k];
            loss += 0.5 * r * r;
            d3[k] = r / n;
        }
        if (!g) continue;
        /* output layer */
        for (int k = 0; k < NOUT; ++k) {
            gb3[k] += d3[k];
            for (int i = 0; i < NH; ++i) gW3[i * NOUT + k] += h2[i] * d3[k];
        }
        /* second hidden layer */
        for (int i = 0; i < NH; ++i) {
            double a = 0.0;
            for (int k = 0; k < NOUT; ++k) a += W3[i * NOUT + k] * d3[k];
            d2[i] = a * mlp_gelu_grad(z2[i]);
        }
        for (int j = 0; j < NH; ++j) {
            gb2[j] += d2[j];
            for (int i = 0; i < NH; ++i) gW2[i * NH + j] += h1[i] * d2[j];
        }
        /* first hidden layer */
        for (int i = 0; i < NH; ++i) {
            double a = 0.0;
            for (int j = 0; j < NH; ++j) a += W2[i * NH + j] * d2[j];
            d1[i] = a * mlp_gelu_grad(z1[i]);
        }
        for (int j = 0; j < NH; ++j) {
            gb1[j] += d1[j];
            for (int i = 0; i < NIN; ++i) gW1[i * NH + j] += x[i] * d1[j];
        }
    }
    return loss / n;
}

/* One Adam step (bias-corrected, step number t >= 1) on theta with moments
 * m and v, all NPAR values. */
void mlp_adam(double *theta, double *m, double *v, const double *grad, int t, double lr, double b1,
              double b2, double eps)
{
    double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    for (int i = 0; i < NPAR; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * grad[i];
        v[i] = b2 * v[i] + (1.0 - b2) * grad[i] * grad[i];
        double mh = m[i] / c1, vh = v[i] / c2;
        theta[i] -= lr * mh / (sqrt(vh) + eps);
    }
}
