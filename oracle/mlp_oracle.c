/*
 * mlp_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * FP64 reference for the small network that chooses the restart stride.  The
 * paper leaves the stride a free parameter (Sec. 2.4, Sec. 3.1); the network
 * is this project's addition and has no passage in the paper to follow, so
 * this file states plain calculus: a 12-32-32-1 perceptron with ReLU hidden
 * layers, a sigmoid-squashed output mapped to log m in [ln 1/4, ln 8], the
 * mean-squared error on log m, its gradient by the chain rule, and one Adam
 * step (Kingma & Ba, 2015).  Shares no code with the HIP kernels.
 *
 * Parameter vector (1505 doubles), row-major, out x in:
 *   W1[32][12], b1[32], W2[32][32], b2[32], W3[1][32], b3[1]
 * Inputs are already standardised features x[n][12].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NI 12
#define NH 32
#define NP (NH * NI + NH + NH * NH + NH + NH + 1)

static const double LOG_MIN = -1.3862943611198906; /* ln(1/4)            */
static const double LOG_SPAN = 3.4657359027997265; /* ln(8) - ln(1/4)     */

int orc_mlp_nparams(void) { return NP; }

/* forward pass of one sample; keeps the activations for the backward pass */
static double forward1(const double *P, const double *x, double *h1, double *h2, double *zout)
{
    const double *W1 = P, *b1 = W1 + NH * NI, *W2 = b1 + NH, *b2 = W2 + NH * NH, *W3 = b2 + NH,
                 *b3 = W3 + NH;
    for (int o = 0; o < NH; ++o) {
        double s = b1[o];
        for (int i = 0; i < NI; ++i) s += W1[o * NI + i] * x[i];
        h1[o] = s > 0 ? s : 0;
    }
    for (int o = 0; o < NH; ++o) {
        double s = b2[o];
        for (int i = 0; i < NH; ++i) s += W2[o * NH + i] * h1[i];
        h2[o] = s > 0 ? s : 0;
    }
    double z = b3[0];
    for (int i = 0; i < NH; ++i) z += W3[i] * h2[i];
    *zout = z;
    double sig = 1.0 / (1.0 + exp(-z));
    return LOG_MIN + LOG_SPAN * sig; /* predicted log of the stride multiplier */
}

/* y[s] = predicted log multiplier of sample s */
int orc_mlp_forward(const double *P, const double *X, int64_t n, double *y)
{
    double h1[NH], h2[NH], z;
    for (int64_t s = 0; s < n; ++s) y[s] = forward1(P, X + s * NI, h1, h2, &z);
    return 0;
}

/* loss = (1/n) sum_s (y_s - t_s)^2 and its gradient with respect to P */
int orc_mlp_loss_grad(const double *P, const double *X, const double *T, int64_t n,
                      double *loss, double *grad)
{
    if (n <= 0) return -1;
    const double *W2 = P + NH * NI + NH, *W3 = W2 + NH * NH + NH;
    double *gW1 = grad, *gb1 = gW1 + NH * NI, *gW2 = gb1 + NH, *gb2 = gW2 + NH * NH,
           *gW3 = gb2 + NH, *gb3 = gW3 + NH;
    memset(grad, 0, NP * sizeof(double));
    double L = 0;
    for (int64_t s = 0; s < n; ++s) {
        const double *x = X + s * NI;
        double h1[NH], h2[NH], z;
        double y = forward1(P, x, h1, h2, &z);
        double e = y - T[s];
        L += e * e;
        double sig = 1.0 / (1.0 + exp(-z));
        double dz = (2.0 * e / (double)n) * LOG_SPAN * sig * (1.0 - sig);
        double dh2[NH], dh1[NH];
        gb3[0] += dz;
        for (int i = 0; i < NH; ++i) {
            gW3[i] += dz * h2[i];
            dh2[i] = (h2[i] > 0) ? dz * W3[i] : 0;
        }
        for (int i = 0; i < NH; ++i) dh1[i] = 0;
        for (int o = 0; o < NH; ++o) {
            gb2[o] += dh2[o];
            for (int i = 0; i < NH; ++i) {
                gW2[o * NH + i] += dh2[o] * h1[i];
                dh1[i] += dh2[o] * W2[o * NH + i];
            }
        }
        for (int o = 0; o < NH; ++o) {
            double d = (h1[o] > 0) ? dh1[o] : 0;
            gb1[o] += d;
            for (int i = 0; i < NI; ++i) gW1[o * NI + i] += d * x[i];
        }
    }
    *loss = L / (double)n;
    return 0;
}

/* One Adam step at iteration t >= 1 (Kingma & Ba, 2015, Algorithm 1). */
int orc_adam_step(double *P, const double *g, double *m, double *v, int64_t np, double lr,
                  double beta1, double beta2, double eps, int64_t t)
{
    if (t < 1) return -1;
    const double c1 = 1.0 - pow(beta1, (double)t), c2 = 1.0 - pow(beta2, (double)t);
    for (int64_t i = 0; i < np; ++i) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
        double mh = m[i] / c1, vh = v[i] / c2;
        P[i] -= lr * mh / (sqrt(vh) + eps);
    }
    return 0;
}
