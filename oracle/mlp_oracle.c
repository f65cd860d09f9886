/*
 * mlp_oracle.c -- TEST INFRASTRUCTURE: FP64 reference of the small network
 * that predicts the starting point of the per-cell root solve (the learned
 * guess; not part of the paper's method, which only says the root solve takes
 * a variable number of iterations, App. A.3).
 *
 * Network (4 -> 32 -> 32 -> 1, tanh hidden layers):
 *   inputs  f = (ln E / 5, M/E, (M/E)^2, ln(max(lo/E, 1e-30)) / 10)
 *           with E = K^tau, M = |K|, lo = max(0, E - M^2/E) (the root solve's
 *           lower bracket end; the root lies in [lo, E]);
 *   h1 = tanh(W1 f + b1), h2 = tanh(W2 h1 + b2), z = w3 . h2 + b3;
 *   guess = lo + sigmoid(z) (E - lo), always inside the bracket.
 * Loss over a batch of (E, M, e) with target e: mean of ((guess - e)/E)^2.
 * Parameters, flat: W1[32][4], b1[32], W2[32][32], b2[32], w3[32], b3.
 * Adam: Kingma & Ba (2015), bias-corrected first and second moments.
 *
 * Only the test suite loads this; it shares no code with the HIP library.
 */
#include <math.h>
#include <string.h>

#define NH 32
#define NPARAM (NH * 4 + NH + NH * NH + NH + NH + 1)

static void features(double E, double M, double f[4], double *lo_out) {
    double r = M / E;
    double lo = E - M * M / E;
    if (lo < 0.0) lo = 0.0;
    double q = lo / E;
    if (q < 1e-30) q = 1e-30;
    f[0] = log(E) / 5.0;
    f[1] = r;
    f[2] = r * r;
    f[3] = log(q) / 10.0;
    *lo_out = lo;
}

/* Forward pass of one sample; keeps the activations for the backward pass. */
static double forward(const double *p, const double f[4], double h1[NH], double h2[NH]) {
    const double *W1 = p, *b1 = p + NH * 4, *W2 = b1 + NH, *b2 = W2 + NH * NH, *w3 = b2 + NH;
    const double b3 = w3[NH];
    for (int j = 0; j < NH; ++j) {
        double a = b1[j];
        for (int k = 0; k < 4; ++k) a += W1[j * 4 + k] * f[k];
        h1[j] = tanh(a);
    }
    for (int i = 0; i < NH; ++i) {
        double a = b2[i];
        for (int j = 0; j < NH; ++j) a += W2[i * NH + j] * h1[j];
        h2[i] = tanh(a);
    }
    double z = b3;
    for (int i = 0; i < NH; ++i) z += w3[i] * h2[i];
    return z;
}

int orc_mlp_nparam(void) { return NPARAM; }

/* guess[i] for n samples (E, M). */
int orc_mlp_forward(const double *p, int n, const double *E, const double *M, double *guess) {
    for (int s = 0; s < n; ++s) {
        double f[4], lo, h1[NH], h2[NH];
        features(E[s], M[s], f, &lo);
        double z = forward(p, f, h1, h2);
        double sg = 1.0 / (1.0 + exp(-z));
        guess[s] = lo + sg * (E[s] - lo);
    }
    return 0;
}

/* Mean loss and its gradient with respect to every parameter. */
int orc_mlp_loss_grad(const double *p, int n, const double *E, const double *M,
                      const double *eps, double *loss, double *grad) {
    const double *W2 = p + NH * 4 + NH, *w3 = W2 + NH * NH + NH;
    double *gW1 = grad, *gb1 = grad + NH * 4, *gW2 = gb1 + NH, *gb2 = gW2 + NH * NH,
           *gw3 = gb2 + NH;
    memset(grad, 0, sizeof(double) * NPARAM);
    double L = 0.0;
    for (int s = 0; s < n; ++s) {
        double f[4], lo, h1[NH], h2[NH];
        features(E[s], M[s], f, &lo);
        double z = forward(p, f, h1, h2);
        double sg = 1.0 / (1.0 + exp(-z));
        double r = (E[s] - lo) / E[s];          /* guess - e = (sg - t)(E - lo) */
        double t = (E[s] > lo) ? (eps[s] - lo) / (E[s] - lo) : 0.0;
        double d = r * (sg - t);
        L += d * d;
        double dz = 2.0 * d * r * sg * (1.0 - sg) / n;
        double d2[NH], d1[NH];
        for (int i = 0; i < NH; ++i) {
            gw3[i] += dz * h2[i];
            d2[i] = dz * w3[i] * (1.0 - h2[i] * h2[i]);
            gb2[i] += d2[i];
            for (int j = 0; j < NH; ++j) gW2[i * NH + j] += d2[i] * h1[j];
        }
        gw3[NH] += dz;
        for (int j = 0; j < NH; ++j) {
            double a = 0.0;
            for (int i = 0; i < NH; ++i) a += W2[i * NH + j] * d2[i];
            d1[j] = a * (1.0 - h1[j] * h1[j]);
            gb1[j] += d1[j];
            for (int k = 0; k < 4; ++k) gW1[j * 4 + k] += d1[j] * f[k];
        }
    }
    *loss = L / n;
    return 0;
}

/* One Adam step (t counts from 1). */
int orc_mlp_adam(double *p, const double *g, double *m, double *v, int t, double lr,
                 double b1, double b2, double epsilon) {
    double c1 = 1.0 - pow(b1, t), c2 = 1.0 - pow(b2, t);
    for (int k = 0; k < NPARAM; ++k) {
        m[k] = b1 * m[k] + (1.0 - b1) * g[k];
        v[k] = b2 * v[k] + (1.0 - b2) * g[k] * g[k];
        double mh = m[k] / c1, vh = v[k] / c2;
        p[k] -= lr * mh / (sqrt(vh) + epsilon);
    }
    return 0;
}
