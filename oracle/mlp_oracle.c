/*
 * mlp_oracle.c -- plain FP64 reference of the closure network: a multilayer
 * perceptron 37 -> 64 -> 64 -> 64 -> 4 with tanh hidden layers and a linear
 * output, its mean-squared-error gradient by back-propagation, and one Adam
 * step.
 *
 * TEST INFRASTRUCTURE.  Only the test suite, the smoke check and the CPU
 * baseline of the benchmark may load this code; it shares nothing with the
 * GPU kernels.  The network is not part of the paper: it is the learned
 * closure of the throughput study, pinned here by finite differences.
 *
 * Parameter layout (flat, FP64): W1[64][37] b1[64] W2[64][64] b2[64]
 * W3[64][64] b3[64] W4[4][64] b4[4]; weights are row-major (output, input).
 * Loss L = (1/(4n)) sum_i sum_o (y_io - t_io)^2.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#define NIN 37
#define NH 64
#define NOUT 4
#define NPARAM (NH * NIN + NH + NH * NH + NH + NH * NH + NH + NOUT * NH + NOUT)

int mlp_nparam(void) { return NPARAM; }

typedef struct {
  const double *W[4], *b[4];
} layers_t;

static void split(const double *p, layers_t *L) {
  const int nin[4] = {NIN, NH, NH, NH}, nout[4] = {NH, NH, NH, NOUT};
  for (int l = 0; l < 4; ++l) {
    L->W[l] = p;
    p += nout[l] * nin[l];
    L->b[l] = p;
    p += nout[l];
  }
}

/* one sample: activations a0 (input), a1..a3 (hidden, after tanh), y */
static void forward1(const layers_t *L, const double *x, double *a1, double *a2,
                     double *a3, double *y) {
  const double *in[4] = {x, a1, a2, a3};
  double *out[4] = {a1, a2, a3, y};
  const int nin[4] = {NIN, NH, NH, NH}, nout[4] = {NH, NH, NH, NOUT};
  for (int l = 0; l < 4; ++l)
    for (int o = 0; o < nout[l]; ++o) {
      double z = L->b[l][o];
      for (int i = 0; i < nin[l]; ++i) z += L->W[l][o * nin[l] + i] * in[l][i];
      out[l][o] = (l < 3) ? tanh(z) : z;
    }
}

void mlp_forward(const double *p, const double *x, double *y, int n) {
  layers_t L;
  split(p, &L);
  double a1[NH], a2[NH], a3[NH];
  for (int s = 0; s < n; ++s) forward1(&L, x + (size_t)s * NIN, a1, a2, a3, y + (size_t)s * NOUT);
}

/* loss and its gradient with respect to every parameter (same layout) */
double mlp_loss_grad(const double *p, const double *x, const double *t, int n, double *g) {
  layers_t L;
  split(p, &L);
  memset(g, 0, sizeof(double) * NPARAM);
  layers_t G;
  split(g, &G);
  double loss = 0.0;
  double a1[NH], a2[NH], a3[NH], y[NOUT];
  double d4[NOUT], d3[NH], d2[NH], d1[NH];
  const double scale = 1.0 / (4.0 * n);
  for (int s = 0; s < n; ++s) {
    const double *xs = x + (size_t)s * NIN, *ts = t + (size_t)s * NOUT;
    forward1(&L, xs, a1, a2, a3, y);
    for (int o = 0; o < NOUT; ++o) {
      const double e = y[o] - ts[o];
      loss += e * e;
      d4[o] = 2.0 * e * scale; /* dL/dz4 */
    }
    const double *acts[4] = {xs, a1, a2, a3};
    double *dz[4] = {d1, d2, d3, d4};
    const int nin[4] = {NIN, NH, NH, NH}, nout[4] = {NH, NH, NH, NOUT};
    /* back-propagate: dL/da_{l} = W_l^T dz_l, dz_{l-1} = dL/da (1 - a^2) */
    for (int l = 3; l >= 0; --l) {
      double *gW = (double *)G.W[l], *gb = (double *)G.b[l];
      for (int o = 0; o < nout[l]; ++o) {
        gb[o] += dz[l][o];
        for (int i = 0; i < nin[l]; ++i) gW[o * nin[l] + i] += dz[l][o] * acts[l][i];
      }
      if (l > 0) {
        for (int i = 0; i < nin[l]; ++i) {
          double acc = 0.0;
          for (int o = 0; o < nout[l]; ++o) acc += L.W[l][o * nin[l] + i] * dz[l][o];
          dz[l - 1][i] = acc * (1.0 - acts[l][i] * acts[l][i]);
        }
      }
    }
  }
  return loss * scale;
}

/* Adam (Kingma & Ba) with bias correction; `step` counts from 1 */
void mlp_adam(double *p, const double *g, double *m, double *v, double lr, double b1,
              double b2, double eps, int step) {
  const double c1 = 1.0 - pow(b1, step), c2 = 1.0 - pow(b2, step);
  for (int i = 0; i < NPARAM; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    p[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
  }
}
