/*
 * FP64 reference of the learned Ewald surrogate (a small MLP standing in for
 * the Ewald correction table).  TEST INFRASTRUCTURE ONLY (see octoracle.h).
 *
 * Network: 3 -> 64 -> 64 -> 64 -> 10, the gated activation f(z) = z S(z)
 * after the three hidden layers, identity output.  S is the cubic smoothstep
 * rising from 0 at z = -3 to 1 at z = 3: S = t^2 (3 - 2t), t = clamp(z/6 + 1/2,
 * 0, 1).  f is continuously differentiable, close to z sigma(z) (same slope at
 * 0), and costs no exponential or reciprocal.  The ten outputs are the Ewald
 * table's channels: phi_c, A_c (3) and the six second derivatives of phi_c.
 * Parameter vector layout (9226 values):
 *   W1[64][3], b1[64], W2[64][64], b2[64], W3[64][64], b3[64], W4[10][64], b4[10]
 * (row-major, W[out][in]).  Loss over a batch of B samples: mean squared error
 * over the 10 outputs, L = 1/(10B) sum_s sum_o (y_so - t_so)^2.
 * Plain loops, no blocking; the gradient is the textbook back-propagation.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { H = 64, NI = 3, NO = 10 };
enum { OW1 = 0, OB1 = OW1 + H * NI, OW2 = OB1 + H, OB2 = OW2 + H * H, OW3 = OB2 + H,
       OB3 = OW3 + H * H, OW4 = OB3 + H, OB4 = OW4 + NO * H, NPARAM = OB4 + NO };

static double gate_t(double z) {
  double t = z / 6.0 + 0.5;
  return t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
}
static double act(double z) {
  double t = gate_t(z);
  return z * t * t * (3.0 - 2.0 * t);
}
/* f'(z) = S + z S'(z), S'(z) = t (1 - t) (zero outside [-3, 3]) */
static double dact(double z) {
  double t = gate_t(z);
  return t * t * (3.0 - 2.0 * t) + z * t * (1.0 - t);
}

int or_mlp_nparam(void) { return NPARAM; }

/* forward of one sample; keeps pre-activations for the backward pass */
static void forward1(const double *p, const double *x, double z1[H], double z2[H], double z3[H],
                     double y[NO]) {
  double h1[H], h2[H], h3[H];
  for (int o = 0; o < H; ++o) {
    double a = p[OB1 + o];
    for (int i = 0; i < NI; ++i) a += p[OW1 + o * NI + i] * x[i];
    z1[o] = a;
    h1[o] = act(a);
  }
  for (int o = 0; o < H; ++o) {
    double a = p[OB2 + o];
    for (int i = 0; i < H; ++i) a += p[OW2 + o * H + i] * h1[i];
    z2[o] = a;
    h2[o] = act(a);
  }
  for (int o = 0; o < H; ++o) {
    double a = p[OB3 + o];
    for (int i = 0; i < H; ++i) a += p[OW3 + o * H + i] * h2[i];
    z3[o] = a;
    h3[o] = act(a);
  }
  for (int o = 0; o < NO; ++o) {
    double a = p[OB4 + o];
    for (int i = 0; i < H; ++i) a += p[OW4 + o * H + i] * h3[i];
    y[o] = a;
  }
}

/* y[B][10] = f(x[B][3]) */
void or_mlp_forward(const double *p, int64_t B, const double *x, double *y) {
  for (int64_t s = 0; s < B; ++s) {
    double z1[H], z2[H], z3[H];
    forward1(p, x + NI * s, z1, z2, z3, y + NO * s);
  }
}

/* loss and gradient g[NPARAM] of the batch MSE */
double or_mlp_grad(const double *p, int64_t B, const double *x, const double *t, double *g) {
  memset(g, 0, sizeof(double) * NPARAM);
  double loss = 0.0;
  const double scale = 1.0 / (double)(NO * B);
  for (int64_t s = 0; s < B; ++s) {
    const double *xs = x + NI * s;
    double z1[H], z2[H], z3[H], y[NO];
    forward1(p, xs, z1, z2, z3, y);
    double h1[H], h2[H], h3[H];
    for (int i = 0; i < H; ++i) {
      h1[i] = act(z1[i]);
      h2[i] = act(z2[i]);
      h3[i] = act(z3[i]);
    }
    double dy[NO];
    for (int o = 0; o < NO; ++o) {
      double e = y[o] - t[NO * s + o];
      loss += e * e * scale;
      dy[o] = 2.0 * e * scale;
    }
    /* layer 4 */
    double dh3[H] = {0};
    for (int o = 0; o < NO; ++o) {
      g[OB4 + o] += dy[o];
      for (int i = 0; i < H; ++i) {
        g[OW4 + o * H + i] += dy[o] * h3[i];
        dh3[i] += dy[o] * p[OW4 + o * H + i];
      }
    }
    /* layer 3 */
    double dh2[H] = {0};
    for (int o = 0; o < H; ++o) {
      double dz = dh3[o] * dact(z3[o]);
      g[OB3 + o] += dz;
      for (int i = 0; i < H; ++i) {
        g[OW3 + o * H + i] += dz * h2[i];
        dh2[i] += dz * p[OW3 + o * H + i];
      }
    }
    /* layer 2 */
    double dh1[H] = {0};
    for (int o = 0; o < H; ++o) {
      double dz = dh2[o] * dact(z2[o]);
      g[OB2 + o] += dz;
      for (int i = 0; i < H; ++i) {
        g[OW2 + o * H + i] += dz * h1[i];
        dh1[i] += dz * p[OW2 + o * H + i];
      }
    }
    /* layer 1 */
    for (int o = 0; o < H; ++o) {
      double dz = dh1[o] * dact(z1[o]);
      g[OB1 + o] += dz;
      for (int i = 0; i < NI; ++i) g[OW1 + o * NI + i] += dz * xs[i];
    }
  }
  return loss;
}

/* One step of Adam (Kingma & Ba 2015, Algorithm 1) on n parameters p with the
 * gradient g: first and second moment estimates m, v with decay rates
 * beta1 = 0.9, beta2 = 0.999, bias corrections 1 - beta^step (step >= 1),
 * step size lr and eps = 1e-8 added to the root of the corrected second
 * moment.  m and v are updated in place. */
void or_adam_update(double *p, const double *g, double *m, double *v, int64_t n, double lr, int64_t step) {
  const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
  const double c1 = 1.0 - pow(b1, (double)step), c2 = 1.0 - pow(b2, (double)step);
  for (int64_t i = 0; i < n; ++i) {
    m[i] = b1 * m[i] + (1.0 - b1) * g[i];
    v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
    const double mhat = m[i] / c1, vhat = v[i] / c2;
    p[i] = p[i] - lr * mhat / (sqrt(vhat) + eps);
  }
}

/* The training step: the batch gradient of the MSE, then one Adam step;
 * returns the batch loss before the step. */
double or_mlp_adam(double *p, double *m, double *v, int64_t B, const double *x, const double *t, double lr,
                   int64_t step) {
  double *g = (double *)malloc(sizeof(double) * NPARAM);
  const double loss = or_mlp_grad(p, B, x, t, g);
  or_adam_update(p, g, m, v, NPARAM, lr, step);
  free(g);
  return loss;
}
