/* Oracle of the learned Poisson initial guess (see cnn_oracle.h).
 * TEST INFRASTRUCTURE ONLY: serial FP64, written for reading, not speed.
 * Every sum is a plain loop; gradients are formed by scattering each term
 * of the forward sums (the chain rule term by term). */
#include "cnn_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static const int COUT[OCNN_LAYERS] = {16, 16, 16, 1};

static int inputs_ok(int inputs) { return inputs == 1 || inputs == 3; }
int ocnn_cin(int inputs, int l) {
  if (!inputs_ok(inputs) || l < 0 || l >= OCNN_LAYERS) return -1;
  return l == 0 ? inputs : COUT[l - 1];
}
int ocnn_cout(int l) { return l >= 0 && l < OCNN_LAYERS ? COUT[l] : -1; }

int ocnn_weight_offset(int inputs, int l) {
  if (!inputs_ok(inputs) || l < 0 || l > OCNN_LAYERS) return -1;
  int off = 0;
  for (int q = 0; q < l; ++q) off += OCNN_TAPS * ocnn_cin(inputs, q) * COUT[q] + COUT[q];
  return off;
}
int ocnn_bias_offset(int inputs, int l) {
  if (!inputs_ok(inputs) || l < 0 || l >= OCNN_LAYERS) return -1;
  return ocnn_weight_offset(inputs, l) + OCNN_TAPS * ocnn_cin(inputs, l) * COUT[l];
}
int ocnn_param_count(int inputs) { return ocnn_weight_offset(inputs, OCNN_LAYERS); }

void ocnn_layer_size(const ocnn_dims *d, int l, int *ny, int *nx) {
  int trim = d->periodic ? 0 : 2 * l;
  *ny = d->ny - trim;
  *nx = d->nx - trim;
}

/* bfloat16: 8 significant bits, exponent range of FP32 (normal numbers from
 * 2^-126, subnormal spacing 2^-133, largest finite (2 - 2^-7) 2^127). */
double ocnn_bf16(double v) {
  if (v == 0.0 || !isfinite(v)) return v;
  if (fabs(v) < ldexp(1.0, -126)) return ldexp(nearbyint(ldexp(v, 133)), -133);
  int e;
  double m = frexp(v, &e);            /* |m| in [0.5, 1) */
  double r = ldexp(nearbyint(ldexp(m, 8)), e - 8);  /* ties to even */
  if (fabs(r) > ldexp(2.0 - ldexp(1.0, -7), 127)) return v > 0 ? INFINITY : -INFINITY;
  return r;
}

static int check_dims(const ocnn_dims *d) {
  if (!d || d->batch < 1 || d->nz < 1 || d->alpha < 0.0 || !inputs_ok(d->inputs) || d->reserved)
    return -1;
  int ny, nx;
  ocnn_layer_size(d, OCNN_LAYERS, &ny, &nx);
  return ny >= 1 && nx >= 1 ? 0 : -1;
}

static int zmirror(int k, int nz) { return k < 0 ? -k - 1 : k >= nz ? 2 * nz - k - 1 : k; }
static int wrap(int i, int n) { return ((i % n) + n) % n; }

/* Index of the input cell read by output (k, j, i) at tap (dz, dy, dx). */
static size_t src_index(const ocnn_dims *d, int nyi, int nxi, int k, int j, int i, int dz, int dy,
                        int dx) {
  int kk = zmirror(k + dz, d->nz);
  int jj = d->periodic ? wrap(j + dy, nyi) : j + 1 + dy;
  int ii = d->periodic ? wrap(i + dx, nxi) : i + 1 + dx;
  return ((size_t)kk * nyi + jj) * nxi + ii;
}

static double *rounded_weights(const ocnn_dims *d, const double *params, int l) {
  int nw = OCNN_TAPS * ocnn_cin(d->inputs, l) * COUT[l];
  double *w = malloc(nw * sizeof(double));
  if (!w) return NULL;
  const double *src = params + ocnn_weight_offset(d->inputs, l);
  for (int q = 0; q < nw; ++q) w[q] = d->bf16 ? ocnn_bf16(src[q]) : src[q];
  return w;
}

/* y[b][o][cell] = bias[o] + sum_tap sum_i W[tap][o][i] a[b][i][src(cell, tap)] */
static int conv_layer(const ocnn_dims *d, int l, const double *params, const double *a, double *y) {
  int nyi, nxi, nyo, nxo;
  ocnn_layer_size(d, l, &nyi, &nxi);
  ocnn_layer_size(d, l + 1, &nyo, &nxo);
  const int ci = ocnn_cin(d->inputs, l), co = COUT[l];
  const size_t ni = (size_t)d->nz * nyi * nxi, no = (size_t)d->nz * nyo * nxo;
  double *w = rounded_weights(d, params, l);
  if (!w) return -1;
  const double *bias = params + ocnn_bias_offset(d->inputs, l);
  for (int b = 0; b < d->batch; ++b)
    for (int o = 0; o < co; ++o)
      for (int k = 0; k < d->nz; ++k)
        for (int j = 0; j < nyo; ++j)
          for (int i = 0; i < nxo; ++i) {
            double s = bias[o];
            for (int dz = -1; dz <= 1; ++dz)
              for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                  int tap = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1);
                  size_t src = src_index(d, nyi, nxi, k, j, i, dz, dy, dx);
                  for (int c = 0; c < ci; ++c)
                    s += w[(tap * co + o) * ci + c] * a[((size_t)b * ci + c) * ni + src];
                }
            y[((size_t)b * co + o) * no + ((size_t)k * nyo + j) * nxo + i] = s;
          }
  free(w);
  return 0;
}

static size_t act_len(const ocnn_dims *d, int l, int channels) {
  int ny, nx;
  ocnn_layer_size(d, l, &ny, &nx);
  return (size_t)d->batch * channels * d->nz * ny * nx;
}

int ocnn_forward(const ocnn_dims *d, const double *params, const double *x, double *out,
                 double *const *acts, double *const *pre) {
  if (check_dims(d) || !params || !x || !out) return -1;
  double *a[OCNN_LAYERS] = {0}, *y[OCNN_LAYERS] = {0};
  int rc = 0;
  for (int l = 0; l < OCNN_LAYERS && rc == 0; ++l) {
    a[l] = acts ? acts[l] : malloc(act_len(d, l, ocnn_cin(d->inputs, l)) * sizeof(double));
    y[l] = l == OCNN_LAYERS - 1 ? out
           : pre                ? pre[l]
                                : malloc(act_len(d, l + 1, COUT[l]) * sizeof(double));
    if (!a[l] || !y[l]) rc = -1;
  }
  if (rc == 0) {
    size_t n0 = act_len(d, 0, d->inputs);
    for (size_t q = 0; q < n0; ++q) a[0][q] = d->bf16 ? ocnn_bf16(x[q]) : x[q];
    for (int l = 0; l < OCNN_LAYERS; ++l) {
      if ((rc = conv_layer(d, l, params, a[l], y[l]))) break;
      if (l == OCNN_LAYERS - 1) break;
      size_t n = act_len(d, l + 1, COUT[l]);
      for (size_t q = 0; q < n; ++q) {
        double v = y[l][q] >= 0.0 ? y[l][q] : d->alpha * y[l][q];
        a[l + 1][q] = d->bf16 ? ocnn_bf16(v) : v;
      }
    }
  }
  for (int l = 0; l < OCNN_LAYERS; ++l) {
    if (!acts) free(a[l]);
    if (!pre && l < OCNN_LAYERS - 1) free(y[l]);
  }
  return rc;
}

int ocnn_backward(const ocnn_dims *d, const double *params, double *const *acts,
                  double *const *pre, const double *gout, double *grad) {
  if (check_dims(d) || !params || !acts || !pre || !gout || !grad) return -1;
  memset(grad, 0, (size_t)ocnn_param_count(d->inputs) * sizeof(double));
  /* gy: gradient with respect to the current layer's output (pre-activation) */
  double *gy = malloc(act_len(d, OCNN_LAYERS, 1) * sizeof(double));
  if (!gy) return -1;
  memcpy(gy, gout, act_len(d, OCNN_LAYERS, 1) * sizeof(double));
  for (int l = OCNN_LAYERS - 1; l >= 0; --l) {
    int nyi, nxi, nyo, nxo;
    ocnn_layer_size(d, l, &nyi, &nxi);
    ocnn_layer_size(d, l + 1, &nyo, &nxo);
    const int ci = ocnn_cin(d->inputs, l), co = COUT[l];
    const size_t ni = (size_t)d->nz * nyi * nxi, no = (size_t)d->nz * nyo * nxo;
    double *w = rounded_weights(d, params, l);
    double *ga = l > 0 ? calloc(act_len(d, l, ci), sizeof(double)) : NULL;
    if (!w || (l > 0 && !ga)) { free(w); free(ga); free(gy); return -1; }
    double *gw = grad + ocnn_weight_offset(d->inputs, l), *gb = grad + ocnn_bias_offset(d->inputs, l);
    const double *a = acts[l];
    for (int b = 0; b < d->batch; ++b)
      for (int o = 0; o < co; ++o)
        for (int k = 0; k < d->nz; ++k)
          for (int j = 0; j < nyo; ++j)
            for (int i = 0; i < nxo; ++i) {
              double g = gy[((size_t)b * co + o) * no + ((size_t)k * nyo + j) * nxo + i];
              gb[o] += g;
              for (int dz = -1; dz <= 1; ++dz)
                for (int dy = -1; dy <= 1; ++dy)
                  for (int dx = -1; dx <= 1; ++dx) {
                    int tap = 9 * (dz + 1) + 3 * (dy + 1) + (dx + 1);
                    size_t src = src_index(d, nyi, nxi, k, j, i, dz, dy, dx);
                    for (int c = 0; c < ci; ++c) {
                      size_t qa = ((size_t)b * ci + c) * ni + src;
                      gw[(tap * co + o) * ci + c] += g * a[qa];
                      if (ga) ga[qa] += g * w[(tap * co + o) * ci + c];
                    }
                  }
            }
    free(w);
    free(gy);
    gy = NULL;
    if (l > 0) {
      /* through the leaky ReLU of layer l-1 */
      size_t n = act_len(d, l, ci);
      for (size_t q = 0; q < n; ++q)
        if (pre[l - 1][q] < 0.0) ga[q] *= d->alpha;
      gy = ga;
    }
  }
  return 0;
}

int ocnn_loss(int32_t batch, int32_t nz, int32_t ny, int32_t nx, double dx, double dy, double dz,
              const double *y, const double *t, double *loss, double *gy) {
  if (batch < 1 || nz < 1 || ny < 3 || nx < 3 || !y || !t || !loss) return -1;
  const double d = 2.0 / (dx * dx) + 2.0 / (dy * dy) + 2.0 / (dz * dz);
  const double w[3] = {1.0 / (dx * dx * d), 1.0 / (dy * dy * d), 1.0 / (dz * dz * d)};
  const size_t n = (size_t)nz * ny * nx;
  double num = 0.0, den = 0.0;
  double *q = calloc((size_t)batch * n, sizeof(double));
  if (!q) return -1;
  /* Lh f at an interior cell; field f of one batch item */
#define LH(f, k, j, i)                                                                          \
  (w[0] * ((f)[((size_t)(k)*ny + (j)) * nx + (i) + 1] + (f)[((size_t)(k)*ny + (j)) * nx + (i)-1] -   \
           2.0 * (f)[((size_t)(k)*ny + (j)) * nx + (i)]) +                                      \
   w[1] * ((f)[((size_t)(k)*ny + (j) + 1) * nx + (i)] + (f)[((size_t)(k)*ny + (j)-1) * nx + (i)] -   \
           2.0 * (f)[((size_t)(k)*ny + (j)) * nx + (i)]) +                                      \
   w[2] * ((f)[((size_t)zmirror((k) + 1, nz) * ny + (j)) * nx + (i)] +                          \
           (f)[((size_t)zmirror((k)-1, nz) * ny + (j)) * nx + (i)] -                            \
           2.0 * (f)[((size_t)(k)*ny + (j)) * nx + (i)]))
  double *e = malloc(n * sizeof(double));
  if (!e) { free(q); return -1; }
  for (int b = 0; b < batch; ++b) {
    const double *yb = y + (size_t)b * n, *tb = t + (size_t)b * n;
    for (size_t c = 0; c < n; ++c) e[c] = yb[c] - tb[c];
    for (int k = 0; k < nz; ++k)
      for (int j = 1; j < ny - 1; ++j)
        for (int i = 1; i < nx - 1; ++i) {
          double qe = LH(e, k, j, i), qt = LH(tb, k, j, i);
          q[(size_t)b * n + ((size_t)k * ny + j) * nx + i] = qe;
          num += qe * qe;
          den += qt * qt;
        }
  }
  free(e);
#undef LH
  if (!(den > 0.0)) { free(q); return -1; }
  *loss = num / den;
  if (gy) {
    /* d(sum q^2)/dy: scatter 2 q(c) times each stencil coefficient of c */
    memset(gy, 0, (size_t)batch * n * sizeof(double));
    for (int b = 0; b < batch; ++b)
      for (int k = 0; k < nz; ++k)
        for (int j = 1; j < ny - 1; ++j)
          for (int i = 1; i < nx - 1; ++i) {
            double s = 2.0 * q[(size_t)b * n + ((size_t)k * ny + j) * nx + i] / den;
            double *g = gy + (size_t)b * n;
            g[((size_t)k * ny + j) * nx + i + 1] += s * w[0];
            g[((size_t)k * ny + j) * nx + i - 1] += s * w[0];
            g[((size_t)k * ny + j + 1) * nx + i] += s * w[1];
            g[((size_t)k * ny + j - 1) * nx + i] += s * w[1];
            g[((size_t)zmirror(k + 1, nz) * ny + j) * nx + i] += s * w[2];
            g[((size_t)zmirror(k - 1, nz) * ny + j) * nx + i] += s * w[2];
            g[((size_t)k * ny + j) * nx + i] -= 2.0 * s * (w[0] + w[1] + w[2]);
          }
  }
  free(q);
  return 0;
}

int ocnn_adam(int32_t n, double *params, const double *grad, double *m, double *v, int32_t step,
              double lr, double beta1, double beta2, double eps) {
  if (n < 0 || step < 1 || !params || !grad || !m || !v) return -1;
  const double c1 = 1.0 - pow(beta1, step), c2 = 1.0 - pow(beta2, step);
  for (int32_t q = 0; q < n; ++q) {
    m[q] = beta1 * m[q] + (1.0 - beta1) * grad[q];
    v[q] = beta2 * v[q] + (1.0 - beta2) * grad[q] * grad[q];
    params[q] -= lr * (m[q] / c1) / (sqrt(v[q] / c2) + eps);
  }
  return 0;
}
