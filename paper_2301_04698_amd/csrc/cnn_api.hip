// C ABI of the guess network's training path (include/les_cnn.h): work
// buffer layout, validation and the stream-ordered composition of the
// forward, loss, backward and update kernels of k_cnn.hip.
#include "les_cnn.h"

#include <hip/hip_runtime.h>

#include <cstring>

#include "api_util.h"
#include "cnn_internal.h"

using namespace lesmi;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

int check_dims(const les_cnn_dims *d) {
  if (!d) return fail(LES_ERR_ARG, "dims is NULL");
  if (d->batch < 1 || d->nz < 1 || d->ny < 1 || d->nx < 1)
    return fail(LES_ERR_ARG, "dims %d x %d x %d x %d: every size must be >= 1", d->batch, d->nz,
                d->ny, d->nx);
  if (d->periodic != 0 && d->periodic != 1) return fail(LES_ERR_ARG, "periodic must be 0 or 1");
  if (!cnn_inputs_ok(d->inputs)) return fail(LES_ERR_ARG, "inputs must be 1 or 3, got %d", d->inputs);
  if (!d->periodic && (d->ny < 11 || d->nx < 11))
    return fail(LES_ERR_ARG, "valid crops need ny, nx >= 11 (output >= 3), got %d x %d", d->ny,
                d->nx);
  if (!(d->alpha >= 0.0)) return fail(LES_ERR_ARG, "alpha must be >= 0");
  if ((double)d->batch * d->nz * d->ny * d->nx * 64.0 > 1.0e12)
    return fail(LES_ERR_ARG, "dims too large");
  // the tiled layers address a z plane of 16-channel activations with
  // 32-bit element offsets
  if ((int64_t)d->ny * d->nx * kCnnCh >= (int64_t)1 << 31)
    return fail(LES_ERR_ARG, "at most 2^27 cells per z plane");
  return LES_OK;
}

// Per-layer input counts n[0..3] and the output count n[4].
void counts(const les_cnn_dims *d, int64_t n[kCnnLayers + 1]) {
  for (int l = 0; l <= kCnnLayers; ++l) {
    const CnnGeom G = cnn_geom(d->batch, d->nz, d->ny, d->nx, d->periodic,
                               l < kCnnLayers ? l : kCnnLayers - 1, d->inputs);
    n[l] = l < kCnnLayers ? G.n_in : G.n_out;
  }
}

struct Work {
  size_t a[kCnnLayers];  // stored layer inputs (bfloat16)
  size_t g1, g2;         // activation gradients (FP32, 16 channels)
  size_t q;              // loss scratch (FP32, output size)
  size_t partials;       // FP64 partial sums
  size_t stats;          // 4 doubles: loss, denominator, 2/denominator
  size_t total;
};

Work work_layout(const les_cnn_dims *d) {
  int64_t n[kCnnLayers + 1];
  counts(d, n);
  Work W;
  size_t off = 0;
  for (int l = 0; l < kCnnLayers; ++l) {
    W.a[l] = off;
    off = align_up(off + (size_t)n[l] * cnn_cin(d->inputs, l) * sizeof(uint16_t));
  }
  W.g1 = off;
  off = align_up(off + (size_t)n[1] * kCnnCh * sizeof(float));
  W.g2 = off;
  off = align_up(off + (size_t)n[2] * kCnnCh * sizeof(float));
  W.q = off;
  off = align_up(off + (size_t)n[4] * sizeof(float));
  W.partials = off;
  const size_t np = (size_t)kCnnWgradBlocks * kCnnMaxEntries > 2 * (size_t)kReduceBlocks
                        ? (size_t)kCnnWgradBlocks * kCnnMaxEntries
                        : 2 * (size_t)kReduceBlocks;
  off = align_up(off + np * sizeof(double));
  W.stats = off;
  off = align_up(off + 4 * sizeof(double));
  W.total = off;
  return W;
}

template <typename P>
P *at(void *base, size_t off) {
  return (P *)((char *)base + off);
}

int forward_impl(const les_cnn_dims *d, const float *params, const uint16_t *packed,
                 const float *x, void *work, float *out, hipStream_t s) {
  const Work W = work_layout(d);
  int64_t n[kCnnLayers + 1];
  counts(d, n);
  launch_cnn_round(n[0], d->inputs, (int64_t)d->nz * d->ny * d->nx, x, nullptr,
                   at<uint16_t>(work, W.a[0]), s);
  for (int l = 0; l < kCnnLayers; ++l) {
    const CnnGeom G = cnn_geom(d->batch, d->nz, d->ny, d->nx, d->periodic, l, d->inputs);
    launch_cnn_conv(l, G, at<uint16_t>(work, W.a[l]), params, packed, (float)d->alpha,
                    l + 1 < kCnnLayers ? at<uint16_t>(work, W.a[l + 1]) : nullptr,
                    l + 1 < kCnnLayers ? nullptr : out, s);
  }
  LAUNCH_TRY();
  return LES_OK;
}

int loss_impl(const les_cnn_dims *d, double dx, double dy, double dz, const float *out,
              const float *target, void *work, float *gout, double *loss, hipStream_t s) {
  const Work W = work_layout(d);
  const CnnGeom G = cnn_geom(d->batch, d->nz, d->ny, d->nx, 0, kCnnLayers - 1, d->inputs);
  const double D = 2.0 / (dx * dx) + 2.0 / (dy * dy) + 2.0 / (dz * dz);
  launch_cnn_loss(d->batch, d->nz, G.nyo, G.nxo, 1.0 / (dx * dx * D), 1.0 / (dy * dy * D),
                  1.0 / (dz * dz * D), out, target, at<float>(work, W.q),
                  at<double>(work, W.partials), at<double>(work, W.stats), gout, s);
  LAUNCH_TRY();
  if (loss) {
    double st[2];
    HIP_TRY(hipMemcpyAsync(st, at<double>(work, W.stats), sizeof(st), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (!(st[1] > 0.0))
      return fail(LES_ERR_ARG, "loss undefined: the targets have no interior residual");
    *loss = st[0];
  }
  return LES_OK;
}

int backward_impl(const les_cnn_dims *d, const uint16_t *packed, void *work, const float *gout,
                  float *grad, hipStream_t s) {
  const Work W = work_layout(d);
  double *partials = at<double>(work, W.partials);
  float *g1 = at<float>(work, W.g1), *g2 = at<float>(work, W.g2);
  // gradient with respect to each layer's output: layer 3 gout, 2 -> g1,
  // 1 -> g2, 0 -> g1 (g1 is free again once layer 2 is done)
  const float *gy = gout;
  float *next[kCnnLayers] = {nullptr, g1, g2, g1};
  for (int l = kCnnLayers - 1; l >= 0; --l) {
    const CnnGeom G = cnn_geom(d->batch, d->nz, d->ny, d->nx, 0, l, d->inputs);
    const uint16_t *ain = at<uint16_t>(work, W.a[l]);
    launch_cnn_wgrad(l, G, gy, ain, partials, grad, s);
    if (l > 0) {
      launch_cnn_dgrad(l, G, gy, packed, ain, (float)d->alpha, next[l], s);
      gy = next[l];
    }
  }
  LAUNCH_TRY();
  return LES_OK;
}

bool grid_ok(const les_config *c) {
  return c && c->nx >= 4 && c->ny >= 4 && c->nz >= 4 && c->dx > 0 && c->dy > 0 && c->dz > 0 &&
         (c->precision == LES_FP64 || c->precision == LES_FP32) &&
         (double)c->nx * c->ny * c->nz < 4.0e9;
}

Grid pair_grid(const les_config *cfg) {
  Grid g;
  g.nx = cfg->nx;
  g.ny = cfg->ny;
  g.nz = cfg->nz;
  g.nxy = (int64_t)g.nx * g.ny;
  g.sy = g.ny == 1 ? 0 : g.nx;
  g.n = g.nxy * g.nz;
  g.dx = cfg->dx;
  g.dy = cfg->dy;
  g.dz = cfg->dz;
  g.dt = cfg->dt;
  return g;
}

// Pair of the three-input network (les_cnn_pair3).
template <typename T>
void pair3_impl(const Grid &g, const T *rhs, const T *base, const T *phi, float *r,
                double *partials, double *sc, float *x, float *t, hipStream_t s) {
  const double D = 2.0 / (g.dx * g.dx) + 2.0 / (g.dy * g.dy) + 2.0 / (g.dz * g.dz);
  launch_cnn_residual<T>(g, rhs, base, r, partials, s);
  launch_cnn_scale(partials, (double)g.n, D, sc, s);
  launch_cnn_pair3<T>(g, r, base, rhs, phi, sc, D, x, t, s);
}

}  // namespace

extern "C" {

int32_t les_cnn_param_count(int32_t inputs) {
  if (!cnn_inputs_ok(inputs)) return fail(LES_ERR_ARG, "inputs must be 1 or 3, got %d", inputs);
  return cnn_param_count(inputs);
}

size_t les_cnn_work_bytes(const les_cnn_dims *d) {
  if (check_dims(d)) return 0;
  return work_layout(d).total;
}

int les_cnn_pack(int32_t inputs, const float *params, uint16_t *packed, void *stream) {
  if (!cnn_inputs_ok(inputs)) return fail(LES_ERR_ARG, "inputs must be 1 or 3, got %d", inputs);
  if (!params || !packed) return fail(LES_ERR_ARG, "params and packed must be non-NULL");
  launch_cnn_pack(params, cnn_param_count(inputs), packed, (hipStream_t)stream);
  LAUNCH_TRY();
  return LES_OK;
}

int les_cnn_forward(const les_cnn_dims *d, const float *params, const uint16_t *packed,
                    const float *x, void *work, float *out, void *stream) {
  if (int rc = check_dims(d)) return rc;
  if (!params || !packed || !x || !work || !out) return fail(LES_ERR_ARG, "NULL argument");
  return forward_impl(d, params, packed, x, work, out, (hipStream_t)stream);
}

int les_cnn_loss(const les_cnn_dims *d, double dx, double dy, double dz, const float *out,
                 const float *target, void *work, float *gout, double *loss, void *stream) {
  if (int rc = check_dims(d)) return rc;
  if (d->periodic) return fail(LES_ERR_ARG, "the loss is defined on valid crops only");
  if (!(dx > 0 && dy > 0 && dz > 0)) return fail(LES_ERR_ARG, "dx, dy, dz must be > 0");
  if (!out || !target || !work || !gout) return fail(LES_ERR_ARG, "NULL argument");
  return loss_impl(d, dx, dy, dz, out, target, work, gout, loss, (hipStream_t)stream);
}

int les_cnn_backward(const les_cnn_dims *d, const uint16_t *packed, void *work,
                     const float *gout, float *grad, void *stream) {
  if (int rc = check_dims(d)) return rc;
  if (d->periodic) return fail(LES_ERR_ARG, "the backward pass is defined on valid crops only");
  if (!packed || !work || !gout || !grad) return fail(LES_ERR_ARG, "NULL argument");
  return backward_impl(d, packed, work, gout, grad, (hipStream_t)stream);
}

int les_cnn_stored_input(const les_cnn_dims *d, const void *work, int32_t layer, float *out,
                         void *stream) {
  if (int rc = check_dims(d)) return rc;
  if (layer < 0 || layer >= kCnnLayers) return fail(LES_ERR_ARG, "layer %d out of range", layer);
  if (!work || !out) return fail(LES_ERR_ARG, "NULL argument");
  const Work W = work_layout(d);
  const CnnGeom G = cnn_geom(d->batch, d->nz, d->ny, d->nx, d->periodic, layer, d->inputs);
  launch_cnn_unpack(G, cnn_cin(d->inputs, layer),
                    at<uint16_t>(const_cast<void *>(work), W.a[layer]), out,
                    (hipStream_t)stream);
  LAUNCH_TRY();
  return LES_OK;
}

int les_cnn_adam(int32_t n, float *params, const float *grad, float *m, float *v, int32_t step,
                 double lr, double beta1, double beta2, double eps, void *stream) {
  if (n < 0 || step < 1 || !params || !grad || !m || !v)
    return fail(LES_ERR_ARG, "adam: invalid argument (n %d, step %d)", n, step);
  if (!(lr > 0 && beta1 >= 0 && beta1 < 1 && beta2 >= 0 && beta2 < 1 && eps > 0))
    return fail(LES_ERR_ARG, "adam: invalid hyper-parameters");
  if (n == 0) return LES_OK;
  launch_cnn_adam(n, params, grad, m, v, step, lr, beta1, beta2, eps, (hipStream_t)stream);
  LAUNCH_TRY();
  return LES_OK;
}

int les_cnn_train_step(const les_cnn_dims *d, double dx, double dy, double dz, float *params,
                       uint16_t *packed, float *m, float *v, int32_t step, double lr,
                       double beta1, double beta2, double eps, const float *x,
                       const float *target, void *work, float *grad, double *loss,
                       void *stream) {
  if (int rc = check_dims(d)) return rc;
  if (d->periodic) return fail(LES_ERR_ARG, "training runs on valid crops only");
  if (!params || !packed || !m || !v || !x || !target || !work || !grad)
    return fail(LES_ERR_ARG, "NULL argument");
  if (!(dx > 0 && dy > 0 && dz > 0)) return fail(LES_ERR_ARG, "dx, dy, dz must be > 0");
  hipStream_t s = (hipStream_t)stream;
  const Work W = work_layout(d);
  int64_t n[kCnnLayers + 1];
  counts(d, n);
  // the output and its gradient share the loss scratch region's neighbour:
  // out in g2 (large enough: n[2] * 16 >= n[4]), gout in g1
  float *out = at<float>(work, W.g2);
  float *gout = at<float>(work, W.g1);
  if (int rc = forward_impl(d, params, packed, x, work, out, s)) return rc;
  if (int rc = loss_impl(d, dx, dy, dz, out, target, work, gout, nullptr, s)) return rc;
  // gout must survive until layer 3's backward is done: copy it to the q
  // scratch (the loss no longer needs q)
  HIP_TRY(hipMemcpyAsync(at<float>(work, W.q), gout, (size_t)n[4] * sizeof(float),
                         hipMemcpyDeviceToDevice, s));
  if (int rc = backward_impl(d, packed, work, at<float>(work, W.q), grad, s)) return rc;
  const int np = cnn_param_count(d->inputs);
  if (int rc = les_cnn_adam(np, params, grad, m, v, step, lr, beta1, beta2, eps, s)) return rc;
  launch_cnn_pack(params, np, packed, s);
  LAUNCH_TRY();
  if (loss) {
    double st[2];
    HIP_TRY(hipMemcpyAsync(st, at<double>(work, W.stats), sizeof(st), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    *loss = st[0];
  }
  return LES_OK;
}

size_t les_cnn_pair_scratch_bytes(const les_config *cfg) {
  if (!grid_ok(cfg)) return 0;
  const size_t n = (size_t)cfg->nx * cfg->ny * cfg->nz;
  return align_up(n * sizeof(float)) + align_up(kReduceBlocks * sizeof(double)) +
         align_up(4 * sizeof(double));
}

int les_cnn_pair(const les_config *cfg, const void *rhs, const void *base, const void *phi,
                 float *x, float *target, void *scratch, double *scale, void *stream) {
  if (!grid_ok(cfg)) return fail(LES_ERR_ARG, "invalid grid in config");
  if (!rhs || !phi || !x || !target || !scratch) return fail(LES_ERR_ARG, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  const Grid g = pair_grid(cfg);
  const double D = 2.0 / (g.dx * g.dx) + 2.0 / (g.dy * g.dy) + 2.0 / (g.dz * g.dz);
  float *r = (float *)scratch;
  double *partials = at<double>(scratch, align_up((size_t)g.n * sizeof(float)));
  double *sc = at<double>(scratch, align_up((size_t)g.n * sizeof(float)) +
                                       align_up(kReduceBlocks * sizeof(double)));
  if (cfg->precision == LES_FP64) {
    launch_cnn_residual<double>(g, (const double *)rhs, (const double *)base, r, partials, s);
    launch_cnn_scale(partials, (double)g.n, D, sc, s);
    launch_cnn_pair<double>(g, r, (const double *)phi, (const double *)base, sc, D, x, target, s);
  } else {
    launch_cnn_residual<float>(g, (const float *)rhs, (const float *)base, r, partials, s);
    launch_cnn_scale(partials, (double)g.n, D, sc, s);
    launch_cnn_pair<float>(g, r, (const float *)phi, (const float *)base, sc, D, x, target, s);
  }
  LAUNCH_TRY();
  if (scale) {
    HIP_TRY(hipMemcpyAsync(scale, sc, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  return LES_OK;
}

int les_cnn_pair3(const les_config *cfg, const void *rhs, const void *base, const void *phi,
                  float *x, float *target, void *scratch, double *scale, void *stream) {
  if (!grid_ok(cfg)) return fail(LES_ERR_ARG, "invalid grid in config");
  if (!rhs || !base || !x || !scratch || (phi && !target) || (!phi && target))
    return fail(LES_ERR_ARG, "NULL argument");
  hipStream_t s = (hipStream_t)stream;
  const Grid g = pair_grid(cfg);
  float *r = (float *)scratch;
  double *partials = at<double>(scratch, align_up((size_t)g.n * sizeof(float)));
  double *sc = at<double>(scratch, align_up((size_t)g.n * sizeof(float)) +
                                       align_up(kReduceBlocks * sizeof(double)));
  if (cfg->precision == LES_FP64)
    pair3_impl<double>(g, (const double *)rhs, (const double *)base, (const double *)phi, r,
                       partials, sc, x, target, s);
  else
    pair3_impl<float>(g, (const float *)rhs, (const float *)base, (const float *)phi, r, partials,
                      sc, x, target, s);
  LAUNCH_TRY();
  if (scale) {
    HIP_TRY(hipMemcpyAsync(scale, sc, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  return LES_OK;
}

int les_cnn_gather(int32_t inputs, const float *x_pairs, const float *t_pairs, int32_t npairs,
                   int32_t nz, int32_t ny, int32_t nx, const int32_t *crops, int32_t batch,
                   int32_t cy, int32_t cx, float *xb, float *tb, void *stream) {
  if (!cnn_inputs_ok(inputs)) return fail(LES_ERR_ARG, "inputs must be 1 or 3, got %d", inputs);
  if (!x_pairs || !t_pairs || !crops || !xb || !tb) return fail(LES_ERR_ARG, "NULL argument");
  if (npairs < 1 || nz < 1 || ny < 5 || nx < 5 || batch < 1 || cy < 1 || cx < 1)
    return fail(LES_ERR_ARG, "gather: invalid sizes");
  // crop entries live in device memory: the kernel reduces each modulo its
  // range, so every read stays inside the stored pairs
  launch_cnn_gather(x_pairs, t_pairs, npairs, inputs, nz, ny, nx, crops, batch, cy, cx, xb, tb,
                    (hipStream_t)stream);
  LAUNCH_TRY();
  return LES_OK;
}

}  // extern "C"
