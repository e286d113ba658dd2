// Training-pair entry point that allocates nothing (les_cnn_pair_noalloc in
// include/les_cnn.h): the same kernels as les_cnn_pair, with the residual
// written straight into the caller's x and scaled there, and the reduction
// partials and scale factors in a file-scope device array instead of a
// caller workspace.
#include "les_cnn.h"

#include <hip/hip_runtime.h>

#include <mutex>

#include "api_util.h"
#include "cnn_internal.h"

using namespace lesmi;

// Scratch of les_cnn_pair_noalloc: one copy per GPU, held until the process
// ends.  In host code `scratch` names a host-side stand-in: kernels get the
// device address looked up by device_scratch(), never this name.
static __device__ __align__(256) unsigned char scratch[16384];

namespace {

// Scratch of one call: kReduceBlocks FP64 partial sums of r^2, then the
// scale factors (s, 1/s, s/d).  Its size does not depend on the grid.
constexpr size_t kScratchBytes = sizeof(scratch);
constexpr size_t kPartialsOff = 0;
constexpr size_t kScaleOff = ((size_t)kReduceBlocks * sizeof(double) + 255) / 256 * 256;
constexpr size_t kScratchNeed = kScaleOff + 4 * sizeof(double);
static_assert(kScratchNeed <= kScratchBytes, "pair scratch does not fit");

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices];

// Device address of the current device's scratch, looked up once per device
// (with that device current) on its first call.
int device_scratch(unsigned char **out) {
  int dev = -1;
  HIP_TRY(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices)
    return fail(LES_ERR_ARG, "les_cnn_pair_noalloc: device %d beyond the %d supported", dev,
                kMaxDevices);
  std::lock_guard<std::mutex> lock(g_mu);
  if (!g_scratch[dev]) {
    void *ptr = nullptr;
    HIP_TRY(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr) return fail(LES_ERR_HIP, "les_cnn_pair_noalloc: no device address for the scratch");
    g_scratch[dev] = ptr;
  }
  *out = (unsigned char *)g_scratch[dev];
  return LES_OK;
}

bool grid_ok(const les_config *c) {
  return c && c->nx >= 4 && c->ny >= 4 && c->nz >= 4 && c->dx > 0 && c->dy > 0 && c->dz > 0 &&
         (c->precision == LES_FP64 || c->precision == LES_FP32) &&
         (double)c->nx * c->ny * c->nz < 4.0e9;
}

}  // namespace

extern "C" {

int les_cnn_pair_noalloc(const les_config *cfg, const void *rhs, const void *base,
                         const void *phi, float *x, float *target, double *scale,
                         void *stream) {
  if (!grid_ok(cfg)) return fail(LES_ERR_ARG, "invalid grid in config");
  if (!rhs || !phi || !x || !target) return fail(LES_ERR_ARG, "NULL argument");
  if (kScratchNeed > kScratchBytes)
    return fail(LES_ERR_ARG, "les_cnn_pair_noalloc needs %zu bytes of scratch, has %zu",
                kScratchNeed, kScratchBytes);
  unsigned char *ptr = nullptr;
  if (int rc = device_scratch(&ptr)) return rc;
  hipStream_t s = (hipStream_t)stream;
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
  const double D = 2.0 / (g.dx * g.dx) + 2.0 / (g.dy * g.dy) + 2.0 / (g.dz * g.dz);
  double *partials = (double *)(ptr + kPartialsOff);
  double *sc = (double *)(ptr + kScaleOff);
  // every partial and scale factor is written before it is read: nothing
  // of an earlier call's contents is used
  if (cfg->precision == LES_FP64) {
    launch_cnn_residual<double>(g, (const double *)rhs, (const double *)base, x, partials, s);
    launch_cnn_scale(partials, (double)g.n, D, sc, s);
    launch_cnn_pair_inplace<double>(g, (const double *)phi, (const double *)base, sc, D, x,
                                    target, s);
  } else {
    launch_cnn_residual<float>(g, (const float *)rhs, (const float *)base, x, partials, s);
    launch_cnn_scale(partials, (double)g.n, D, sc, s);
    launch_cnn_pair_inplace<float>(g, (const float *)phi, (const float *)base, sc, D, x, target,
                                   s);
  }
  LAUNCH_TRY();
  if (scale) {
    HIP_TRY(hipMemcpyAsync(scale, sc, sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
  }
  return LES_OK;
}

}  // extern "C"
