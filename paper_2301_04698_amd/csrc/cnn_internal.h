// Internal declarations of the guess network (learned Poisson initial
// guess): layer geometry and the launchers implemented in k_cnn.hip.
//
// Network: four 3x3x3 convolutions, channels C -> 16 -> 16 -> 16 -> 1 (C = 1
// or 3 inputs), with biases and a leaky ReLU after the first three.
// Weights and layer inputs are bfloat16 (round to nearest even), sums FP32
// (inference on the matrix cores), the output FP32.
// Activations are stored channels-last: element (cell, c) at cell * C + c.
#pragma once

#include "les_internal.h"

namespace lesmi {

constexpr int kCnnLayers = 4;
constexpr int kCnnTaps = 27;
constexpr int kCnnCh = 16;

constexpr int kCnnMaxInputs = 3;
__host__ __device__ constexpr bool cnn_inputs_ok(int inputs) { return inputs == 1 || inputs == 3; }
__host__ __device__ constexpr int cnn_cin(int inputs, int l) { return l == 0 ? inputs : kCnnCh; }
__host__ __device__ constexpr int cnn_cout(int l) { return l == kCnnLayers - 1 ? 1 : kCnnCh; }
// Flat FP32 parameter vector: per layer W[tap][cout][cin] then b[cout].
__host__ __device__ constexpr int cnn_weight_offset(int inputs, int l) {
  int off = 0;
  for (int q = 0; q < l; ++q) off += kCnnTaps * cnn_cin(inputs, q) * cnn_cout(q) + cnn_cout(q);
  return off;
}
__host__ __device__ constexpr int cnn_bias_offset(int inputs, int l) {
  return cnn_weight_offset(inputs, l) + kCnnTaps * cnn_cin(inputs, l) * cnn_cout(l);
}
__host__ __device__ constexpr int cnn_param_count(int inputs) {
  return cnn_weight_offset(inputs, kCnnLayers);
}
// Largest weight-gradient entry count of one layer (weights + biases).
constexpr int kCnnMaxEntries = kCnnTaps * kCnnCh * kCnnCh + kCnnCh;

// Geometry of layer l of the network with `inputs` input channels: input
// (batch, nz, nyi, nxi), output (batch, nz, nyo, nxo).  periodic: x, y wrap
// and sizes are kept; otherwise x, y are "valid" (output cell (j, i) reads
// input (j + 1 + dy, i + 1 + dx)).  z always reads the even mirror of the
// layer input.
struct CnnGeom {
  int batch, nz, nyi, nxi, nyo, nxo, periodic, inputs;
  int64_t n_in, n_out;
};
CnnGeom cnn_geom(int batch, int nz, int ny, int nx, int periodic, int layer, int inputs);

// Weight-gradient reduction: blocks of one launch (their partials).
constexpr int kCnnWgradBlocks = 1024;

// ------------------------------------------------------------ launchers
// wbf[q] = bf16(params[q]), q < n.
void launch_cnn_pack(const float *params, int n, uint16_t *wbf, hipStream_t s);
// Network input: x channels-first (batch, C, cells) to channels-last
// a0[(b cells + r) C + c] = bf16(x[(b C + c) cells + r] * scale) (scale:
// device double, nullptr = 1); n = batch * cells.
void launch_cnn_round(int64_t n, int C, int64_t cells, const float *x, const double *scale,
                      uint16_t *a0, hipStream_t s);
// Layers 0..2: aout = bf16(leaky(conv(ain) + b)).  Layer 3: yout = conv(ain) + b.
void launch_cnn_conv(int layer, const CnnGeom &G, const uint16_t *ain, const float *params,
                     const uint16_t *wbf, float alpha, uint16_t *aout, float *yout, hipStream_t s);
// Layers 0 and 1 of the one-input network on a periodic field in one pass
// (G: layer 1's geometry, batch items of (nz, ny, nx)): the input is the
// FP32 residual r (batch, nz, ny, nx) times *scale, rounded to bfloat16 as
// launch_cnn_round does; aout = layer 1's output, as launch_cnn_conv
// writes it.  Layer 0's activations stay on chip.
void launch_cnn_in_mid(const CnnGeom &G, const float *r, const double *scale, const float *params,
                       const uint16_t *wbf, float alpha, uint16_t *aout, hipStream_t s);
// Layer 3 fused with the guess: guess = base + s_over_d * (conv(ain) + b).
template <typename T>
void launch_cnn_guess(const CnnGeom &G, const uint16_t *ain, const float *params,
                      const uint16_t *wbf, const T *base, const double *s_over_d, T *guess,
                      hipStream_t s);

// Residual loss on (batch, nz, ny, nx) crops (see the oracle for the
// definition).  stats[0] = loss, stats[1] = denominator.  gy = dloss/dy.
// partials: 2 * kReduceBlocks doubles; q: scratch of the crop size.
void launch_cnn_loss(int batch, int nz, int ny, int nx, double wx, double wy, double wz,
                     const float *y, const float *t, float *q, double *partials, double *stats,
                     float *gy, hipStream_t s);

// Backward through layer l (valid geometry): gprev = (W^T gy) * leaky'(ain)
// for l >= 1, where ain is the stored input of layer l.
void launch_cnn_dgrad(int layer, const CnnGeom &G, const float *gy, const uint16_t *wbf,
                      const uint16_t *ain, float alpha, float *gprev, hipStream_t s);
// Weight and bias gradient of layer l: per-block FP64 partials, then a
// fixed-order sum into grad (FP32, parameter layout).
void launch_cnn_wgrad(int layer, const CnnGeom &G, const float *gy, const uint16_t *ain,
                      double *partials, float *grad, hipStream_t s);

// Stored input of a layer of geometry G (C channels, channels-last
// bfloat16) as FP32 in (batch, C, nz, nyi, nxi) order.
void launch_cnn_unpack(const CnnGeom &G, int C, const uint16_t *a, float *out, hipStream_t s);

void launch_cnn_adam(int n, float *params, const float *grad, float *m, float *v, int step,
                     double lr, double beta1, double beta2, double eps, hipStream_t s);

// Network input of a solve: r = rhs - L base (compact Laplacian, periodic
// x, y, mirror z, FP64 arithmetic) and FP64 partial sums of r^2.
template <typename T>
void launch_cnn_residual(const Grid &g, const T *rhs, const T *base, float *r, double *partials,
                         hipStream_t s);
// From kReduceBlocks partials of sum r^2: sc[0] = s = RMS(r), sc[1] = 1/s
// (0 if s = 0), sc[2] = s/d.
void launch_cnn_scale(const double *partials, double n, double d, double *sc, hipStream_t s);
// Training pair: x = r/s and t = (phi - base) d/s, FP32.
template <typename T>
void launch_cnn_pair(const Grid &g, const float *r, const T *phi, const T *base, const double *sc,
                     double d, float *x, float *t, hipStream_t s);
// Three-input network: the input channels (r/s, base d/s, rhs/s) with
// s = sc[0] (sc as launch_cnn_scale makes it), channels-last bfloat16 into
// a0 (whole field), or FP32 channels-first into x (x, x + n, x + 2n) with
// the target t = (phi - base) d/s (a training pair; phi nullable: no t).
template <typename T>
void launch_cnn_input3(const Grid &g, const float *r, const T *base, const T *rhs,
                       const double *sc, double d, uint16_t *a0, hipStream_t s);
template <typename T>
void launch_cnn_pair3(const Grid &g, const float *r, const T *base, const T *rhs, const T *phi,
                      const double *sc, double d, float *x, float *t, hipStream_t s);
// launch_cnn_pair with the residual already in x (scaled there).
template <typename T>
void launch_cnn_pair_inplace(const Grid &g, const T *phi, const T *base, const double *sc,
                             double d, float *x, float *t, hipStream_t s);
// Crops of npairs stored pairs (inputs of C channels, channels-first).
// crops[3b..3b+2] = (pair, j0, i0), each taken modulo its range: input crop
// (C, nz, cy + 8, cx + 8) from (j0 - 4, i0 - 4), target crop (nz, cy, cx)
// from (j0, i0), both wrapping in x, y.
void launch_cnn_gather(const float *X, const float *Tt, int npairs, int C, int nz, int ny, int nx,
                       const int32_t *crops, int batch, int cy, int cx, float *xb, float *tb,
                       hipStream_t s);

}  // namespace lesmi
