/* Oracle of the learned Poisson initial guess: a plain, serial FP64 CPU
 * implementation of the small 3D convolutional network, its loss, its
 * gradients and the Adam update.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the CPU
 * baseline of the benchmark call this code; the library never does.
 *
 * Network (the guess network of the learned Poisson initial guess):
 *   four 3x3x3 convolutions, channels C -> 16 -> 16 -> 16 -> 1, biases,
 *   leaky ReLU with slope alpha after the first three; C = 1 or 3 inputs.
 *   Inputs (C = 1): the residual of the base guess, divided by its RMS s;
 *   (C = 3): that residual, the base guess times d/s and the right-hand
 *   side divided by s (the previous pressures and the divergence).
 *   Output: the correction to the base guess in units of s/d, with
 *   d = 2/dx^2 + 2/dy^2 + 2/dz^2 the diagonal of the compact Laplacian.
 * Geometry per batch item, arrays (nz, ny, nx), x fastest:
 *   periodic = 1: x and y wrap; output has the input's size;
 *   periodic = 0: x and y "valid"; each layer trims one cell per side.
 *   z: every layer reads the even mirror of its input (ghost -1 -> 0,
 *   nz -> nz-1), the Neumann wall convention of the pressure.
 * Rounding (bf16 = 1): weights and every layer input are rounded to
 *   bfloat16 (round to nearest even); sums are exact FP64 here (the GPU
 *   accumulates in FP32); biases and the output stay unrounded.
 *   bf16 = 0: plain FP64 throughout (for finite-difference checks).
 *
 * Parameter vector (FP32 values held in doubles), layer by layer:
 *   W_l[tap][cout][cin] then b_l[cout], tap = 9 (dz+1) + 3 (dy+1) + (dx+1).
 */
#ifndef CNN_ORACLE_H
#define CNN_ORACLE_H
#include <stdint.h>

#define OCNN_LAYERS 4
#define OCNN_TAPS 27

typedef struct ocnn_dims {
  int32_t batch, nz, ny, nx; /* input size per batch item */
  int32_t periodic;          /* 1 periodic x,y; 0 valid x,y */
  int32_t bf16;              /* 1 emulate bfloat16 rounding */
  int32_t inputs;            /* input channels C: 1 or 3 */
  int32_t reserved;          /* 0 */
  double alpha;              /* leaky ReLU slope */
} ocnn_dims;

/* Channel counts and parameter offsets of the network with `inputs` input
 * channels (-1 for an invalid layer or input count). */
int ocnn_cin(int inputs, int l);
int ocnn_cout(int l);
int ocnn_weight_offset(int inputs, int l);
int ocnn_bias_offset(int inputs, int l);
int ocnn_param_count(int inputs);
/* Per-item size of the input of layer l (l = 4: the output). */
void ocnn_layer_size(const ocnn_dims *d, int l, int *ny, int *nx);

/* bfloat16 round to nearest even of a double. */
double ocnn_bf16(double v);

/* Forward pass on x [b][c][z][y][x] (C input channels).  acts (nullable)
 * receives, for l = 0..3, the rounded input of layer l (channels-first
 * [b][c][z][y][x]) and pre (nullable) the pre-activation y_l of layers
 * 0..2 (needed by the backward pass); out gets y_3 [b][z][y][x]. */
int ocnn_forward(const ocnn_dims *d, const double *params, const double *x, double *out,
                 double *const *acts, double *const *pre);

/* Backward pass from gout = dLoss/dout; fills grad (same layout as params).
 * acts and pre are those of the forward pass. */
int ocnn_backward(const ocnn_dims *d, const double *params, double *const *acts,
                  double *const *pre, const double *gout, double *grad);

/* Residual loss of a batch of outputs against targets on (nz, ny, nx)
 * crops: e = y - t, q = Lh e on the interior cells (one-cell ring in x and
 * y excluded; z with the mirror), Lh = compact Laplacian / d.
 * loss = sum q^2 / sum (Lh t)^2 over the same cells, gy = dloss/dy. */
int ocnn_loss(int32_t batch, int32_t nz, int32_t ny, int32_t nx, double dx, double dy, double dz,
              const double *y, const double *t, double *loss, double *gy);

/* One Adam step (Kingma & Ba 2015) with bias correction; step counts from 1. */
int ocnn_adam(int32_t n, double *params, const double *grad, double *m, double *v, int32_t step,
              double lr, double beta1, double beta2, double eps);

#endif
