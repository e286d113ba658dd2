/*
 * les_cnn.h — C ABI of the learned initial guess of the pressure-correction
 * Poisson solve (the guess network) and of its training on the GPU.
 *
 * Role in the method.  Each sub-iteration of the time step solves the
 * pressure-correction equation (Sec. 2.4 of the paper, compact Laplacian of
 * phi = alpha0 dp equal to the divergence right-hand side) by weighted-
 * Jacobi sweeps that stop when ||rhs - L phi||_2 <= tol ||rhs||_2.  A
 * starting iterate closer to the solution ends the sweeps sooner but never
 * changes that test.  With LES_GUESS_LEARNED the starting iterate of every
 * solve (after the first step) is
 *     phi_0 = base + (s / d) CNN(r / s),
 * base = the previous step's solution of the same sub-iteration (a previous
 * pressure correction), r = rhs - L base its residual for the new
 * right-hand side, s = RMS(r), d = 2/dx^2 + 2/dy^2 + 2/dz^2 (the one-input
 * network).  With LES_GUESS_LEARNED3 the first solve of each step starts
 * from
 *     phi_0 = base + (s / d) CNN(r / s, base d / s, rhs / s),
 * base = alpha0 (p^n - p^{n-1}) (the previous pressures), r and s as above
 * (the three-input network: the previous pressures and the divergence
 * right-hand side, their differences formed in FP64 before any rounding,
 * so the step-to-step change is not lost to bfloat16).
 *
 * Network.  Four 3x3x3 convolutions with biases, channels C -> 16 -> 16 ->
 * 16 -> 1 (C = 1 or 3 inputs), leaky ReLU of slope alpha after the first
 * three.  Weights and every layer input are rounded to bfloat16 (nearest
 * even); sums are FP32 (the first three layers on the matrix cores); the
 * output is FP32.
 * x and y wrap on whole fields (periodic = 1) or are "valid" on training
 * crops (periodic = 0: each layer trims one cell per side, 8 in total);
 * every layer reads the even mirror of its input in z.
 *
 * Parameters.  One FP32 vector of les_cnn_param_count(C) values in device
 * memory: per layer l = 0..3, W_l[tap][cout][cin] then b_l[cout], with
 * tap = 9 (dz+1) + 3 (dy+1) + (dx+1).  "packed" is its bfloat16 copy
 * (les_cnn_param_count(C) uint16 values) made by les_cnn_pack.
 *
 * Training loss.  On output crops (nz, ny, nx): e = out - target,
 * q = (L e)/d on interior cells (one-cell ring in x and y excluded, mirror
 * in z); loss = sum q^2 / sum ((L target)/d)^2 over the same cells: the
 * squared residual of the corrected guess relative to that of the base.
 * Targets are (phi* - base) d / s with phi* the solver's solution.
 *
 * Conventions are those of les.h: device pointers, stream-ordered calls,
 * no device allocation by the library (work buffers come from the caller),
 * negative return codes with les_last_error().  Every array argument is
 * device memory unless marked host.
 */
#ifndef LES_CNN_H
#define LES_CNN_H

#include "les.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct les_cnn_dims {
  int32_t batch;     /* number of fields / crops, >= 1 */
  int32_t nz, ny, nx; /* network input size of each (valid: ny, nx >= 11) */
  int32_t periodic;  /* 1: whole periodic fields; 0: valid crops */
  int32_t inputs;    /* input channels C: 1 or 3 */
  double alpha;      /* leaky ReLU slope, >= 0 */
} les_cnn_dims;

/* Number of FP32 parameters of the network with `inputs` input channels
 * (14737 for 1, 15601 for 3); LES_ERR_ARG for another count. */
int32_t les_cnn_param_count(int32_t inputs);

/* Bytes of the work buffer of les_cnn_forward / _loss / _backward /
 * _train_step for these dims (stored layer inputs, gradients, partial sums). */
size_t les_cnn_work_bytes(const les_cnn_dims *d);

/* packed[q] = bfloat16(params[q]) for the les_cnn_param_count(inputs)
 * parameters. */
int les_cnn_pack(int32_t inputs, const float *params, uint16_t *packed, void *stream);

/* Forward pass on a batch: x (batch, inputs, nz, ny, nx) FP32 (rounded to
 * bfloat16 on entry), out (batch, nz, ny - 8, nx - 8) for valid crops or
 * (batch, nz, ny, nx) for periodic fields.  Keeps the layer inputs in work
 * for les_cnn_backward. */
int les_cnn_forward(const les_cnn_dims *d, const float *params, const uint16_t *packed,
                    const float *x, void *work, float *out, void *stream);

/* Residual loss of out against target (both of the output size; valid
 * crops only) and gout = dloss/dout.  loss (host, nullable): synchronizes
 * the stream and stores the loss. */
int les_cnn_loss(const les_cnn_dims *d, double dx, double dy, double dz, const float *out,
                 const float *target, void *work, float *gout, double *loss, void *stream);

/* Gradient of the loss with respect to the parameters (FP32, parameter
 * layout) from gout and the layer inputs kept by the last les_cnn_forward
 * on the same work buffer (valid crops only).  Leaky-ReLU slopes come from
 * the sign of the stored bfloat16 activations; weight-gradient sums are
 * FP64 in a fixed order (deterministic). */
int les_cnn_backward(const les_cnn_dims *d, const uint16_t *packed, void *work,
                     const float *gout, float *grad, void *stream);

/* The input of layer `layer` (0..3) kept in work by the last
 * les_cnn_forward with these dims (bfloat16 values, written as FP32) in the
 * order (batch, channels, nz, ny_l, nx_l), ny_l = ny - 2 layer on valid
 * crops (ny on periodic fields), nx_l alike: for inspection and for
 * checking the backward pass on the very operands it used. */
int les_cnn_stored_input(const les_cnn_dims *d, const void *work, int32_t layer, float *out,
                         void *stream);

/* One Adam step (Kingma & Ba 2015, bias-corrected, step >= 1) on FP32
 * params with FP32 moments m, v. */
int les_cnn_adam(int32_t n, float *params, const float *grad, float *m, float *v, int32_t step,
                 double lr, double beta1, double beta2, double eps, void *stream);

/* forward + loss + backward + Adam + pack on one batch of crops.
 * loss (host, nullable) as in les_cnn_loss. */
int les_cnn_train_step(const les_cnn_dims *d, double dx, double dy, double dz, float *params,
                       uint16_t *packed, float *m, float *v, int32_t step, double lr,
                       double beta1, double beta2, double eps, const float *x,
                       const float *target, void *work, float *grad, double *loss,
                       void *stream);

/* Training pair from one solve of a run with configuration cfg (fields of
 * the storage type of cfg->precision): r = rhs - L base, s = RMS(r),
 * x = r / s, target = (phi - base) d / s (FP32 fields).  base nullable
 * (zero).  scratch: les_cnn_pair_scratch_bytes(cfg) bytes.  scale (host,
 * nullable): synchronizes and stores s. */
size_t les_cnn_pair_scratch_bytes(const les_config *cfg);
int les_cnn_pair(const les_config *cfg, const void *rhs, const void *base, const void *phi,
                 float *x, float *target, void *scratch, double *scale, void *stream);

/* les_cnn_pair for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid hipMalloc): the
 * same pair, bit for bit, with no scratch argument.  The residual is formed
 * in x itself and scaled there; the reduction partials and the scale
 * factors live in a fixed 16 KiB device array of the library (one per GPU,
 * held until the process ends), of which 8224 bytes are used whatever the
 * grid (1024 FP64 partial sums, then the scale factors), so no grid within the
 * limits of les_cnn_pair is refused for lack of scratch.  Calls no hipMalloc or
 * hipFree.  x and target must not alias rhs, base or phi.  Every call on
 * one GPU shares that GPU's array: calls that overlap on one GPU (two
 * streams, two threads) race and must be serialised by the caller.
 * scale (host, nullable): synchronizes and stores s. */
int les_cnn_pair_noalloc(const les_config *cfg, const void *rhs, const void *base,
                         const void *phi, float *x, float *target, double *scale,
                         void *stream);

/* Training pair of the three-input network from one solve: r = rhs - L
 * base, s = RMS(r), x (3, nz, ny, nx) FP32 = (r/s, base d/s, rhs/s) and
 * target = (phi - base) d/s; base the extrapolated pressure change the
 * solve started from (les_step_opts.dump_base).  phi and target nullable
 * together (the inputs only).  scratch and scale as in les_cnn_pair. */
int les_cnn_pair3(const les_config *cfg, const void *rhs, const void *base, const void *phi,
                  float *x, float *target, void *scratch, double *scale, void *stream);

/* Crops of npairs stored pairs: x_pairs (npairs, inputs, nz, ny, nx) and
 * t_pairs (npairs, nz, ny, nx), FP32.  crops: batch triples (pair, j0, i0),
 * each taken modulo its range.  xb gets (batch, inputs, nz, cy + 8, cx + 8)
 * from (j0 - 4, i0 - 4), tb (batch, nz, cy, cx) from (j0, i0), both
 * wrapping in x and y. */
int les_cnn_gather(int32_t inputs, const float *x_pairs, const float *t_pairs, int32_t npairs,
                   int32_t nz, int32_t ny, int32_t nx, const int32_t *crops, int32_t batch,
                   int32_t cy, int32_t cx, float *xb, float *tb, void *stream);

/* Bind the network used by LES_GUESS_LEARNED (one input) or
 * LES_GUESS_LEARNED3 (three inputs): copies params (device FP32, that
 * network's count) into the handle's workspace and packs them.  The
 * caller's buffer may be freed afterwards.  Error if the handle was created
 * with another guess mode. */
int les_bind_cnn(les_handle *h, const float *params, double alpha);

/* The learned guess of the handle's network on caller fields of its grid
 * and storage type: guess = base + (s/d) CNN(...), r = rhs - L base (rhs
 * is used as given).  scale (host, nullable): synchronizes and stores s. */
int les_cnn_guess(les_handle *h, const void *rhs, const void *base, void *guess, double *scale);

#ifdef __cplusplus
}
#endif

#endif
