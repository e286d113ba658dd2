/* Standalone driver of the FP64 oracle for a host sanitizer build
 * (AddressSanitizer and UndefinedBehaviorSanitizer): time steps of the LES
 * oracle, the diagnostics of the final state, and a forward, loss and
 * backward pass of the guess network, on
 * inputs and sizes read from a file, results written to another.  Built and
 * run by tests/test_oracle_sanitizers.py; the oracle is test
 * infrastructure and so is this program.
 *
 * Input (native byte order):
 *   ocfg; int32 nsteps; u, v, w, thl, qt, p (n doubles each);
 *   ocnn_dims; params; x (batch C nz ny nx); target (batch nz ny_out nx_out)
 * Output:
 *   u, v, w, thl, qt, p; nsteps * n_subiter osolve records;
 *   6 diagnostic scalars and 9 x nz profiles of the final state;
 *   out (batch nz ny_out nx_out); loss; grad (params). */
#include <stdio.h>
#include <stdlib.h>

#include "cnn_oracle.h"
#include "les_oracle.h"

static int read_all(FILE *f, void *p, size_t bytes) { return fread(p, 1, bytes, f) == bytes; }
static int write_all(FILE *f, const void *p, size_t bytes) { return fwrite(p, 1, bytes, f) == bytes; }

static double *alloc_doubles(size_t n) { return (double *)calloc(n ? n : 1, sizeof(double)); }

int main(int argc, char **argv) {
  if (argc != 3) {
    fprintf(stderr, "usage: %s input output\n", argv[0]);
    return 2;
  }
  FILE *in = fopen(argv[1], "rb");
  if (!in) return 3;
  ocfg c;
  int32_t nsteps = 0;
  if (!read_all(in, &c, sizeof c) || !read_all(in, &nsteps, sizeof nsteps)) return 4;
  const size_t n = (size_t)c.nx * c.ny * c.nz;
  double *f[6];
  for (int k = 0; k < 6; ++k) {
    f[k] = alloc_doubles(n);
    if (!f[k] || !read_all(in, f[k], n * sizeof(double))) return 5;
  }
  ocnn_dims d;
  if (!read_all(in, &d, sizeof d)) return 6;
  const int np = ocnn_param_count(d.inputs);
  if (np <= 0) return 7;
  int ly[OCNN_LAYERS + 1], lx[OCNN_LAYERS + 1];
  for (int l = 0; l <= OCNN_LAYERS; ++l) ocnn_layer_size(&d, l, &ly[l], &lx[l]);
  const size_t nx_in = (size_t)d.batch * d.inputs * d.nz * d.ny * d.nx;
  const size_t n_out = (size_t)d.batch * d.nz * ly[OCNN_LAYERS] * lx[OCNN_LAYERS];
  double *params = alloc_doubles((size_t)np), *x = alloc_doubles(nx_in);
  double *target = alloc_doubles(n_out);
  if (!params || !x || !target) return 8;
  if (!read_all(in, params, (size_t)np * sizeof(double)) ||
      !read_all(in, x, nx_in * sizeof(double)) || !read_all(in, target, n_out * sizeof(double)))
    return 9;
  fclose(in);

  /* the LES steps */
  const size_t nsolve = (size_t)nsteps * c.n_subiter;
  osolve *rec = (osolve *)calloc(nsolve ? nsolve : 1, sizeof(osolve));
  if (!rec) return 10;
  int rc = oracle_step(&c, f[0], f[1], f[2], f[3], f[4], f[5], nsteps, NULL, rec, NULL);
  if (rc) {
    fprintf(stderr, "oracle_step failed (%d)\n", rc);
    return 11;
  }

  /* diagnostics of the final state */
  double scalars[6];
  double *profiles = alloc_doubles((size_t)9 * c.nz);
  if (!profiles) return 19;
  if ((rc = oracle_diagnostics(&c, f[0], f[1], f[2], f[3], f[4], scalars, profiles))) {
    fprintf(stderr, "oracle_diagnostics failed (%d)\n", rc);
    return 20;
  }

  /* the network: forward with the activations kept, loss, backward */
  double *acts[OCNN_LAYERS], *pre[OCNN_LAYERS] = {NULL, NULL, NULL, NULL};
  for (int l = 0; l < OCNN_LAYERS; ++l) {
    const size_t m = (size_t)d.batch * ocnn_cin(d.inputs, l) * d.nz * ly[l] * lx[l];
    acts[l] = alloc_doubles(m);
    if (!acts[l]) return 12;
    if (l < OCNN_LAYERS - 1) {
      const size_t mp = (size_t)d.batch * ocnn_cout(l) * d.nz * ly[l + 1] * lx[l + 1];
      pre[l] = alloc_doubles(mp);
      if (!pre[l]) return 12;
    }
  }
  double *out = alloc_doubles(n_out), *gy = alloc_doubles(n_out), *grad = alloc_doubles((size_t)np);
  if (!out || !gy || !grad) return 13;
  double loss = 0.0;
  if ((rc = ocnn_forward(&d, params, x, out, acts, pre))) {
    fprintf(stderr, "ocnn_forward failed (%d)\n", rc);
    return 14;
  }
  if ((rc = ocnn_loss(d.batch, d.nz, ly[OCNN_LAYERS], lx[OCNN_LAYERS], c.dx, c.dy, c.dz, out,
                      target, &loss, gy))) {
    fprintf(stderr, "ocnn_loss failed (%d)\n", rc);
    return 15;
  }
  if ((rc = ocnn_backward(&d, params, acts, pre, gy, grad))) {
    fprintf(stderr, "ocnn_backward failed (%d)\n", rc);
    return 16;
  }

  FILE *o = fopen(argv[2], "wb");
  if (!o) return 17;
  int ok = 1;
  for (int k = 0; k < 6; ++k) ok = ok && write_all(o, f[k], n * sizeof(double));
  ok = ok && write_all(o, rec, nsolve * sizeof(osolve));
  ok = ok && write_all(o, scalars, sizeof scalars);
  ok = ok && write_all(o, profiles, (size_t)9 * c.nz * sizeof(double));
  ok = ok && write_all(o, out, n_out * sizeof(double));
  ok = ok && write_all(o, &loss, sizeof loss);
  ok = ok && write_all(o, grad, (size_t)np * sizeof(double));
  if (fclose(o) != 0 || !ok) return 18;

  for (int k = 0; k < 6; ++k) free(f[k]);
  for (int l = 0; l < OCNN_LAYERS; ++l) {
    free(acts[l]);
    free(pre[l]);
  }
  free(params); free(x); free(target); free(rec); free(out); free(gy); free(grad); free(profiles);
  return 0;
}
