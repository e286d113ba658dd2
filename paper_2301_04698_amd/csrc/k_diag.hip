// Diagnostics of the state: FP64 horizontal means per level (the mean
// profiles the paper reports for its stratocumulus case, Sec. 4.1), the
// domain integrals of rho0 theta_l and rho0 q_t (conserved by the scheme,
// Sec. 2.4), kinetic energy, central divergence and CFL number.
#include "les_device.h"

namespace lesmi {

namespace {

// One block per level; threads stride over the level's cells in a fixed
// order so the sums are deterministic.
template <typename T>
__global__ __launch_bounds__(kBlock) void diag_kernel(Grid g, Dyn<T> d, Profiles<T> P,
                                                      const T *__restrict__ u,
                                                      const T *__restrict__ v,
                                                      const T *__restrict__ w,
                                                      const T *__restrict__ thl,
                                                      const T *__restrict__ qt,
                                                      const T *__restrict__ ql,
                                                      const T *__restrict__ b,
                                                      double *__restrict__ out) {
  const int k = blockIdx.x;
  const double r0 = P.rho0[k];
  const double rm = P.rho0[k > 0 ? k - 1 : 0];
  const double rp = P.rho0[k + 1 < g.nz ? k + 1 : g.nz - 1];
  double acc[13];
#pragma unroll
  for (int m = 0; m < 13; ++m) acc[m] = 0.0;
  double dmax = 0.0, cmax = 0.0;
  for (int64_t r = threadIdx.x; r < g.nxy; r += blockDim.x) {
    const int j = (int)(r / g.nx);
    const int i = (int)(r - (int64_t)g.nx * j);
    const int64_t q = r + g.nxy * k;
    const double uu = u[q], vv = v[q], ww = w[q], th = thl[q], qq = qt[q];
    acc[0] += th;
    acc[1] += qq;
    acc[2] += (double)ql[q];
    acc[3] += uu;
    acc[4] += vv;
    acc[5] += ww;
    acc[6] += ww * ww;
    acc[7] += ww * ww * ww;
    acc[8] += (double)b[q];
    acc[9] += r0 * th;
    acc[10] += r0 * qq;
    acc[11] += 0.5 * r0 * (uu * uu + vv * vv + ww * ww);
    const double div =
        (r0 * (double)gload(u, g, i + 1, j, k, T(-1)) - r0 * (double)gload(u, g, i - 1, j, k, T(-1))) /
            (2.0 * g.dx) +
        (r0 * (double)gload(v, g, i, j + 1, k, T(-1)) - r0 * (double)gload(v, g, i, j - 1, k, T(-1))) /
            (2.0 * g.dy) +
        (rp * (double)gload(w, g, i, j, k + 1, T(-1)) - rm * (double)gload(w, g, i, j, k - 1, T(-1))) /
            (2.0 * g.dz);
    acc[12] += div * div;
    dmax = fmax(dmax, fabs(div));
    cmax = fmax(cmax, fabs(uu) * g.dt / g.dx + fabs(vv) * g.dt / g.dy + fabs(ww) * g.dt / g.dz);
  }
  (void)d;
#pragma unroll
  for (int m = 0; m < 13; ++m) {
    const double s = block_sum(acc[m]);
    if (threadIdx.x == 0) out[(int64_t)k * kDiagStride + m] = s;
  }
  const double a = block_max(dmax);
  const double c = block_max(cmax);
  if (threadIdx.x == 0) {
    out[(int64_t)k * kDiagStride + 13] = a;
    out[(int64_t)k * kDiagStride + 14] = c;
    out[(int64_t)k * kDiagStride + 15] = 0.0;
  }
}

}  // namespace

template <typename T>
void launch_diag(const Grid &g, const Dyn<T> &d, const Profiles<T> &P, const T *u, const T *v,
                 const T *w, const T *thl, const T *qt, const T *ql, const T *b,
                 double *level_sums, hipStream_t s) {
  diag_kernel<T><<<g.nz, kBlock, 0, s>>>(g, d, P, u, v, w, thl, qt, ql, b, level_sums);
}

template void launch_diag<float>(const Grid &, const Dyn<float> &, const Profiles<float> &,
                                 const float *, const float *, const float *, const float *,
                                 const float *, const float *, const float *, double *, hipStream_t);
template void launch_diag<double>(const Grid &, const Dyn<double> &, const Profiles<double> &,
                                  const double *, const double *, const double *, const double *,
                                  const double *, const double *, const double *, double *,
                                  hipStream_t);

}  // namespace lesmi
