// Pressure-correction Poisson path (paper Sec. 2.4 and App. A): right-hand
// side with the collocated-grid correction, projection, and the fixed-order
// FP64 reductions that drive the device-side stopping test.  The sweeps are
// in k_tsweep.hip.
#include "les_column.h"

namespace lesmi {

namespace {

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// rhs = (alpha0/dt) div_c(rho0 u_hat) - C(phi_lag), with C the App. A
// fourth difference (wide minus compact Laplacian) of the previous
// sub-iteration's correction (phi_lag == nullptr: C = 0).  Column-marching.
template <typename T, bool EDGE>
__device__ __forceinline__ void rhs_level(const Grid &g, const Dyn<T> &d, const Profiles<T> &P,
                                          const ColPts<T> &pts, int k, bool active,
                                          const T *__restrict__ u, const T *__restrict__ v,
                                          const T *__restrict__ w, const T *__restrict__ lag,
                                          T *__restrict__ rhs) {
  const Lvl<T, EDGE> at(g, pts, k);
  const T r0 = at.prof(P.rho0_t, 0);
  const T rm = at.prof(P.rho0_t, -1), rp = at.prof(P.rho0_t, 1);
  const T div = (r0 * at(u, 1, 0, 0, T(-1)) - r0 * at(u, -1, 0, 0, T(-1))) * d.inv_2dx +
                (r0 * at(v, 0, 1, 0, T(-1)) - r0 * at(v, 0, -1, 0, T(-1))) * d.inv_2dy +
                (rp * at(w, 0, 0, 1, T(-1)) - rm * at(w, 0, 0, -1, T(-1))) * d.inv_2dz;
  T val = at.prof(P.alpha0_t, 0) / d.dt * div;
  if (lag) {
    T corr = T(0);
    const T inv4[3] = {T(0.25) * d.inv_dx * d.inv_dx, T(0.25) * d.inv_dy * d.inv_dy,
                       T(0.25) * d.inv_dz * d.inv_dz};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const int di = ax == 0, dj = ax == 1, dk = ax == 2;
      const T a2 = at(lag, 2 * di, 2 * dj, 2 * dk, T(1));
      const T a1 = at(lag, di, dj, dk, T(1));
      const T a0 = at(lag, 0, 0, 0, T(1));
      const T b1 = at(lag, -di, -dj, -dk, T(1));
      const T b2 = at(lag, -2 * di, -2 * dj, -2 * dk, T(1));
      corr += (a2 - T(4) * a1 + T(6) * a0 - T(4) * b1 + b2) * inv4[ax];
    }
    val -= corr;
  }
  at.store(rhs, val, active);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void rhs_kernel(Grid g, ColMap m, Dyn<T> d, Profiles<T> P,
                                                     const T *__restrict__ u,
                                                     const T *__restrict__ v,
                                                     const T *__restrict__ w,
                                                     const T *__restrict__ lag,
                                                     T *__restrict__ rhs) {
  const ColWave c = col_wave(g, m);
  if (!c.valid) return;
  const ColPts<T> pts = col_pts<T>(g, c.i, c.j);
  for (int k = c.k0; k < c.k1; ++k) {
    if (k >= 2 && k + 2 < g.nz)
      rhs_level<T, false>(g, d, P, pts, k, c.active, u, v, w, lag, rhs);
    else
      rhs_level<T, true>(g, d, P, pts, k, c.active, u, v, w, lag, rhs);
  }
}

// rhs_out = rhs_in - mean (in and out may alias); FP64 partial sums of
// rhs_out^2; phi0 := 0 when given.
template <typename T>
__global__ __launch_bounds__(kBlock) void center_kernel(int64_t n, const T *in, T *out,
                                                        T *__restrict__ phi0,
                                                        const SolveCtl *__restrict__ ctl,
                                                        double *__restrict__ partials) {
  const T mean = (T)ctl->rhs_mean;
  double acc = 0.0;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x) {
    const T val = in[q] - mean;
    out[q] = val;
    acc += (double)val * (double)val;
    if (phi0) phi0[q] = T(0);
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// U^{k+1} = U_hat - dt rho0 grad_c phi (stored as velocity), p += rho0 (phi - mean).
// Column-marching.
template <typename T, bool EDGE>
__device__ __forceinline__ void project_level(const Grid &g, const Dyn<T> &d,
                                              const Profiles<T> &P, const ColPts<T> &pts, int k,
                                              bool active, T mean, const T *__restrict__ phi,
                                              T *__restrict__ u, T *__restrict__ v,
                                              T *__restrict__ w, T *__restrict__ p) {
  const Lvl<T, EDGE> at(g, pts, k);
  const T gx = (at(phi, 1, 0, 0, T(1)) - at(phi, -1, 0, 0, T(1))) * d.inv_2dx;
  const T gy = (at(phi, 0, 1, 0, T(1)) - at(phi, 0, -1, 0, T(1))) * d.inv_2dy;
  const T gz = (at(phi, 0, 0, 1, T(1)) - at(phi, 0, 0, -1, T(1))) * d.inv_2dz;
  const T uo = at(u, 0, 0, 0, T(1)) - d.dt * gx;
  const T vo = at(v, 0, 0, 0, T(1)) - d.dt * gy;
  const T wo = at(w, 0, 0, 0, T(1)) - d.dt * gz;
  const T po = at(p, 0, 0, 0, T(1)) + at.prof(P.rho0_t, 0) * (at(phi, 0, 0, 0, T(1)) - mean);
  at.store(u, uo, active);
  at.store(v, vo, active);
  at.store(w, wo, active);
  at.store(p, po, active);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void project_kernel(Grid g, ColMap m, Dyn<T> d,
                                                         Profiles<T> P,
                                                         const T *__restrict__ phi,
                                                         const SolveCtl *__restrict__ ctl,
                                                         T *__restrict__ u, T *__restrict__ v,
                                                         T *__restrict__ w, T *__restrict__ p) {
  const ColWave c = col_wave(g, m);
  if (!c.valid) return;
  const ColPts<T> pts = col_pts<T>(g, c.i, c.j);
  const T mean = (T)ctl->phi_mean;
  for (int k = c.k0; k < c.k1; ++k) {
    if (k >= 1 && k + 1 < g.nz)
      project_level<T, false>(g, d, P, pts, k, c.active, mean, phi, u, v, w, p);
    else
      project_level<T, true>(g, d, P, pts, k, c.active, mean, phi, u, v, w, p);
  }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void sub_mean_kernel(int64_t n, const T *__restrict__ in,
                                                          const SolveCtl *__restrict__ ctl,
                                                          T *__restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  out[q] = in[q] - (T)ctl->phi_mean;
}

template <typename T>
__global__ __launch_bounds__(kBlock) void extrapolate_kernel(Grid g, Profiles<T> P,
                                                             const T *__restrict__ p,
                                                             const T *__restrict__ pm,
                                                             T *__restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.n) return;
  out[q] = P.alpha0_t[(int)(q / g.nxy)] * (p[q] - pm[q]);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void block_sum_kernel(const T *__restrict__ a, int64_t n,
                                                           int mode, double *__restrict__ partials) {
  double acc = 0.0;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < n;
       q += (int64_t)gridDim.x * blockDim.x) {
    const double x = (double)a[q];
    acc += mode == 1 ? x * x : x;
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) partials[blockIdx.x] = s;
}

// One block of 1024 threads sums `np` partials in a fixed order and
// applies the operation to the control block.
__global__ __launch_bounds__(1024) void final_kernel(const double *__restrict__ partials, int np,
                                                     int op, SolveCtl *ctl, double n,
                                                     double tol2_scale, int m, double *out) {
  double acc = 0.0;
  for (int q = threadIdx.x; q < np; q += blockDim.x) acc += partials[q];
  double s = block_sum(acc);
  if (threadIdx.x != 0) return;
  switch (op) {
    case kFinalRhsMean:
      ctl->rhs_mean = s / n;
      break;
    case kFinalRhsNormRef:
    case kFinalRhsNorm:
      if (op == kFinalRhsNormRef) s = ctl->ref_norm2;
      ctl->rhs_norm2 = s;
      ctl->tol2 = tol2_scale * s;
      if (!isfinite(s)) {
        ctl->done = 2;
        ctl->stop_m = 0;
        ctl->res_norm2 = s;
      } else if (s == 0.0) {
        ctl->done = 1;
        ctl->stop_m = 0;
        ctl->res_norm2 = 0.0;
      }
      break;
    case kFinalCheck:
      check_decision(ctl, s, m);
      break;
    case kFinalPhiMean:
      ctl->phi_mean = s / n;
      break;
    case kFinalStore:
      out[0] = s;
      break;
    default:
      break;
  }
}

// Defect right-hand side of a starting iterate: rhs_d = rhs - L phi0 in
// FP64, with FP64 partial sums of rhs_d^2 (partials[b]) and of rhs^2
// (partials[gridDim.x + b]); L the compact Laplacian, periodic x, y and
// mirror z.
template <typename T>
__global__ __launch_bounds__(kBlock) void guess_residual_kernel(Grid g, double ix2, double iy2,
                                                                double iz2,
                                                                const T *__restrict__ rhs,
                                                                const T *__restrict__ phi0,
                                                                T *__restrict__ rhs_d,
                                                                double *__restrict__ partials) {
  double rr = 0.0, bb = 0.0;
  for (int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; q < g.n;
       q += (int64_t)gridDim.x * blockDim.x) {
    const int k = (int)(q / g.nxy);
    const int64_t r2 = q - g.nxy * k;
    const int j = (int)(r2 / g.nx);
    const int i = (int)(r2 - (int64_t)g.nx * j);
    const double c = phi0[q];
    const double lap =
        ((double)gload(phi0, g, i + 1, j, k, T(1)) + (double)gload(phi0, g, i - 1, j, k, T(1)) -
         2.0 * c) * ix2 +
        ((double)gload(phi0, g, i, j + 1, k, T(1)) + (double)gload(phi0, g, i, j - 1, k, T(1)) -
         2.0 * c) * iy2 +
        ((double)gload(phi0, g, i, j, k + 1, T(1)) + (double)gload(phi0, g, i, j, k - 1, T(1)) -
         2.0 * c) * iz2;
    const double b = rhs[q];
    const double d = b - lap;
    rhs_d[q] = (T)d;
    rr += d * d;
    bb += b * b;
  }
  const double sr = block_sum(rr);
  const double sb = block_sum(bb);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = sr;
    partials[gridDim.x + blockIdx.x] = sb;
  }
}

// ctl->guess_kept = 1 when the starting iterate's residual is below the
// zero start's (sum r^2 < sum rhs^2), else 0.
__global__ __launch_bounds__(1024) void guess_gate_kernel(const double *__restrict__ partials,
                                                          int np, SolveCtl *ctl) {
  double a = 0.0, b = 0.0;
  for (int q = threadIdx.x; q < np; q += blockDim.x) {
    a += partials[q];
    b += partials[np + q];
  }
  a = block_sum(a);
  b = block_sum(b);
  if (threadIdx.x == 0) {
    ctl->guess_kept = a < b ? 1 : 0;
    ctl->ref_norm2 = b;
  }
}

// A rejected starting iterate: the solve takes rhs itself from zero.
template <typename T>
__global__ __launch_bounds__(kBlock) void guess_clear_kernel(int64_t n,
                                                             const SolveCtl *__restrict__ ctl,
                                                             const T *__restrict__ rhs,
                                                             T *__restrict__ rhs_d) {
  if (ctl->guess_kept) return;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) rhs_d[q] = rhs[q];
}

template <typename T>
__global__ __launch_bounds__(kBlock) void add_guess_kernel(int64_t n,
                                                           const SolveCtl *__restrict__ ctl,
                                                           const T *__restrict__ phi0,
                                                           T *__restrict__ phi) {
  if (!ctl->guess_kept) return;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) phi[q] = (T)((double)phi[q] + (double)phi0[q]);
}

__global__ void ctl_reset_kernel(SolveCtl *ctl, int max_sweeps, int fixed) {
  if (threadIdx.x != 0) return;
  ctl->rhs_mean = 0.0;
  ctl->rhs_norm2 = 0.0;
  ctl->res_norm2 = 0.0;
  ctl->tol2 = 0.0;
  ctl->phi_mean = 0.0;
  ctl->aux = 0.0;
  ctl->done = 0;
  ctl->stop_m = -1;
  ctl->max_sweeps = max_sweeps;
  ctl->fixed = fixed;
}

}  // namespace

template <typename T>
void launch_poisson_rhs(const Grid &g, const Dyn<T> &d, const Profiles<T> &P, const T *u,
                        const T *v, const T *w, const T *phi_lag, T *rhs, double *partials,
                        hipStream_t s) {
  (void)partials;
  const ColMap m = col_map(g);
  rhs_kernel<T><<<m.blocks, kBlock, 0, s>>>(g, m, d, P, u, v, w, phi_lag, rhs);
}

template <typename T>
void launch_rhs_center(const Grid &g, const T *rhs_in, T *rhs_out, T *phi0, const SolveCtl *ctl,
                       double *partials, hipStream_t s) {
  center_kernel<T><<<kReduceBlocks, kBlock, 0, s>>>(g.n, rhs_in, rhs_out, phi0, ctl, partials);
}

template <typename T>
void launch_project(const Grid &g, const Dyn<T> &d, const Profiles<T> &P, const T *phi,
                    const SolveCtl *ctl, T *u, T *v, T *w, T *p, hipStream_t s) {
  const ColMap m = col_map(g);
  project_kernel<T><<<m.blocks, kBlock, 0, s>>>(g, m, d, P, phi, ctl, u, v, w, p);
}

template <typename T>
void launch_sub_mean(const Grid &g, const T *in, const SolveCtl *ctl, T *out, hipStream_t s) {
  sub_mean_kernel<T><<<blocks_for(g.n), kBlock, 0, s>>>(g.n, in, ctl, out);
}

template <typename T>
void launch_extrapolate(const Grid &g, const Profiles<T> &P, const T *p, const T *p_prev, T *phi0,
                        hipStream_t s) {
  extrapolate_kernel<T><<<blocks_for(g.n), kBlock, 0, s>>>(g, P, p, p_prev, phi0);
}

template <typename T>
void launch_guess_gate(const Grid &g, const T *rhs, const T *phi0, T *rhs_d, double *partials,
                       SolveCtl *ctl, hipStream_t s) {
  guess_residual_kernel<T><<<kReduceBlocks, kBlock, 0, s>>>(
      g, 1.0 / (g.dx * g.dx), 1.0 / (g.dy * g.dy), 1.0 / (g.dz * g.dz), rhs, phi0, rhs_d,
      partials);
  guess_gate_kernel<<<1, 1024, 0, s>>>(partials, kReduceBlocks, ctl);
  guess_clear_kernel<T><<<blocks_for(g.n), kBlock, 0, s>>>(g.n, ctl, rhs, rhs_d);
}

template <typename T>
void launch_add_guess(const Grid &g, const T *phi0, const SolveCtl *ctl, T *phi, hipStream_t s) {
  add_guess_kernel<T><<<blocks_for(g.n), kBlock, 0, s>>>(g.n, ctl, phi0, phi);
}

template <typename T>
void launch_block_sum(const T *a, int64_t n, int mode, double *partials, hipStream_t s) {
  block_sum_kernel<T><<<kReduceBlocks, kBlock, 0, s>>>(a, n, mode, partials);
}

void launch_final(const double *partials, int np, int op, SolveCtl *ctl, double n, double tol2_scale,
                  int m, double *out, hipStream_t s) {
  final_kernel<<<1, 1024, 0, s>>>(partials, np, op, ctl, n, tol2_scale, m, out);
}

void launch_ctl_reset(SolveCtl *ctl, int max_sweeps, int fixed, hipStream_t s) {
  ctl_reset_kernel<<<1, 64, 0, s>>>(ctl, max_sweeps, fixed);
}

#define LES_INST(T)                                                                              \
  template void launch_poisson_rhs<T>(const Grid &, const Dyn<T> &, const Profiles<T> &,         \
                                      const T *, const T *, const T *, const T *, T *, double *, \
                                      hipStream_t);                                              \
  template void launch_rhs_center<T>(const Grid &, const T *, T *, T *, const SolveCtl *,        \
                                     double *, hipStream_t);                                     \
  template void launch_project<T>(const Grid &, const Dyn<T> &, const Profiles<T> &, const T *,  \
                                  const SolveCtl *, T *, T *, T *, T *, hipStream_t);            \
  template void launch_sub_mean<T>(const Grid &, const T *, const SolveCtl *, T *, hipStream_t); \
  template void launch_block_sum<T>(const T *, int64_t, int, double *, hipStream_t);            \
  template void launch_guess_gate<T>(const Grid &, const T *, const T *, T *, double *,        \
                                     SolveCtl *, hipStream_t);                                   \
  template void launch_add_guess<T>(const Grid &, const T *, const SolveCtl *, T *, hipStream_t); \
  template void launch_extrapolate<T>(const Grid &, const Profiles<T> &, const T *, const T *,   \
                                      T *, hipStream_t);
LES_INST(float)
LES_INST(double)
#undef LES_INST

}  // namespace lesmi
