// Pressure-correction Poisson path (paper Sec. 2.4 and App. A): right-hand
// side with the collocated-grid correction, weighted-Jacobi sweeps with a
// fused FP64 residual norm, projection, and the fixed-order FP64 reductions
// that drive the device-side stopping test.
#include "les_device.h"

namespace lesmi {

namespace {

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// rhs = (alpha0/dt) div_c(rho0 u_hat) - C(phi_lag), with C the App. A
// fourth difference (wide minus compact Laplacian) of the previous
// sub-iteration's correction (phi_lag == nullptr: C = 0).
template <typename T>
__global__ __launch_bounds__(kBlock) void rhs_kernel(Grid g, Dyn<T> d, Profiles<T> P,
                                                     const T *__restrict__ u,
                                                     const T *__restrict__ v,
                                                     const T *__restrict__ w,
                                                     const T *__restrict__ lag,
                                                     T *__restrict__ rhs) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.n) return;
  const int k = (int)(q / g.nxy);
  const int64_t r = q - g.nxy * k;
  const int j = (int)(r / g.nx);
  const int i = (int)(r - (int64_t)g.nx * j);
  const T r0 = P.rho0_t[k];
  const T rm = pload(P.rho0_t, k - 1, g.nz), rp = pload(P.rho0_t, k + 1, g.nz);
  const T div = (r0 * gload(u, g, i + 1, j, k, T(-1)) - r0 * gload(u, g, i - 1, j, k, T(-1))) * d.inv_2dx +
                (r0 * gload(v, g, i, j + 1, k, T(-1)) - r0 * gload(v, g, i, j - 1, k, T(-1))) * d.inv_2dy +
                (rp * gload(w, g, i, j, k + 1, T(-1)) - rm * gload(w, g, i, j, k - 1, T(-1))) * d.inv_2dz;
  T val = P.alpha0_t[k] / d.dt * div;
  if (lag) {
    T corr = T(0);
    const T inv4[3] = {T(0.25) * d.inv_dx * d.inv_dx, T(0.25) * d.inv_dy * d.inv_dy,
                       T(0.25) * d.inv_dz * d.inv_dz};
#pragma unroll
    for (int ax = 0; ax < 3; ++ax) {
      const int di = ax == 0, dj = ax == 1, dk = ax == 2;
      const T a2 = gload(lag, g, i + 2 * di, j + 2 * dj, k + 2 * dk, T(1));
      const T a1 = gload(lag, g, i + di, j + dj, k + dk, T(1));
      const T a0 = gload(lag, g, i, j, k, T(1));
      const T b1 = gload(lag, g, i - di, j - dj, k - dk, T(1));
      const T b2 = gload(lag, g, i - 2 * di, j - 2 * dj, k - 2 * dk, T(1));
      corr += (a2 - T(4) * a1 + T(6) * a0 - T(4) * b1 + b2) * inv4[ax];
    }
    val -= corr;
  }
  rhs[q] = val;
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

// Logical tile of physical block b.  Workgroups are dealt to the 8 XCDs
// round-robin (b mod 8); this remap gives each XCD one contiguous range of
// tiles (x fastest, then y, then z chunk), so the y/z neighbours a tile
// reads were fetched into that XCD's L2 by its neighbours.
__device__ __forceinline__ int xcd_tile(int b, int nblocks) {
  const int per = nblocks >> 3;  // nblocks is a multiple of 8
  return (b & 7) * per + (b >> 3);
}

// One sweep of the compact 7-point operator (periodic x/y, mirror z):
//   r         = rhs - L phi = rhs - (N(phi) - D phi), N = off-diagonal sum
//   J(phi)    = phi - omega_j r / D          (weighted Jacobi)
//   Jacobi:     out = J(phi)
//   Chebyshev:  out = prev + omega_c (J(phi) - prev)   (out may alias prev)
// The residual and the update are formed in FP64 from the stored values and
// rounded once to the storage type: an FP32 update written as
// (N - rhs)/D - phi cancels catastrophically and its rounding error, the
// same from sweep to sweep, accumulates in the slow modes.
// CHECK: also FP64 partial sums of r^2 for the input iterate.
// Each thread owns one (i, j) column of a 64 x 4 tile and marches kc
// levels keeping phi(k-1), phi(k), phi(k+1) in registers.
template <typename T, bool CHEB, bool CHECK>
__global__ __launch_bounds__(kSweepTX *kSweepTY) void sweep_kernel(
    Grid g, int kc, int tiles_x, int tiles_y, int ntiles, double ix2, double iy2, double iz2,
    double diag, double inv_diag, double omega_j, double omega_c, const T *__restrict__ phi,
    const T *prev, T *out,
    const T *__restrict__ rhs, const SolveCtl *__restrict__ ctl, double *__restrict__ partials) {
  if (ctl->done) return;
  const int tile = xcd_tile(blockIdx.x, gridDim.x);
  double acc = 0.0;
  if (tile < ntiles) {
    const int tx = tile % tiles_x;
    const int rest = tile / tiles_x;
    const int ty = rest % tiles_y;
    const int tz = rest / tiles_y;
    const int i = tx * kSweepTX + (threadIdx.x & (kSweepTX - 1));
    const int j = ty * kSweepTY + (threadIdx.x / kSweepTX);
    if (i < g.nx && j < g.ny) {
      const int k0 = tz * kc;
      const int k1 = min(g.nz, k0 + kc);
      const int ip = i + 1 == g.nx ? 0 : i + 1, im = i == 0 ? g.nx - 1 : i - 1;
      const int jp = j + 1 == g.ny ? 0 : j + 1, jm = j == 0 ? g.ny - 1 : j - 1;
      const int64_t col = (int64_t)i + (int64_t)g.nx * j;
      const int64_t oxp = ip - i, oxm = im - i;
      const int64_t oyp = (int64_t)(jp - j) * g.nx, oym = (int64_t)(jm - j) * g.nx;
      T below = phi[col + g.nxy * (k0 > 0 ? k0 - 1 : 0)];
      T cur = phi[col + g.nxy * k0];
      for (int k = k0; k < k1; ++k) {
        const int64_t q = col + g.nxy * k;
        const T above = phi[q + (k + 1 < g.nz ? g.nxy : 0)];
        const double hx = (double)phi[q + oxp] + (double)phi[q + oxm];
        const double hy = (double)phi[q + oyp] + (double)phi[q + oym];
        const double hz = (double)above + (double)below;
        const double c0 = (double)cur;
        const double res = (double)rhs[q] - (hx * ix2 + hy * iy2 + hz * iz2 - diag * c0);
        if (CHECK) acc += res * res;
        const double jac = c0 - omega_j * res * inv_diag;
        if (CHEB) {
          const double pv = (double)prev[q];
          out[q] = (T)(pv + omega_c * (jac - pv));
        } else {
          out[q] = (T)jac;
        }
        below = cur;
        cur = above;
      }
    }
  }
  if (CHECK) {
    const double s = block_sum(acc);
    if (threadIdx.x == 0) partials[blockIdx.x] = s;
  }
}

// U^{k+1} = U_hat - dt rho0 grad_c phi (stored as velocity), p += rho0 (phi - mean).
template <typename T>
__global__ __launch_bounds__(kBlock) void project_kernel(Grid g, Dyn<T> d, Profiles<T> P,
                                                         const T *__restrict__ phi,
                                                         const SolveCtl *__restrict__ ctl,
                                                         T *__restrict__ u, T *__restrict__ v,
                                                         T *__restrict__ w, T *__restrict__ p) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.n) return;
  const int k = (int)(q / g.nxy);
  const int64_t r = q - g.nxy * k;
  const int j = (int)(r / g.nx);
  const int i = (int)(r - (int64_t)g.nx * j);
  const T gx = (gload(phi, g, i + 1, j, k, T(1)) - gload(phi, g, i - 1, j, k, T(1))) * d.inv_2dx;
  const T gy = (gload(phi, g, i, j + 1, k, T(1)) - gload(phi, g, i, j - 1, k, T(1))) * d.inv_2dy;
  const T gz = (gload(phi, g, i, j, k + 1, T(1)) - gload(phi, g, i, j, k - 1, T(1))) * d.inv_2dz;
  u[q] = u[q] - d.dt * gx;
  v[q] = v[q] - d.dt * gy;
  w[q] = w[q] - d.dt * gz;
  p[q] = p[q] + P.rho0_t[k] * (phi[q] - (T)ctl->phi_mean);
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
  const double s = block_sum(acc);
  if (threadIdx.x != 0) return;
  switch (op) {
    case kFinalRhsMean:
      ctl->rhs_mean = s / n;
      break;
    case kFinalRhsNorm:
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
      if (ctl->done) break;
      ctl->res_norm2 = s;
      if (!isfinite(s)) {
        ctl->done = 2;
        ctl->stop_m = m;
      } else if (ctl->fixed) {
        if (m >= ctl->max_sweeps) {
          ctl->done = s <= ctl->tol2 ? 1 : 3;
          ctl->stop_m = m;
        }
      } else if (s <= ctl->tol2) {
        ctl->done = 1;
        ctl->stop_m = m;
      } else if (m >= ctl->max_sweeps) {
        ctl->done = 3;
        ctl->stop_m = m;
      }
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

struct SweepShape {
  int kc, tiles_x, tiles_y, ntiles, blocks;
};

SweepShape sweep_shape(const Grid &g) {
  SweepShape s;
  s.tiles_x = (g.nx + kSweepTX - 1) / kSweepTX;
  s.tiles_y = (g.ny + kSweepTY - 1) / kSweepTY;
  s.kc = kSweepKC;
  for (;;) {
    const int tz = (g.nz + s.kc - 1) / s.kc;
    const int64_t nt = (int64_t)s.tiles_x * s.tiles_y * tz;
    if (nt <= kPartials || s.kc >= g.nz) {
      s.ntiles = (int)nt;
      break;
    }
    s.kc *= 2;
  }
  s.blocks = (s.ntiles + 7) / 8 * 8;
  return s;
}

}  // namespace

int sweep_grid_blocks(const Grid &g) { return sweep_shape(g).blocks; }

template <typename T>
void launch_poisson_rhs(const Grid &g, const Dyn<T> &d, const Profiles<T> &P, const T *u,
                        const T *v, const T *w, const T *phi_lag, T *rhs, double *partials,
                        hipStream_t s) {
  (void)partials;
  rhs_kernel<T><<<blocks_for(g.n), kBlock, 0, s>>>(g, d, P, u, v, w, phi_lag, rhs);
}

template <typename T>
void launch_rhs_center(const Grid &g, const T *rhs_in, T *rhs_out, T *phi0, const SolveCtl *ctl,
                       double *partials, hipStream_t s) {
  center_kernel<T><<<kReduceBlocks, kBlock, 0, s>>>(g.n, rhs_in, rhs_out, phi0, ctl, partials);
}

template <typename T>
void launch_sweep(const Grid &g, bool chebyshev, bool check, double omega_jacobi, double omega_cheb,
                  const T *phi, const T *prev, T *out, const T *rhs, const SolveCtl *ctl,
                  double *partials, hipStream_t s) {
  const SweepShape sh = sweep_shape(g);
  const double ix2 = 1.0 / (g.dx * g.dx), iy2 = 1.0 / (g.dy * g.dy), iz2 = 1.0 / (g.dz * g.dz);
  const double diag = 2.0 * (ix2 + iy2 + iz2), inv_diag = 1.0 / diag;
  const dim3 grid(sh.blocks), block(kSweepTX * kSweepTY);
#define LES_SWEEP(CH, CK)                                                                          \
  sweep_kernel<T, CH, CK><<<grid, block, 0, s>>>(g, sh.kc, sh.tiles_x, sh.tiles_y, sh.ntiles, ix2, \
                                                 iy2, iz2, diag, inv_diag, omega_jacobi,          \
                                                 omega_cheb, phi, prev, out, rhs, ctl, partials)
  if (chebyshev) {
    if (check) LES_SWEEP(true, true);
    else LES_SWEEP(true, false);
  } else {
    if (check) LES_SWEEP(false, true);
    else LES_SWEEP(false, false);
  }
#undef LES_SWEEP
}

template <typename T>
void launch_project(const Grid &g, const Dyn<T> &d, const Profiles<T> &P, const T *phi,
                    const SolveCtl *ctl, T *u, T *v, T *w, T *p, hipStream_t s) {
  project_kernel<T><<<blocks_for(g.n), kBlock, 0, s>>>(g, d, P, phi, ctl, u, v, w, p);
}

template <typename T>
void launch_sub_mean(const Grid &g, const T *in, const SolveCtl *ctl, T *out, hipStream_t s) {
  sub_mean_kernel<T><<<blocks_for(g.n), kBlock, 0, s>>>(g.n, in, ctl, out);
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
  template void launch_sweep<T>(const Grid &, bool, bool, double, double, const T *, const T *,  \
                                T *, const T *, const SolveCtl *, double *, hipStream_t);        \
  template void launch_project<T>(const Grid &, const Dyn<T> &, const Profiles<T> &, const T *,  \
                                  const SolveCtl *, T *, T *, T *, T *, hipStream_t);            \
  template void launch_sub_mean<T>(const Grid &, const T *, const SolveCtl *, T *, hipStream_t); \
  template void launch_block_sum<T>(const T *, int64_t, int, double *, hipStream_t);
LES_INST(float)
LES_INST(double)
#undef LES_INST

}  // namespace lesmi
