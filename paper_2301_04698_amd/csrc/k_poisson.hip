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
    // the horizontally uniform part of phi_lag, kept as an FP64 profile:
    // its fourth difference in z, rounded once
    val -= corr + at.prof(P.cbar_t, 0);
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

// Level decomposition of the per-level kernels: block (p, k) covers part p
// of level k's plane (lp parts per level).
struct LevelPart {
  int64_t b, e;
};
__device__ __forceinline__ LevelPart level_part(const Grid &g, int lp) {
  const int64_t chunk = (g.nxy + lp - 1) / lp;
  LevelPart r;
  r.b = (int64_t)blockIdx.x * chunk;
  r.e = r.b + chunk < g.nxy ? r.b + chunk : g.nxy;
  return r;
}

// FP64 sum of part p of level k of f into part[k * lp + p].
template <typename T>
__global__ __launch_bounds__(kBlock) void level_sum_kernel(Grid g, const T *__restrict__ f, int lp,
                                                           double *__restrict__ part) {
  const int k = blockIdx.y;
  const LevelPart r = level_part(g, lp);
  const T *row = f + (int64_t)k * g.nxy;
  double acc = 0.0;
  for (int64_t q = r.b + threadIdx.x; q < r.e; q += blockDim.x) acc += (double)row[q];
  const double s = block_sum(acc);
  if (threadIdx.x == 0) part[(int64_t)k * lp + blockIdx.x] = s;
}

// From the level partials of the raw rhs: its mean m (ctl->rhs_mean) and
// what the centring subtracts per level, rsub[k]: the level mean when the
// horizontally uniform part is solved exactly, else m.  Exact mode also
// solves that part, (pb_{k+1} - 2 pb_k + pb_{k-1}) / dz^2 = rb_k with
// rb_k = level mean - m and mirror ghosts: the face gradient is zero at the
// bottom wall and grows by dz rb_k across level k; pb has zero mean.  One
// block; the level sums are one wave per level, the running sums
// sequential in a fixed order over LDS chunks of kScan levels.
constexpr int kScan = 2048;
__global__ __launch_bounds__(256) void mean_mode_kernel(const double *__restrict__ part, int lp,
                                                        int nz, double nxy, double dz, int exact,
                                                        SolveCtl *ctl, double *__restrict__ rsub,
                                                        double *__restrict__ pb) {
  __shared__ double buf[kScan];
  __shared__ double bcast;
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int k = wv; k < nz; k += 4) {
    double s = 0.0;
    for (int q = lane; q < lp; q += 64) s += part[(int64_t)k * lp + q];
    s = wave_sum(s);
    if (lane == 0) rsub[k] = s / nxy;
  }
  __syncthreads();
  double t = 0.0;
  for (int k = threadIdx.x; k < nz; k += blockDim.x) t += rsub[k];
  t = block_sum(t);
  if (threadIdx.x == 0) {
    bcast = t / nz;
    ctl->rhs_mean = bcast;
  }
  __syncthreads();
  const double m = bcast;
  if (!exact) {
    for (int k = threadIdx.x; k < nz; k += blockDim.x) {
      rsub[k] = m;
      pb[k] = 0.0;
    }
    return;
  }
  double G = 0.0, p = 0.0, acc = 0.0;  // G, p: thread 0's running sums
  for (int c0 = 0; c0 < nz; c0 += kScan) {
    const int c1 = c0 + kScan < nz ? c0 + kScan : nz;
    for (int k = c0 + threadIdx.x; k < c1; k += blockDim.x) buf[k - c0] = rsub[k] - m;
    __syncthreads();
    if (threadIdx.x == 0)
      for (int k = c0; k < c1; ++k) {  // buf: rb_k in, pb_k out
        const double r = buf[k - c0];
        buf[k - c0] = p;
        G += dz * r;
        p += dz * G;
      }
    __syncthreads();
    for (int k = c0 + threadIdx.x; k < c1; k += blockDim.x) {
      pb[k] = buf[k - c0];
      acc += buf[k - c0];
    }
    __syncthreads();
  }
  acc = block_sum(acc);
  if (threadIdx.x == 0) bcast = acc / nz;
  __syncthreads();
  const double mp = bcast;
  for (int k = threadIdx.x; k < nz; k += blockDim.x) pb[k] -= mp;
}

// rhs_out = rhs_in - rsub[k], rounded once (in and out may alias); FP64
// partial sums of (rhs_in - m)^2, the norm of the centred right-hand side;
// phi0 := 0 when given.
template <typename T>
__global__ __launch_bounds__(kBlock) void center_kernel(Grid g, int lp, const T *in, T *out,
                                                        T *__restrict__ phi0,
                                                        const double *__restrict__ rsub,
                                                        const SolveCtl *__restrict__ ctl,
                                                        double *__restrict__ partials) {
  const int k = blockIdx.y;
  const LevelPart r = level_part(g, lp);
  const double m = ctl->rhs_mean, sub = rsub[k];
  const int64_t base = (int64_t)k * g.nxy;
  double acc = 0.0;
  for (int64_t q = base + r.b + threadIdx.x; q < base + r.e; q += blockDim.x) {
    const double x = (double)in[q];
    out[q] = (T)(x - sub);
    acc += (x - m) * (x - m);
    if (phi0) phi0[q] = T(0);
  }
  const double s = block_sum(acc);
  if (threadIdx.x == 0) partials[(int64_t)k * lp + blockIdx.x] = s;
}

// gbar[k] = level mean from the level partials (exact mode), else 0; and
// gbar[nz] = the overall mean (the mean of the level means).
__global__ __launch_bounds__(256) void level_mean_kernel(const double *__restrict__ part, int lp,
                                                         int nz, double nxy, int exact,
                                                         double *__restrict__ gbar) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int k = wv; k < nz; k += 4) {
    double s = 0.0;
    if (exact)
      for (int q = lane; q < lp; q += 64) s += part[(int64_t)k * lp + q];
    s = wave_sum(s);
    if (lane == 0) gbar[k] = s / nxy;
  }
  __syncthreads();
  double t = 0.0;
  for (int k = threadIdx.x; k < nz; k += blockDim.x) t += gbar[k];
  t = block_sum(t);
  if (threadIdx.x == 0) gbar[nz] = t / nz;
}

// Profiles of the horizontally uniform part pb of a solution (FP64 in,
// storage type out, each rounded once; even mirror across the walls):
// phigz = d_c pb / dz (projection), cbar = its App. A fourth difference in z
// (the next sub-iteration's right-hand side), and with add_p pbar += rho0
// pb.  Then pgz = d_c(alpha0 pbar)/dz (momentum predictor).  pb nullable
// (only pgz).  One block.
template <typename T>
__global__ __launch_bounds__(256) void mean_profiles_kernel(int nz, double dz,
                                                            const double *__restrict__ pb,
                                                            const double *__restrict__ rho0,
                                                            const double *__restrict__ alpha0,
                                                            int add_p, double *pbar,
                                                            T *__restrict__ phigz,
                                                            T *__restrict__ cbar,
                                                            T *__restrict__ pgz) {
  if (pb) {
    for (int k = threadIdx.x; k < nz; k += blockDim.x) {
      const double a2 = pb[zmirror(k + 2, nz)], a1 = pb[zmirror(k + 1, nz)], a0 = pb[k];
      const double b1 = pb[zmirror(k - 1, nz)], b2 = pb[zmirror(k - 2, nz)];
      phigz[k] = (T)((a1 - b1) / (2.0 * dz));
      cbar[k] = (T)((a2 - 4.0 * a1 + 6.0 * a0 - 4.0 * b1 + b2) / (4.0 * dz * dz));
      if (add_p) pbar[k] += rho0[k] * a0;
    }
    __syncthreads();
  }
  for (int k = threadIdx.x; k < nz; k += blockDim.x) {
    const int kp = zmirror(k + 1, nz), km = zmirror(k - 1, nz);
    pgz[k] = (T)((alpha0[kp] * pbar[kp] - alpha0[km] * pbar[km]) / (2.0 * dz));
  }
}

// ------------------------------------------------ vertically uniform part

// Vertical mean of every column: out[i + nx j] = mean over k of f (FP64,
// fixed order).  A block takes 64 consecutive columns; its four waves sum
// a quarter of the levels each (consecutive lanes read consecutive cells
// of a level), then the quarters are added in order.
template <typename T>
__global__ __launch_bounds__(256) void column_mean_kernel(Grid g, const T *__restrict__ f,
                                                          double *__restrict__ out) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, part = threadIdx.x >> 6;
  const int64_t q = (int64_t)blockIdx.x * 64 + lane;
  const int k0 = (int)((int64_t)part * g.nz / 4), k1 = (int)((int64_t)(part + 1) * g.nz / 4);
  double s = 0.0;
  if (q < g.nxy)
    for (int k = k0; k < k1; ++k) s += (double)f[q + g.nxy * k];
  red[part][lane] = s;
  __syncthreads();
  if (part == 0 && q < g.nxy) out[q] = (((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane]) / g.nz;
}

// One direction of the separable real Fourier (Hartley) transform of an
// ny x nx FP64 array a[j][i] (i fastest): along y (axis 1),
// out[ky][i] = sum_j cas(2 pi ky j / ny) a[j][i]; along x (axis 0),
// out[j][kx] = sum_i a[j][i] cas(2 pi i kx / nx).  cas values come from
// the table tab[m] = cas(2 pi m / n), m = 0 .. n-1, indexed by (k j) mod n,
// advanced incrementally.  out may subtract a constant first (sub, the
// mean of a; nullable).  A block takes 64 consecutive outputs; its four
// waves sum a quarter of the terms each, added in order at the end.
template <int AXIS>
__global__ __launch_bounds__(256) void hartley_kernel(int nx, int ny,
                                                      const double *__restrict__ a,
                                                      const double *__restrict__ tab,
                                                      const double *__restrict__ sub,
                                                      double *__restrict__ out) {
  __shared__ double red[4][64];
  const int lane = threadIdx.x & 63, part = threadIdx.x >> 6;
  const int64_t q = (int64_t)blockIdx.x * 64 + lane;
  const bool ok = q < (int64_t)nx * ny;
  const int row = ok ? (int)(q / nx) : 0, col = ok ? (int)(q - (int64_t)row * nx) : 0;
  const double c0 = sub ? *sub : 0.0;
  const int n = AXIS == 1 ? ny : nx;
  const int t0 = (int)((int64_t)part * n / 4), t1 = (int)((int64_t)(part + 1) * n / 4);
  double s = 0.0;
  if (ok) {
    if (AXIS == 1) {  // row = ky, col = i
      int m = (int)((int64_t)row * t0 % ny);
#pragma unroll 4
      for (int j = t0; j < t1; ++j) {
        s += tab[m] * (a[(int64_t)j * nx + col] - c0);
        m += row;
        if (m >= ny) m -= ny;
      }
    } else {  // row = j, col = kx
      int m = (int)((int64_t)col * t0 % nx);
      const double *ar = a + (int64_t)row * nx;
#pragma unroll 4
      for (int i = t0; i < t1; ++i) {
        s += (ar[i] - c0) * tab[m];
        m += col;
        if (m >= nx) m -= nx;
      }
    }
  }
  red[part][lane] = s;
  __syncthreads();
  if (part == 0 && ok) out[q] = ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// Divide the transform of the vertical-mean right-hand side by the
// eigenvalue of mode (kx, ky) of the x-y compact Laplacian (and by nx ny,
// the scale of the inverse transform); mode (0, 0) to zero.
__global__ __launch_bounds__(kBlock) void hartley_divide_kernel(int nx, int ny, double idx2,
                                                                double idy2,
                                                                double *__restrict__ b) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= (int64_t)nx * ny) return;
  const int ky = (int)(q / nx), kx = (int)(q - (int64_t)ky * nx);
  const double lam = -(2.0 - 2.0 * cospi(2.0 * kx / nx)) * idx2 -
                     (2.0 - 2.0 * cospi(2.0 * ky / ny)) * idy2;
  b[q] = (kx == 0 && ky == 0) ? 0.0 : b[q] / (lam * ((double)nx * ny));
}

// The sweeps' right-hand side with both uniform parts removed:
// out = rhs_level - (cmean[i,j] - mean), rhs_level the right-hand side
// without its level means, cmean the raw right-hand side's column means,
// mean its overall mean; FP64, rounded once.  out may alias rhs_level.
template <typename T>
__global__ __launch_bounds__(kBlock) void remove_columns_kernel(Grid g, const T *rhs_level,
                                                                const double *__restrict__ cmean,
                                                                const SolveCtl *__restrict__ ctl,
                                                                T *out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.n) return;
  const int64_t c = q % g.nxy;
  out[q] = (T)((double)rhs_level[q] - (cmean[c] - ctl->rhs_mean));
}

// The returned iterate of an exact-mode solve: the sweeps' correction d
// with its level means dbar[k], column means dv and overall mean dbar[nz]
// added back removed (each zero in exact arithmetic: it removes what
// rounding put there), plus the vertically uniform part pv, plus (when
// ctl->guess_kept and gs) the guess with its level means gbar[k] and
// column means gv removed and its overall mean gbar[nz] added back; FP64
// sum rounded once, in place.
template <typename T>
__global__ __launch_bounds__(kBlock) void combine_kernel(Grid g, T *phi,
                                                         const double *__restrict__ dbar,
                                                         const double *__restrict__ dv,
                                                         const double *__restrict__ pv,
                                                         const T *__restrict__ gs,
                                                         const double *__restrict__ gbar,
                                                         const double *__restrict__ gv,
                                                         const SolveCtl *__restrict__ ctl) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.n) return;
  const int k = (int)(q / g.nxy);
  const int64_t c = q - g.nxy * k;
  // dbar[nz], gbar[nz]: the overall means
  double v = (double)phi[q] - dbar[k] - dv[c] + dbar[g.nz] + pv[c];
  if (gs && ctl->guess_kept) v += (double)gs[q] - gbar[k] - gv[c] + gbar[g.nz];
  phi[q] = (T)v;
}

// out = in - ctl->phi_mean (if ctl) + prof[k], in FP64, rounded once.
template <typename T>
__global__ __launch_bounds__(kBlock) void add_profile_kernel(Grid g, const T *__restrict__ in,
                                                             const SolveCtl *__restrict__ ctl,
                                                             const double *__restrict__ prof,
                                                             T *__restrict__ out) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.n) return;
  const double mean = ctl ? ctl->phi_mean : 0.0;
  out[q] = (T)((double)in[q] - mean + prof[(int)(q / g.nxy)]);
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
  const T gz = (at(phi, 0, 0, 1, T(1)) - at(phi, 0, 0, -1, T(1))) * d.inv_2dz +
               at.prof(P.phigz_t, 0);
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
      check_decision(ctl, s, m);
      break;
    case kFinalPhiMean:
      ctl->phi_mean = s / n;
      break;
    case kFinalStore:
      out[0] = s;
      break;
    case kFinalReturned:
      ctl->res_out2 = s;
      break;
    default:
      break;
  }
}

// Defect right-hand side of a starting iterate: rhs_d = rhs - L (phi0 -
// gbar - gv) in FP64 (gbar: per-level means, gv: per-column means to
// remove, nullable; a constant drops out of L), with FP64 partial sums of
// rhs_d^2 (partials[b]) and of rhs^2 (partials[gridDim.x + b]); L the
// compact Laplacian, periodic x, y and mirror z.  rhs_d nullable (only the
// sums: the residual of a returned iterate); rhs_d may alias rhs.  With
// `when`, only if when->guess_kept (and then the partial sums are not
// written either).  GBAR, GV: gbar, gv are given (compile-time, so that
// the loads of several rows are in flight together).
template <typename T, bool GBAR, bool GV>
__global__ __launch_bounds__(kBlock) void guess_residual_kernel(Grid g, double ix2, double iy2,
                                                                double iz2, const T *rhs,
                                                                const T *__restrict__ phi0,
                                                                const double *__restrict__ gbar,
                                                                const double *__restrict__ gv,
                                                                T *rhs_d,
                                                                double *__restrict__ partials,
                                                                const SolveCtl *__restrict__ when) {
  if (when && !when->guess_kept) return;
  double rr = 0.0, bb = 0.0;
  // each block takes a run of x rows (xcd_rows), four at a time so that
  // their loads are in flight together (rows past the run repeat its first
  // row and are not counted); a row's level and y index (and its neighbour
  // rows) are uniform over the block
  const int64_t rows = (int64_t)g.ny * g.nz;
  constexpr int R = 4;
  const RowRange run = xcd_rows(rows);
  // (level, y row) of row r0 + u, stepped without divisions
  const RowStep rs(g.ny, 1);
  RowPos p0 = rs.at(run.r0);
  for (int64_t r0 = run.r0; r0 < run.r1; r0 += R) {
    RowPos pu[R];
    pu[0] = p0;
#pragma unroll
    for (int u = 1; u < R; ++u) pu[u] = rs.next(pu[u - 1]);
    p0 = rs.next(pu[R - 1]);
    for (int i = threadIdx.x; i < g.nx; i += blockDim.x) {
      const int ip = i + 1 < g.nx ? i + 1 : 0, im = i > 0 ? i - 1 : g.nx - 1;
      double dv[R], bv[R];
#pragma unroll
      for (int u = 0; u < R; ++u) {
        const bool in = r0 + u < run.r1;
        const int64_t row = in ? r0 + u : r0;
        const RowPos q = in ? pu[u] : pu[0];
        const int k = q.k, j = q.j;
        const int jp = pwrap(j + 1, g.ny), jm = pwrap(j - 1, g.ny);
        const int kp = zmirror(k + 1, g.nz), km = zmirror(k - 1, g.nz);
        const T *c0 = phi0 + row * g.nx;
        const T *yp = phi0 + ((int64_t)k * g.ny + jp) * g.nx;
        const T *ym = phi0 + ((int64_t)k * g.ny + jm) * g.nx;
        const T *zp = phi0 + ((int64_t)kp * g.ny + j) * g.nx;
        const T *zm = phi0 + ((int64_t)km * g.ny + j) * g.nx;
        const double gz = GBAR ? (gbar[kp] - 2.0 * gbar[k] + gbar[km]) * iz2 : 0.0;
        const double c = c0[i];
        double lap = ((double)c0[ip] + (double)c0[im] - 2.0 * c) * ix2 +
                     ((double)yp[i] + (double)ym[i] - 2.0 * c) * iy2 +
                     ((double)zp[i] + (double)zm[i] - 2.0 * c) * iz2;
        lap -= gz;
        if constexpr (GV) {  // the x-y second differences of the guess's column means
          const double gc = gv[(int64_t)i + g.sy * j];
          lap -= (gv[ip + g.sy * j] + gv[im + g.sy * j] - 2.0 * gc) * ix2 +
                 (gv[i + g.sy * jp] + gv[i + g.sy * jm] - 2.0 * gc) * iy2;
        }
        bv[u] = rhs[row * g.nx + i];
        dv[u] = bv[u] - lap;
      }
#pragma unroll
      for (int u = 0; u < R; ++u) {
        const int64_t row = r0 + u;
        if (row < run.r1) {
          if (rhs_d) rhs_d[row * g.nx + i] = (T)dv[u];
          rr += dv[u] * dv[u];
          bb += bv[u] * bv[u];
        }
      }
    }
  }
  const double sr = block_sum(rr);
  const double sb = block_sum(bb);
  if (threadIdx.x == 0) {
    partials[blockIdx.x] = sr;
    partials[gridDim.x + blockIdx.x] = sb;
  }
}

// ctl->guess_kept = 1 when the starting iterate's residual is below the
// zero start's (sum r^2 < sum rhs^2) or always_keep, else 0.
__global__ __launch_bounds__(1024) void guess_gate_kernel(const double *__restrict__ partials,
                                                          int np, int always_keep, SolveCtl *ctl) {
  double a = 0.0, b = 0.0;
  for (int q = threadIdx.x; q < np; q += blockDim.x) {
    a += partials[q];
    b += partials[np + q];
  }
  a = block_sum(a);
  b = block_sum(b);
  if (threadIdx.x == 0) {
    ctl->guess_kept = (always_keep || a < b) ? 1 : 0;
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

// phi += phi0 - gbar[k] (gbar nullable), FP64 sum rounded once.
template <typename T>
__global__ __launch_bounds__(kBlock) void add_guess_kernel(Grid g,
                                                           const SolveCtl *__restrict__ ctl,
                                                           const T *__restrict__ phi0,
                                                           const double *__restrict__ gbar,
                                                           T *__restrict__ phi) {
  if (!ctl->guess_kept) return;
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.n) return;
  const double gb = gbar ? gbar[(int)(q / g.nxy)] : 0.0;
  phi[q] = (T)((double)phi[q] + ((double)phi0[q] - gb));
}

template <typename T>
__global__ __launch_bounds__(kBlock) void zero_kernel(int64_t n, T *__restrict__ f) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q < n) f[q] = T(0);
}

// A second pass of sweeps on the same right-hand side (the zero start after
// a kept guess reached the cap): the reference norm and tolerance stay.
__global__ void ctl_restart_kernel(SolveCtl *ctl, int max_sweeps) {
  if (threadIdx.x != 0) return;
  ctl->max_sweeps = max_sweeps;
  ctl->done = 0;
  ctl->stop_m = -1;
  ctl->res_norm2 = 0.0;
  ctl->guess_kept = 0;
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

int level_parts(const Grid &g) {
  int64_t lp = g.nxy / 8192;
  if (lp > 64) lp = 64;
  if (lp * g.nz > kPartials) lp = kPartials / g.nz;
  return lp < 1 ? 1 : (int)lp;
}

template <typename T>
void launch_level_sum(const Grid &g, const T *f, double *part, hipStream_t s) {
  const int lp = level_parts(g);
  level_sum_kernel<T><<<dim3(lp, g.nz), kBlock, 0, s>>>(g, f, lp, part);
}

void launch_mean_mode(const Grid &g, const double *part, int exact, SolveCtl *ctl, double *rsub,
                      double *pb, hipStream_t s) {
  mean_mode_kernel<<<1, 256, 0, s>>>(part, level_parts(g), g.nz, (double)g.nxy, g.dz, exact, ctl,
                                     rsub, pb);
}

void launch_level_mean(const Grid &g, const double *part, int exact, double *gbar, hipStream_t s) {
  level_mean_kernel<<<1, 256, 0, s>>>(part, level_parts(g), g.nz, (double)g.nxy, exact, gbar);
}

template <typename T>
void launch_mean_profiles(const Grid &g, const double *pb, const double *rho0,
                          const double *alpha0, int add_p, double *pbar, T *phigz, T *cbar,
                          T *pgz, hipStream_t s) {
  mean_profiles_kernel<T><<<1, 256, 0, s>>>(g.nz, g.dz, pb, rho0, alpha0, add_p, pbar, phigz,
                                            cbar, pgz);
}

template <typename T>
void launch_add_profile(const Grid &g, const T *in, const SolveCtl *ctl, const double *prof,
                        T *out, hipStream_t s) {
  add_profile_kernel<T><<<blocks_for(g.n), kBlock, 0, s>>>(g, in, ctl, prof, out);
}

template <typename T>
void launch_rhs_center(const Grid &g, const T *rhs_in, T *rhs_out, T *phi0, const double *rsub,
                       const SolveCtl *ctl, double *partials, hipStream_t s) {
  const int lp = level_parts(g);
  center_kernel<T><<<dim3(lp, g.nz), kBlock, 0, s>>>(g, lp, rhs_in, rhs_out, phi0, rsub, ctl,
                                                     partials);
}

template <typename T>
void launch_column_mean(const Grid &g, const T *f, double *out, hipStream_t s) {
  column_mean_kernel<T><<<(unsigned)((g.nxy + 63) / 64), 256, 0, s>>>(g, f, out);
}

void launch_vertical_solve(const Grid &g, const double *cmean, const SolveCtl *ctl,
                           const double *tab_x, const double *tab_y, double *work, double *pv,
                           hipStream_t s) {
  const int nx = g.nx, ny = g.ny;
  const unsigned nb = blocks_for((int64_t)nx * ny);
  const unsigned nb64 = (unsigned)(((int64_t)nx * ny + 63) / 64);
  // rv = cmean - mean; a = Hy rv; b = a Hx / lambda; a = Hy b; pv = a Hx
  hartley_kernel<1><<<nb64, 256, 0, s>>>(nx, ny, cmean, tab_y, &ctl->rhs_mean, work);
  hartley_kernel<0><<<nb64, 256, 0, s>>>(nx, ny, work, tab_x, nullptr, pv);
  hartley_divide_kernel<<<nb, kBlock, 0, s>>>(nx, ny, 1.0 / (g.dx * g.dx), 1.0 / (g.dy * g.dy),
                                              pv);
  hartley_kernel<1><<<nb64, 256, 0, s>>>(nx, ny, pv, tab_y, nullptr, work);
  hartley_kernel<0><<<nb64, 256, 0, s>>>(nx, ny, work, tab_x, nullptr, pv);
}

template <typename T>
void launch_remove_columns(const Grid &g, const T *rhs_level, const double *cmean,
                           const SolveCtl *ctl, T *out, hipStream_t s) {
  remove_columns_kernel<T><<<blocks_for(g.n), kBlock, 0, s>>>(g, rhs_level, cmean, ctl, out);
}

template <typename T>
void launch_combine(const Grid &g, T *phi, const double *dbar, const double *dv, const double *pv,
                    const T *guess, const double *gbar, const double *gv, const SolveCtl *ctl,
                    hipStream_t s) {
  combine_kernel<T><<<blocks_for(g.n), kBlock, 0, s>>>(g, phi, dbar, dv, pv, guess, gbar, gv, ctl);
}

void launch_ctl_restart(SolveCtl *ctl, int max_sweeps, hipStream_t s) {
  ctl_restart_kernel<<<1, 64, 0, s>>>(ctl, max_sweeps);
}

__global__ void ctl_limit_kernel(SolveCtl *ctl, int max_sweeps) {
  if (threadIdx.x == 0) ctl->max_sweeps = max_sweeps;
}

void launch_ctl_limit(SolveCtl *ctl, int max_sweeps, hipStream_t s) {
  ctl_limit_kernel<<<1, 64, 0, s>>>(ctl, max_sweeps);
}

template <typename T>
void launch_zero(const Grid &g, T *f, hipStream_t s) {
  zero_kernel<T><<<blocks_for(g.n), kBlock, 0, s>>>(g.n, f);
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

// Blocks of the guess/returned-residual kernel: one x row each at a time,
// enough of them to keep every CU's memory pipes busy; 2 x 4096 partials fit
// the partial buffer.
constexpr int kResidualBlocks = 4096;
static_assert(2 * kResidualBlocks <= kPartials, "residual partials exceed the buffer");

// guess_residual_kernel with its GBAR, GV variant picked from gbar, gv.
template <typename T>
void launch_residual_pass(const Grid &g, const T *rhs, const T *phi0, const double *gbar,
                          const double *gv, T *rhs_d, double *partials, const SolveCtl *when,
                          hipStream_t s) {
  const double ix2 = 1.0 / (g.dx * g.dx), iy2 = 1.0 / (g.dy * g.dy), iz2 = 1.0 / (g.dz * g.dz);
#define LES_RES(GB, GV)                                                            \
  guess_residual_kernel<T, GB, GV><<<kResidualBlocks, kBlock, 0, s>>>(g, ix2, iy2, iz2, rhs, \
                                                                      phi0, gbar, gv, rhs_d, \
                                                                      partials, when)
  if (gbar && gv) LES_RES(true, true);
  else if (gbar) LES_RES(true, false);
  else if (gv) LES_RES(false, true);
  else LES_RES(false, false);
#undef LES_RES
}

template <typename T>
void launch_guess_gate(const Grid &g, const T *rhs, const T *phi0, const double *gbar,
                       const double *gv, T *rhs_d, double *partials, SolveCtl *ctl,
                       int always_keep, hipStream_t s) {
  if (rhs != rhs_d) {
    launch_residual_pass<T>(g, rhs, phi0, gbar, gv, rhs_d, partials, nullptr, s);
    guess_gate_kernel<<<1, 1024, 0, s>>>(partials, kResidualBlocks, always_keep, ctl);
    guess_clear_kernel<T><<<blocks_for(g.n), kBlock, 0, s>>>(g.n, ctl, rhs, rhs_d);
  } else {  // in place: the sums, the gate, then the defect if the guess is kept
    launch_residual_pass<T>(g, rhs, phi0, gbar, gv, nullptr, partials, nullptr, s);
    guess_gate_kernel<<<1, 1024, 0, s>>>(partials, kResidualBlocks, always_keep, ctl);
    launch_residual_pass<T>(g, rhs, phi0, gbar, gv, rhs_d, partials, ctl, s);
  }
}

template <typename T>
void launch_returned_residual(const Grid &g, const T *rhs, const T *phi, double *partials,
                              SolveCtl *ctl, hipStream_t s) {
  launch_residual_pass<T>(g, rhs, phi, nullptr, nullptr, nullptr, partials, nullptr, s);
  final_kernel<<<1, 1024, 0, s>>>(partials, kResidualBlocks, kFinalReturned, ctl, 0.0, 0.0, 0,
                                  nullptr);
}

template <typename T>
void launch_add_guess(const Grid &g, const T *phi0, const double *gbar, const SolveCtl *ctl,
                      T *phi, hipStream_t s) {
  add_guess_kernel<T><<<blocks_for(g.n), kBlock, 0, s>>>(g, ctl, phi0, gbar, phi);
}

template <typename T>
void launch_block_sum(const T *a, int64_t n, int mode, double *partials, hipStream_t s) {
  block_sum_kernel<T><<<kReduceBlocks, kBlock, 0, s>>>(a, n, mode, partials);
}

__global__ void snap_kernel(const SolveCtl *__restrict__ ctl, int64_t *snap, int seq) {
  if (threadIdx.x == 0) *(volatile int64_t *)snap = ((int64_t)seq << 32) | (uint32_t)ctl->done;
}

void launch_final_check(const double *partials, int np, SolveCtl *ctl, double n, int m,
                        int64_t *snap, int snap_seq, hipStream_t s) {
  final_kernel<<<1, 1024, 0, s>>>(partials, np, kFinalCheck, ctl, n, 0.0, m, nullptr);
  if (snap) snap_kernel<<<1, 64, 0, s>>>(ctl, snap, snap_seq);
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
  template void launch_rhs_center<T>(const Grid &, const T *, T *, T *, const double *,        \
                                     const SolveCtl *, double *, hipStream_t);                   \
  template void launch_level_sum<T>(const Grid &, const T *, double *, hipStream_t);           \
  template void launch_zero<T>(const Grid &, T *, hipStream_t);                                 \
  template void launch_column_mean<T>(const Grid &, const T *, double *, hipStream_t);          \
  template void launch_remove_columns<T>(const Grid &, const T *, const double *,               \
                                         const SolveCtl *, T *, hipStream_t);                   \
  template void launch_combine<T>(const Grid &, T *, const double *, const double *,            \
                                  const double *, const T *, const double *, const double *,    \
                                  const SolveCtl *, hipStream_t);                               \
  template void launch_mean_profiles<T>(const Grid &, const double *, const double *,          \
                                        const double *, int, double *, T *, T *, T *,          \
                                        hipStream_t);                                          \
  template void launch_add_profile<T>(const Grid &, const T *, const SolveCtl *, const double *, \
                                      T *, hipStream_t);                                       \
  template void launch_returned_residual<T>(const Grid &, const T *, const T *, double *,       \
                                            SolveCtl *, hipStream_t);                          \
  template void launch_project<T>(const Grid &, const Dyn<T> &, const Profiles<T> &, const T *,  \
                                  const SolveCtl *, T *, T *, T *, T *, hipStream_t);            \
  template void launch_sub_mean<T>(const Grid &, const T *, const SolveCtl *, T *, hipStream_t); \
  template void launch_block_sum<T>(const T *, int64_t, int, double *, hipStream_t);            \
  template void launch_guess_gate<T>(const Grid &, const T *, const T *, const double *,        \
                                     const double *, T *, double *, SolveCtl *, int,             \
                                     hipStream_t);                                               \
  template void launch_add_guess<T>(const Grid &, const T *, const double *, const SolveCtl *,   \
                                    T *, hipStream_t);                                           \
  template void launch_extrapolate<T>(const Grid &, const Profiles<T> &, const T *, const T *,   \
                                      T *, hipStream_t);
LES_INST(float)
LES_INST(double)
#undef LES_INST

}  // namespace lesmi
