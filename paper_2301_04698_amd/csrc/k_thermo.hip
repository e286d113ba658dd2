// Per-cell moist thermodynamics (paper Sec. 2.1-2.2) and the radiative
// flux column (Sec. 2.1, theta_l equation).  The saturation adjustment
// always iterates in FP64, whatever the storage precision.
#include <algorithm>

#include "les.h"
#include "les_device.h"

namespace lesmi {

namespace {

// Saturation specific humidity over liquid (L = L_v0) or ice (L = L_s0):
// Clausius-Clapeyron with a constant latent heat anchored at the triple
// point (the paper cites the formula's source without printing it);
// q = eps e / (p0 - (1 - eps) e).
__device__ __forceinline__ double qsat_of(const Thermo &c, double L_over_Rv, double T, double p0) {
  const double e = c.e_tr * exp(L_over_Rv * (c.inv_Ttr - 1.0 / T));
  return c.eps * e / (p0 - (1.0 - c.eps) * e);
}

// Share of the condensate that is liquid: H(T - T_f) (H(0) = 1), or the
// linear ramp from T_ice to T_f for mixed-phase clouds.
__device__ __forceinline__ double liquid_fraction(const Thermo &c, double T) {
  if (c.phase == LES_PHASE_HEAVISIDE) return T >= c.Tf ? 1.0 : 0.0;
  const double lam = (T - c.T_ice) * c.inv_ramp;
  return lam < 0.0 ? 0.0 : (lam > 1.0 ? 1.0 : lam);
}

struct Phase {
  double ql, qi;
};

// Saturation humidity of the partition, lam q*(liquid) + (1 - lam) q*(ice)
// (the ice term only where some condensate is ice).
__device__ __forceinline__ double qstar(const Thermo &c, double lam, double T, double p0) {
  const double ql = qsat_of(c, c.Lv_over_Rv, T, p0);
  return lam == 1.0 ? ql : lam * ql + (1.0 - lam) * qsat_of(c, c.Ls_over_Rv, T, p0);
}

// q_c = max(0, q_t - q*), split as lam q_c liquid and the rest ice.
__device__ __forceinline__ Phase partition(const Thermo &c, double T, double qt, double p0) {
  const double lam = liquid_fraction(c, T);
  const double qc = fmax(0.0, qt - qstar(c, lam, T, p0));
  const double ql = lam * qc;
  return Phase{ql, qc - ql};
}

__device__ __forceinline__ double cp_moist(const Thermo &c, double qt, double ql, double qi) {
  return (1.0 - qt) * c.cpd + (qt - ql - qi) * c.cpv + ql * c.cl + qi * c.ci;
}

__device__ __forceinline__ double r_moist(const Thermo &c, double qt, double ql, double qi) {
  return (1.0 - qt) * c.Rd + (qt - ql - qi) * c.Rv;
}

// Exner function (p0/p00)^(R_m/c_pm) evaluated as exp(R_m/c_pm * ln(p0/p00)).
__device__ __forceinline__ double exner(const Thermo &c, double lnp, double qt, double ql,
                                        double qi) {
  return exp(r_moist(c, qt, ql, qi) / cp_moist(c, qt, ql, qi) * lnp);
}

// theta_l*(T) - theta_l at saturation partition (f), with that partition
// and its Exner function.
struct ThlResidual {
  double f, pi;
  Phase ph;
};
__device__ __forceinline__ ThlResidual thl_residual(const Thermo &c, double T, double thl,
                                                    double qt, double p0, double lnp) {
  const Phase ph = partition(c, T, qt, p0);
  const double cpm = cp_moist(c, qt, ph.ql, ph.qi);
  const double pi = exner(c, lnp, qt, ph.ql, ph.qi);
  return ThlResidual{T / pi * (1.0 - (c.Lv0 * ph.ql + c.Ls0 * ph.qi) / (cpm * T)) - thl, pi, ph};
}

// The adjusted state and the Exner function of its partition.
struct CellState {
  double T, ql, qi, pi;
};

// Saturation adjustment by the secant method (Sec. 2.2).  Unsaturated test
// first; otherwise secant from T_u and T_u + L_v0 (q_t - q_v*(T_u)) / c_pd,
// stopping at |dT| <= tol, equal residuals or the iteration cap.
__device__ CellState saturation_adjust(const Thermo &c, double thl, double qt, double p0,
                                       double lnp) {
  const double pu = exner(c, lnp, qt, 0.0, 0.0);
  const double tu = thl * pu;
  const double qs = qstar(c, liquid_fraction(c, tu), tu, p0);
  if (qt <= qs) return CellState{tu, 0.0, 0.0, pu};
  double ta = tu, tb = tu + c.Lv0 * (qt - qs) / c.cpd;
  double fa = thl_residual(c, ta, thl, qt, p0, lnp).f;
  ThlResidual rb = thl_residual(c, tb, thl, qt, p0, lnp);  // always that of the last tb
  for (int it = 0; it < c.satadj_maxit; ++it) {
    if (rb.f == fa) break;
    const double tn = tb - rb.f * (tb - ta) / (rb.f - fa);
    ta = tb;
    fa = rb.f;
    tb = tn;
    rb = thl_residual(c, tb, thl, qt, p0, lnp);
    if (fabs(tb - ta) <= c.satadj_tol) break;
  }
  return CellState{tb, rb.ph.ql, rb.ph.qi, rb.pi};
}

template <typename T>
__global__ __launch_bounds__(kBlock) void thermo_kernel(Grid g, Thermo c, Profiles<T> P,
                                                        const T *__restrict__ thl_a,
                                                        const T *__restrict__ qt_a,
                                                        const T *__restrict__ thl_b,
                                                        const T *__restrict__ qt_b,
                                                        T *__restrict__ thl_mid,
                                                        T *__restrict__ qt_mid, T *__restrict__ b,
                                                        T *__restrict__ ql, T *__restrict__ cpmpi,
                                                        T *__restrict__ Tout) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= g.n) return;
  const int k = (int)(q / g.nxy);
  T th = thl_a[q], qw = qt_a[q];
  if (thl_b) {
    // state midway between sub-iterate k and the step-start scalars
    th = T(0.5) * (th + thl_b[q]);
    qw = T(0.5) * (qw + qt_b[q]);
    if (thl_mid) thl_mid[q] = th;
    if (qt_mid) qt_mid[q] = qw;
  }
  const double p0 = P.p0[k], lnp = P.lnp[k], a0 = P.alpha0[k];
  const double qtd = (double)qw;
  const CellState s = saturation_adjust(c, (double)th, qtd, p0, lnp);
  if (b) {
    const double alpha = r_moist(c, qtd, s.ql, s.qi) * s.T / p0;
    b[q] = (T)(c.g * (alpha - a0) / a0);
  }
  if (ql) ql[q] = (T)s.ql;
  if (cpmpi) cpmpi[q] = (T)(cp_moist(c, qtd, s.ql, s.qi) * s.pi);
  if (Tout) Tout[q] = (T)s.T;
}

// Net upward flux F(z_f) = F0 exp(-kappa * sum_{cells above} rho0 q_l dz)
// and the heating -(c_pm Pi)^{-1} dF/dz of each cell, two launch forms.
//
// Many columns: one thread per (i, j) column marching down from the lid;
// consecutive threads take consecutive x, so every level is a coalesced row
// access.
template <typename T>
__global__ __launch_bounds__(kBlock) void radiation_kernel(Grid g, Profiles<T> P, double F0,
                                                           double kappa, const T *__restrict__ ql,
                                                           const T *__restrict__ cpmpi,
                                                           T *__restrict__ out) {
  const int64_t col = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (col >= g.nxy) return;
  double path = 0.0;
  double f_above = F0;
  for (int k = g.nz - 1; k >= 0; --k) {
    const int64_t q = col + g.nxy * k;
    path += P.rho0[k] * (double)ql[q] * g.dz;
    const double f_below = F0 * exp(-kappa * path);
    out[q] = (T)(-(f_above - f_below) / (g.dz * (double)cpmpi[q]));
    f_above = f_below;
  }
}

// Few columns (too few threads to hide the march's latency): a block owns
// the columns of one 64-wide x segment of a y row and its nw waves split
// their levels into chunks (wave w below wave w + 1).  Each wave sums the
// path of its chunk, the sums cross through LDS, and each wave then marches
// its chunk down from the path of the chunks above it; the top kRadRegs
// levels of a chunk stay in registers between the two passes, the rest are
// read again.
constexpr int kRadMaxWaves = 16, kRadRegs = 16;

// Below 4096 row segments (16 waves per CU marching whole columns) the
// chunked form, with chunks of about kRadRegs levels.
inline int rad_waves(const Grid &g) {
  const int64_t segs = (int64_t)((g.nx + 63) / 64) * g.ny;
  if (segs >= 4096) return 1;
  return std::min(kRadMaxWaves, std::max(1, (g.nz + kRadRegs - 1) / kRadRegs));
}

template <typename T>
__global__ __launch_bounds__(64 * kRadMaxWaves) void radiation_chunk_kernel(
    Grid g, Profiles<T> P, double F0, double kappa, const T *__restrict__ ql,
    const T *__restrict__ cpmpi, T *__restrict__ out) {
  __shared__ double part[kRadMaxWaves][64];
  const int lane = (int)(threadIdx.x & 63);
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int nw = (int)(blockDim.x >> 6);
  const int ntx = (g.nx + 63) / 64;
  const int tx = (int)(blockIdx.x % (unsigned)ntx);
  const int j = (int)(blockIdx.x / (unsigned)ntx);
  const int i = tx * 64 + lane;
  const bool active = i < g.nx;
  const int64_t col = (int64_t)(active ? i : g.nx - 1) + (int64_t)g.nx * j;
  const int len = (g.nz + nw - 1) / nw;
  const int k0 = min(g.nz, w * len), k1 = min(g.nz, k0 + len);
  const int n = k1 - k0;  // levels k1 - 1 - t, t = 0 .. n - 1, top down
  T v[kRadRegs];
  double sum = 0.0;
#pragma unroll
  for (int t = 0; t < kRadRegs; ++t) {
    if (t < n) {
      const int k = k1 - 1 - t;
      v[t] = ql[col + g.nxy * k];
      sum += P.rho0[k] * (double)v[t] * g.dz;
    }
  }
  for (int t = kRadRegs; t < n; ++t) {
    const int k = k1 - 1 - t;
    sum += P.rho0[k] * (double)ql[col + g.nxy * k] * g.dz;
  }
  part[w][lane] = sum;
  __syncthreads();
  double path = 0.0;
  for (int u = nw - 1; u > w; --u) path += part[u][lane];
  double f_above = F0 * exp(-kappa * path);
  auto level = [&](int k, T q_l) __attribute__((always_inline)) {
    const int64_t q = col + g.nxy * k;
    path += P.rho0[k] * (double)q_l * g.dz;
    const double f_below = F0 * exp(-kappa * path);
    if (active) out[q] = (T)(-(f_above - f_below) / (g.dz * (double)cpmpi[q]));
    f_above = f_below;
  };
#pragma unroll
  for (int t = 0; t < kRadRegs; ++t)
    if (t < n) level(k1 - 1 - t, v[t]);
  for (int t = kRadRegs; t < n; ++t) level(k1 - 1 - t, ql[col + g.nxy * (k1 - 1 - t)]);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void average_kernel(int64_t n, const T *__restrict__ a0,
                                                         const T *__restrict__ b0,
                                                         T *__restrict__ o0,
                                                         const T *__restrict__ a1,
                                                         const T *__restrict__ b1,
                                                         T *__restrict__ o1,
                                                         const T *__restrict__ a2,
                                                         const T *__restrict__ b2,
                                                         T *__restrict__ o2) {
  const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  o0[q] = T(0.5) * (a0[q] + b0[q]);
  o1[q] = T(0.5) * (a1[q] + b1[q]);
  o2[q] = T(0.5) * (a2[q] + b2[q]);
}

inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

template <typename T>
void launch_thermo(const Grid &g, const Thermo &c, const Profiles<T> &P, const T *thl_a,
                   const T *qt_a, const T *thl_b, const T *qt_b, T *thl_mid, T *qt_mid, T *b,
                   T *ql, T *cpmpi, T *Tout, hipStream_t s) {
  thermo_kernel<T><<<blocks_for(g.n), kBlock, 0, s>>>(g, c, P, thl_a, qt_a, thl_b, qt_b, thl_mid,
                                                        qt_mid, b, ql, cpmpi, Tout);
}

template <typename T>
void launch_radiation(const Grid &g, const Profiles<T> &P, double F0, double kappa, const T *ql,
                      const T *cpmpi, T *out, hipStream_t s) {
  const int nw = rad_waves(g);
  if (nw == 1) {
    radiation_kernel<T><<<blocks_for(g.nxy), kBlock, 0, s>>>(g, P, F0, kappa, ql, cpmpi, out);
  } else {
    const unsigned segs = (unsigned)(((g.nx + 63) / 64) * (int64_t)g.ny);
    radiation_chunk_kernel<T><<<segs, 64 * nw, 0, s>>>(g, P, F0, kappa, ql, cpmpi, out);
  }
}

template <typename T>
void launch_average(const Grid &g, const T *a0, const T *b0, T *o0, const T *a1, const T *b1, T *o1,
                    const T *a2, const T *b2, T *o2, hipStream_t s) {
  average_kernel<T><<<blocks_for(g.n), kBlock, 0, s>>>(g.n, a0, b0, o0, a1, b1, o1, a2, b2, o2);
}

#define LES_INST(T)                                                                             \
  template void launch_thermo<T>(const Grid &, const Thermo &, const Profiles<T> &, const T *,  \
                                 const T *, const T *, const T *, T *, T *, T *, T *, T *, T *, \
                                 hipStream_t);                                                  \
  template void launch_radiation<T>(const Grid &, const Profiles<T> &, double, double, const T *, \
                                    const T *, T *, hipStream_t);                               \
  template void launch_average<T>(const Grid &, const T *, const T *, T *, const T *, const T *, \
                                  T *, const T *, const T *, T *, hipStream_t);
LES_INST(float)
LES_INST(double)
#undef LES_INST

}  // namespace lesmi
