// Internal declarations of the HIP LES library: grid/physics parameter
// blocks passed to kernels by value, the Poisson control block kept in the
// workspace, and the host-side launchers implemented in the kernel files.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace lesmi {

// Grid geometry.  Index of cell (i, j, k) is i + nx*(j + ny*k).
struct Grid {
  int nx, ny, nz;
  int64_t nxy, n;
  int64_t sy;  // row stride of the periodic y wrap: nx, or 0 when ny == 1
  double dx, dy, dz, dt;
};

// Constants needed by the per-cell thermodynamics (always FP64).
struct Thermo {
  double p00, Rd, Rv, cpd, cpv, cl, ci, Lv0, Ls0, Tf, g;
  double e_tr, inv_Ttr, Lv_over_Rv, Ls_over_Rv, eps;  // saturation vapour pressure
  double T_ice, inv_ramp;  // LES_PHASE_RAMP: liquid share (T - T_ice) / (Tf - T_ice)
  double satadj_tol;
  int satadj_maxit;
  int phase;               // LES_PHASE_HEAVISIDE or LES_PHASE_RAMP
};

// Vertical profiles (device pointers, nz entries each).
template <typename T>
struct Profiles {
  const double *p0, *lnp, *alpha0, *rho0;   // FP64: ln(p0/p00) feeds the Exner power
  const T *rho0_t, *alpha0_t, *beta_t, *wsub_t;
  // terms of the horizontally uniform part of phi and p' (kept as FP64
  // profiles, each term rounded once): d_c(alpha0 pbar)/dz for the momentum
  // predictor, the App. A fourth difference of the previous sub-iteration's
  // part for the right-hand side, d_c(phibar)/dz for the projection; all
  // zero when that part is swept with the rest
  const T *pgz_t, *cbar_t, *phigz_t;
};

// Parameters of the dynamics kernels in storage precision.
template <typename T>
struct Dyn {
  T dt, inv_dx, inv_dy, inv_dz, inv_2dx, inv_2dy, inv_2dz;
  T fcor, ug, vg;
  T inv_pr, inv_sc;
  T sfc_thl, sfc_qt;   // surface flux per unit area (rho0-weighted) into the lowest cell
  T smag_l2;           // (c_s Delta)^2
  T pr;                // turbulent Prandtl number of the buoyancy factor
  int advection;       // LES_QUICK or LES_WENO3
  T uv_par;            // wall parity of u and v: -1 no-slip, +1 free-slip
  T nu_const;          // > 0: uniform viscosity in place of the SGS model
};

// Device-resident control block of one Poisson solve.  Sweep kernels read
// `done` and return at once when it is set, so the host can queue sweeps
// ahead of the convergence test without synchronizing.
struct SolveCtl {
  double rhs_mean;    // mean of the raw rhs
  double rhs_norm2;   // ||rhs||^2 after mean removal
  double res_norm2;   // residual^2 of the last checked iterate
  double tol2;        // tol^2 * rhs_norm2
  double phi_mean;    // mean of the returned iterate
  double aux;
  int32_t done;       // 0 running, 1 converged, 2 non-finite, 3 cap reached
  int32_t stop_m;     // sweep index of the returned iterate
  int32_t max_sweeps;
  int32_t fixed;      // 1: stop at max_sweeps whatever the residual
  int32_t guess_kept; // starting-iterate test (not reset by a solve): 1 kept
  int32_t pad;
  double res_out2;    // residual^2 of a guessed solve's returned iterate
};

constexpr int kBlock = 256;          // threads per block of elementwise kernels
constexpr int kReduceBlocks = 1024;  // fixed grid of the generic reductions
constexpr int kPartials = 1 << 16;   // max partials of one reduction (sweep tiles)

// Temporally blocked Poisson sweeps: up to kMaxSweepsPerLaunch sweeps per
// launch (kDefaultSweepsPerLaunch unless the configuration asks otherwise).
constexpr int kMaxSweepsPerLaunch = 2;
constexpr int kDefaultSweepsPerLaunch = 1;

// Blocks of a tsweep launch of S sweeps (its count of residual partials).
int tsweep_blocks(const Grid &g, int S, bool is_double);

// ------------------------------------------------------------ launchers
template <typename T>
void launch_thermo(const Grid &g, const Thermo &c, const Profiles<T> &P, const T *thl_a,
                   const T *qt_a, const T *thl_b, const T *qt_b, T *thl_mid, T *qt_mid, T *b,
                   T *ql, T *cpmpi, T *Tout, hipStream_t s);

template <typename T>
void launch_radiation(const Grid &g, const Profiles<T> &P, double F0, double kappa, const T *ql,
                      const T *cpmpi, T *out, hipStream_t s);

template <typename T>
void launch_average(const Grid &g, const T *a0, const T *b0, T *o0, const T *a1, const T *b1, T *o1,
                    const T *a2, const T *b2, T *o2, hipStream_t s);

template <typename T>
void launch_sgs_nu(const Grid &g, const Dyn<T> &d, const T *u, const T *v, const T *w, const T *b,
                   T *nu, hipStream_t s);

template <typename T>
void launch_scalar_update(const Grid &g, const Dyn<T> &d, const Profiles<T> &P, const T *u,
                          const T *v, const T *w, const T *thl_mid, const T *qt_mid,
                          const T *thl_half, const T *qt_half, const T *nu, const T *rad,
                          T *thl_out, T *qt_out, hipStream_t s);

template <typename T>
void launch_momentum(const Grid &g, const Dyn<T> &d, const Profiles<T> &P, const T *uh,
                     const T *vh, const T *wh, const T *un, const T *vn, const T *wn, const T *p,
                     const T *b, const T *nu, T *uo, T *vo, T *wo, hipStream_t s);

template <typename T>
void launch_poisson_rhs(const Grid &g, const Dyn<T> &d, const Profiles<T> &P, const T *u,
                        const T *v, const T *w, const T *phi_lag, T *rhs, double *partials,
                        hipStream_t s);

// Per-level kernels split each level's plane into level_parts(g) parts
// (level_parts(g) * nz <= kPartials partial sums).
int level_parts(const Grid &g);
// part[k * level_parts + p] = FP64 sum of part p of level k of f.
template <typename T>
void launch_level_sum(const Grid &g, const T *f, double *part, hipStream_t s);
// From the level sums of a raw right-hand side: ctl->rhs_mean, the
// per-level value the centring subtracts (rsub: level mean if exact, else
// the mean) and, if exact, the FP64 solution pb of the horizontally uniform
// part (zero otherwise).
void launch_mean_mode(const Grid &g, const double *part, int exact, SolveCtl *ctl, double *rsub,
                      double *pb, hipStream_t s);
// gbar[k] = level mean from the level sums if exact, else 0; gbar[nz] =
// the overall mean (gbar holds nz + 1 values).
void launch_level_mean(const Grid &g, const double *part, int exact, double *gbar, hipStream_t s);
// out[i + nx j] = vertical mean of column (i, j) of f (FP64).
template <typename T>
void launch_column_mean(const Grid &g, const T *f, double *out, hipStream_t s);
// The vertically uniform part: pv solves the x-y compact Laplacian
// Lh pv = cmean - ctl->rhs_mean exactly (separable real Fourier transforms,
// tab_x[m] = cas(2 pi m / nx), tab_y alike; work: nx ny doubles), mean zero.
void launch_vertical_solve(const Grid &g, const double *cmean, const SolveCtl *ctl,
                           const double *tab_x, const double *tab_y, double *work, double *pv,
                           hipStream_t s);
// out = rhs_level - (cmean[i, j] - ctl->rhs_mean), FP64 rounded once (out
// may alias rhs_level).
template <typename T>
void launch_remove_columns(const Grid &g, const T *rhs_level, const double *cmean,
                           const SolveCtl *ctl, T *out, hipStream_t s);
// phi = (phi - dbar[k] - dv[i, j] + dbar[nz]) + pv[i, j] + (guess kept:
// guess - gbar[k] - gv[i, j] + gbar[nz]), FP64 rounded once, in place.
template <typename T>
void launch_combine(const Grid &g, T *phi, const double *dbar, const double *dv, const double *pv,
                    const T *guess, const double *gbar, const double *gv, const SolveCtl *ctl,
                    hipStream_t s);
// Storage-type profiles of a solution's horizontally uniform part pb
// (nullable): phigz = d_c pb/dz, cbar = App. A fourth difference in z, and
// with add_p pbar += rho0 pb; then pgz = d_c(alpha0 pbar)/dz.
template <typename T>
void launch_mean_profiles(const Grid &g, const double *pb, const double *rho0,
                          const double *alpha0, int add_p, double *pbar, T *phigz, T *cbar,
                          T *pgz, hipStream_t s);
// out = in - ctl->phi_mean (ctl nullable) + prof[k].
template <typename T>
void launch_add_profile(const Grid &g, const T *in, const SolveCtl *ctl, const double *prof,
                        T *out, hipStream_t s);
// rhs_out = rhs_in - rsub[k] (FP64, rounded once); partial sums of
// (rhs_in - ctl->rhs_mean)^2 (level_parts * nz of them); optional zeroing
// of phi0.
template <typename T>
void launch_rhs_center(const Grid &g, const T *rhs_in, T *rhs_out, T *phi0, const double *rsub,
                       const SolveCtl *ctl, double *partials, hipStream_t s);
// Reset the stopping state for a second pass of sweeps on the same rhs,
// with cap max_sweeps.
void launch_ctl_restart(SolveCtl *ctl, int max_sweeps, hipStream_t s);
// ctl->max_sweeps = max_sweeps (a kept guess's budget).
void launch_ctl_limit(SolveCtl *ctl, int max_sweeps, hipStream_t s);
// f = 0 (a fill kernel rather than a memset, so the call records no memset
// node when a caller captures the stream into a graph).
template <typename T>
void launch_zero(const Grid &g, T *f, hipStream_t s);

// S sweeps from (prev, cur) = (phi_{m-1}, phi_m) giving out_prev = phi_{m+S-1}
// (S >= 2, Chebyshev) and out_last = phi_{m+S}; check: FP64 partial sums of
// the residual of cur, one per block (tsweep_blocks of them).  first: sweep
// m is the first of the solve.  omega_cheb: S weights of sweeps m .. m+S-1.
// dec_m >= 0 (S == 1 only): block 0 also reduces the dec_np partials of an
// earlier checking launch of sweep dec_m and applies its stopping decision
// to ctl.  Outputs never alias inputs.
template <typename T>
void launch_tsweep(const Grid &g, int S, bool chebyshev, bool check, bool first,
                   double omega_jacobi, const double *omega_cheb, const T *cur, const T *prev,
                   T *out_last, T *out_prev, const T *rhs, SolveCtl *ctl, double *partials,
                   const double *dec_partials, int dec_np, int dec_m, int64_t *snap,
                   int snap_seq, hipStream_t s);

template <typename T>
void launch_project(const Grid &g, const Dyn<T> &d, const Profiles<T> &P, const T *phi,
                    const SolveCtl *ctl, T *u, T *v, T *w, T *p, hipStream_t s);

template <typename T>
void launch_sub_mean(const Grid &g, const T *in, const SolveCtl *ctl, T *out, hipStream_t s);

// phi0 = alpha0 (p - p_prev): the last step's pressure change as a guess.
template <typename T>
void launch_extrapolate(const Grid &g, const Profiles<T> &P, const T *p, const T *p_prev, T *phi0,
                        hipStream_t s);

// Starting iterate phi0 - gbar - gv (gbar: per-level means, gv: per-column
// means to remove, each nullable) of a solve of L phi = rhs (rhs centred),
// in defect form: rhs_d = rhs - L(phi0 - gbar - gv) (FP64 arithmetic; rhs_d
// may alias rhs), so the sweeps solve L delta = rhs_d from zero.  The iterate is kept if always_keep
// or ||rhs_d||_2 < ||rhs||_2 (the zero start's residual); otherwise rhs_d =
// rhs.  Sets ctl->guess_kept.
template <typename T>
void launch_guess_gate(const Grid &g, const T *rhs, const T *phi0, const double *gbar,
                       const double *gv, T *rhs_d, double *partials, SolveCtl *ctl,
                       int always_keep, hipStream_t s);
// phi += phi0 - gbar (FP64 sum, rounded once) when ctl->guess_kept.
template <typename T>
void launch_add_guess(const Grid &g, const T *phi0, const double *gbar, const SolveCtl *ctl,
                      T *phi, hipStream_t s);
// ctl->res_out2 = ||rhs - L phi||^2 in FP64 (the residual of a returned
// iterate).
template <typename T>
void launch_returned_residual(const Grid &g, const T *rhs, const T *phi, double *partials,
                              SolveCtl *ctl, hipStream_t s);

// Generic FP64 sums over n elements: mode 0 sum(a), 1 sum(a^2).
template <typename T>
void launch_block_sum(const T *a, int64_t n, int mode, double *partials, hipStream_t s);

// Final fixed-order reductions of `np` partials into the control block.
enum FinalOp {
  kFinalRhsMean = 0,   // ctl->rhs_mean = sum / n
  kFinalRhsNorm = 1,   // ctl->rhs_norm2, tol2; converged at once if zero
  kFinalCheck = 2,     // residual check at sweep m
  kFinalPhiMean = 3,   // ctl->phi_mean = sum / n
  kFinalStore = 4,     // out[slot] = sum
  kFinalReturned = 5   // ctl->res_out2 = sum
};
// The residual test of sweep m from its partials (kFinalCheck); snap (a
// device view of pinned host memory, nullable) receives (snap_seq << 32) |
// done after the decision, one 64-bit store.
void launch_final_check(const double *partials, int np, SolveCtl *ctl, double n, int m,
                        int64_t *snap, int snap_seq, hipStream_t s);
void launch_final(const double *partials, int np, int op, SolveCtl *ctl, double n, double tol2_scale,
                  int m, double *out, hipStream_t s);

void launch_ctl_reset(SolveCtl *ctl, int max_sweeps, int fixed, hipStream_t s);

// Per-level FP64 sums for the diagnostics: level_sums[k*kDiagStride + m],
// m = 0..8 horizontal sums of thl, qt, ql, u, v, w, w^2, w^3, b; 9 sum rho0 thl,
// 10 sum rho0 qt, 11 sum rho0 |u|^2/2, 12 sum div^2, 13 max |div|, 14 max CFL.
constexpr int kDiagStride = 16;
template <typename T>
void launch_diag(const Grid &g, const Dyn<T> &d, const Profiles<T> &P, const T *u, const T *v,
                 const T *w, const T *thl, const T *qt, const T *ql, const T *b,
                 double *level_sums, hipStream_t s);

}  // namespace lesmi
