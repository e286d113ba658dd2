/*
 * les.h — C ABI of the MI355X (gfx950) moist anelastic LES time step.
 *
 * Implements one time step of the anelastic moist LES of Chammas et al.,
 * "Accelerating large-eddy simulations of clouds with Tensor Processing
 * Units" (arXiv 2301.04698), Sec. 2: saturation adjustment (Sec. 2.2),
 * Smagorinsky-Lilly subgrid model (Sec. 2.3), QUICK advection, central
 * diffusion, the iterative predictor-corrector time scheme and the
 * pressure-correction Poisson equation solved by weighted-Jacobi sweeps
 * with the collocated-grid correction of App. A (Sec. 2.4).
 *
 * Conventions shared by every entry point:
 *  - Fields are cell-centred arrays of nx*ny*nz elements in DEVICE memory,
 *    index i + nx*(j + ny*k) (x fastest, z slowest), element type double
 *    for LES_FP64 and float for LES_FP32.  x and y are periodic; z has
 *    rigid walls at z = 0 and z = nz*dz.
 *  - The library allocates no device memory.  The caller owns the
 *    prognostic fields and one workspace of les_workspace_bytes() bytes;
 *    the handle owns host metadata, a small pinned host buffer and events.
 *  - Every call is ordered on the HIP stream given to les_init.  Calls that
 *    return host statistics synchronize that stream before returning.
 *  - Return codes: LES_OK (0), LES_WARN_NOT_CONVERGED (1: a Poisson solve
 *    hit its sweep cap; the best iterate is kept and the step goes on), or a
 *    negative error: LES_ERR_ARG (invalid argument, nothing launched),
 *    LES_ERR_HIP (a HIP call failed), LES_ERR_NONFINITE (NaN/Inf found by a
 *    norm), LES_ERR_STATE (handle unusable).  les_last_error() returns a
 *    thread-local message describing the last failure.
 *  - Errors leave the caller's buffers in an unspecified state.
 */
#ifndef LES_H
#define LES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
  LES_OK = 0,
  LES_WARN_NOT_CONVERGED = 1,
  LES_ERR_ARG = -1,
  LES_ERR_HIP = -2,
  LES_ERR_NONFINITE = -3,
  LES_ERR_STATE = -4
};

enum { LES_FP64 = 0, LES_FP32 = 1 };          /* storage / stencil precision */
enum { LES_JACOBI = 0, LES_CHEBYSHEV = 1 };   /* Poisson sweep weighting */
enum { LES_QUICK = 0, LES_WENO3 = 1 };       /* advection scheme */
enum { LES_NO_SLIP = 0, LES_FREE_SLIP = 1 };  /* u, v at the walls z = 0, H */
/* Share of the condensate that is liquid (Sec. 2.2): LES_PHASE_HEAVISIDE,
 * liquid at and above T_f and ice below (the paper's equations), or
 * LES_PHASE_RAMP, the continuous partition for mixed-phase clouds: linear
 * from all ice at T_ice to all liquid at T_f.  Saturation over ice uses the
 * sublimation heat Ls0; the saturation humidity of a partition is the
 * liquid-share-weighted mean of the two. */
enum { LES_PHASE_HEAVISIDE = 0, LES_PHASE_RAMP = 1 };
/* Uniform parts of each pressure-correction solve.  The compact Laplacian
 * maps a function of z alone to its second difference in z and commutes
 * with horizontal averaging, so the horizontal mean of the equation is a
 * one-dimensional Neumann problem; with mirror walls the z second
 * differences of a column sum to zero and vanish on a field constant in z,
 * so its vertical mean is the two-dimensional periodic x-y problem.  Both
 * decouple exactly from the other modes:
 *   LES_MEAN_SWEPT  the sweeps solve every mode (the paper's method as
 *                   written)
 *   LES_MEAN_LEVEL  the horizontally uniform part is solved exactly in FP64
 *                   (two running sums), its parts of phi and of the pressure
 *                   kept as FP64 profiles (see les_buffers.p); the sweeps
 *                   solve the rest from zero
 *   LES_MEAN_EXACT  as LES_MEAN_LEVEL, and the vertically uniform part is
 *                   solved exactly in FP64 too (a real Fourier transform of
 *                   each horizontal direction); the sweeps solve only the
 *                   modes with both horizontal and vertical structure, with
 *                   Chebyshev bounds for those (the slowest modes of these
 *                   grids are vertically uniform, so far fewer sweeps)
 * All meet the same residual test. */
enum { LES_MEAN_SWEPT = 0, LES_MEAN_LEVEL = 1, LES_MEAN_EXACT = 2 };
/* Initial guess of the pressure-correction solves:
 *   LES_GUESS_ZERO         phi_0 = 0 for every solve (the plain method)
 *   LES_GUESS_EXTRAPOLATE  first solve of a step: phi_0 = alpha0 (p^n -
 *                          p^{n-1}), the last step's pressure change; later
 *                          solves start from 0
 *   LES_GUESS_PREVIOUS     each sub-iteration's solve starts from the
 *                          previous step's solution of the same
 *                          sub-iteration (zero on the first step)
 *   LES_GUESS_LEARNED      as LES_GUESS_PREVIOUS, plus the correction of
 *                          the one-input guess network of les_cnn.h
 *                          (parameters bound with les_bind_cnn before the
 *                          second step)
 *   LES_GUESS_LEARNED3     first solve of a step: the three-input guess
 *                          network's guess from the previous pressures and
 *                          the divergence (base alpha0 (p^n - p^{n-1}) as
 *                          with LES_GUESS_EXTRAPOLATE, plus the network's
 *                          correction; parameters bound with les_bind_cnn
 *                          before the first step); later solves start from 0
 * The solve always runs to the same residual tolerance: a guess only
 * changes the number of sweeps, never the acceptance test. */
enum { LES_GUESS_ZERO = 0, LES_GUESS_EXTRAPOLATE = 1, LES_GUESS_PREVIOUS = 2,
       LES_GUESS_LEARNED = 3, LES_GUESS_LEARNED3 = 4 };

/* Run configuration.  nx >= 2, ny >= 1 (ny = 1: a two-dimensional x-z run)
 * and nz >= 4; one z plane of a field at most 2 GiB (nx*ny <= 2^29 in FP32,
 * 2^28 in FP64) and at most 2^34 cells, else LES_ERR_ARG.
 * Table 1 constants of the paper and forcing parameters are explicit so the
 * caller states every value (les_default_config fills Table 1). */
typedef struct les_config {
  int32_t nx, ny, nz;
  int32_t precision;            /* LES_FP64 or LES_FP32 */
  int32_t n_subiter;            /* predictor-corrector sub-iterations K >= 1 */
  int32_t poisson_scheme;       /* LES_JACOBI (fixed weight) or LES_CHEBYSHEV */
  int32_t poisson_check_every;  /* residual checked every m sweeps, m >= 1 */
  int32_t poisson_max_sweeps;   /* cap per solve */
  int32_t satadj_maxit;         /* secant iteration cap */
  int32_t sweeps_per_launch;    /* Poisson sweeps fused per kernel launch, 0..2
                                   (0: default); results do not depend on it */
  double dx, dy, dz, dt;        /* m, m, m, s; all > 0 */
  double poisson_tol;           /* stop when ||rhs - L phi||_2 <= tol ||rhs||_2 */
  double jacobi_omega;          /* 0 selects 2/(mu_min+mu_max) */
  /* Table 1 */
  double p00, theta0, Rd, Rv, cpd, cpv, cl, ci, Lv0, Ls0, Tf, fcor, g, cs, Pr, Sc;
  /* forcing: geostrophic wind, surface sensible/latent flux (W m^-2),
   * large-scale divergence (w_sub = D z, downward), sponge fraction and top
   * rate (s^-1), synthetic longwave flux F0 (W m^-2) and absorption
   * coefficient (m^2 kg^-1) */
  double ug, vg, shf, lhf, wsub_div, sponge_frac, sponge_max, rad_F0, rad_kappa;
  /* saturation vapour pressure anchor (Pa, K) and secant tolerance (K) */
  double e_tr, T_tr, satadj_tol;
  int32_t guess;                /* LES_GUESS_* */
  int32_t advection;            /* LES_QUICK (Sec. 2.4) or LES_WENO3 (third-order
                                   WENO faces, Lax-Friedrichs flux) */
  int32_t wall;                 /* LES_NO_SLIP (u, v mirror oddly across the
                                   walls) or LES_FREE_SLIP (evenly: zero wall
                                   stress, as in the Sec. 3 validation cases);
                                   w has zero wall flux either way */
  int32_t phase;                /* LES_PHASE_HEAVISIDE or LES_PHASE_RAMP */
  double nu_const;              /* > 0: uniform kinematic viscosity (m^2/s) in
                                   place of the Smagorinsky model (Sec. 3
                                   validation cases); scalars diffuse with
                                   nu/Pr and nu/Sc.  0: Smagorinsky */
  double T_ice;                 /* LES_PHASE_RAMP: all condensate is ice at
                                   and below T_ice (K), 0 < T_ice < Tf */
  int32_t mean_mode;            /* LES_MEAN_SWEPT, LES_MEAN_LEVEL or LES_MEAN_EXACT */
  int32_t guess_passes;         /* LES_GUESS_LEARNED: network passes per guessed
                                   solve, 1..4 (0 means 1); pass 2 onward feeds
                                   the previous pass's guess back as the base,
                                   so each pass corrects the residual the last
                                   one left.  Other guess modes: 0 or 1 */
} les_config;

/* Caller-owned device buffers.  u, v, w: velocity (m/s); thl: liquid-ice
 * potential temperature (K) stored at the half step; qt: total water
 * specific humidity (kg/kg) at the half step; p: pressure perturbation p'
 * (Pa) less the horizontally uniform pressure that LES_MEAN_LEVEL and
 * LES_MEAN_EXACT keep in the workspace as an FP64 profile (starts at zero
 * with les_init; with LES_MEAN_SWEPT it stays zero and p is p').  les_pressure returns the
 * whole p'.  workspace: at least les_workspace_bytes(cfg) bytes, 256-byte
 * aligned, not shared with another handle. */
typedef struct les_buffers {
  void *u, *v, *w, *thl, *qt, *p;
  void *workspace;
  size_t workspace_bytes;
} les_buffers;

typedef struct les_handle les_handle;

/* One Poisson solve. */
typedef struct les_solve_stats {
  int32_t sweeps;     /* sweeps applied to reach the returned iterate */
  int32_t status;     /* 0 converged, 1 sweep cap reached, -3 non-finite */
  double rhs_norm;    /* ||rhs||_2 after mean removal (FP64) */
  double res_norm;    /* ||rhs - L phi||_2 of the returned iterate (FP64) */
  double seconds;     /* device time of the solve (HIP events) */
  int32_t guess;      /* les_step: 0 started from zero, 1 from its guess,
                         2 its guess was rejected (residual not below the
                         zero start's) and it started from zero, 3 its kept
                         guess reached the cap, or its budget (the sweeps
                         of the last solve of the same sub-iteration that
                         ran from the zero start), or its returned iterate
                         missed the tolerance, and the sweeps were repeated
                         from the zero start (sweeps and seconds count both
                         passes), 4 its kept guess's sweeps met the test but
                         the returned iterate missed the tolerance, and the
                         solve continued once from that iterate as a new
                         guess (under the same budget, with none under the
                         first pass's count; should that miss again, it is
                         repeated from the zero start: 3);
                         les_poisson_solve: opts->use_guess.
                         "Zero start": phi = 0, or the exact uniform parts
                         (LES_MEAN_LEVEL, LES_MEAN_EXACT).  For a kept guess
                         res_norm is the residual of the returned iterate
                         (guess plus correction, as stored) */
  int32_t guess_sweeps; /* guess 3 and 4: the sweeps before the last pass */
} les_solve_stats;

typedef struct les_poisson_opts {
  int32_t fixed_sweeps;  /* > 0: apply exactly this many sweeps */
  int32_t use_guess;     /* 0: start from the zero start; 1: phi holds a
                            guess, always kept; 2: phi holds a guess, kept
                            and repeated as les_step does (see
                            les_solve_stats.guess) */
  int32_t budget;        /* use_guess 2: > 0 ends a kept guess's sweeps at
                            the first residual check at or beyond this many
                            sweeps, then repeats from the zero start (les_step
                            passes the sweeps of the last zero-start solve of
                            the same sub-iteration); 0 none */
} les_poisson_opts;

/* Optional per-call controls of les_step. */
typedef struct les_step_opts {
  const int32_t *replay_sweeps; /* host, nsteps*n_subiter entries or NULL:
                                   per-solve sweep counts to apply exactly */
  les_solve_stats *records;     /* host, nsteps*n_subiter entries or NULL */
  int32_t time_sweeps;          /* 1: time runs of consecutive plain sweeps
                                   (between residual checks) with HIP events */
  int32_t reserved;
  void *dump_rhs;               /* device, n_subiter*n elements or NULL: the
                                   right-hand sides the sweeps of the call's
                                   last step solved, sub-iteration k at
                                   offset k*n: centred, and with
                                   LES_MEAN_LEVEL or LES_MEAN_EXACT also
                                   without their horizontal mean per level */
  void *dump_phi;               /* device, n_subiter*n elements or NULL:
                                   those solves' zero-mean solutions, with
                                   LES_MEAN_LEVEL or LES_MEAN_EXACT without
                                   their horizontally uniform part */
  double *dump_mean;            /* host, n_subiter*(2*nz+1) doubles or NULL:
                                   per solve of the last step, the values the
                                   centring subtracted per level (the mean of
                                   the raw rhs, or with LES_MEAN_LEVEL and
                                   LES_MEAN_EXACT its horizontal mean per
                                   level), the
                                   horizontally uniform part of the solution
                                   (zero with LES_MEAN_SWEPT), and the mean
                                   of the raw rhs.  The whole centred rhs is
                                   dump_rhs + (first profile - mean) and the
                                   whole solution dump_phi + second profile */
  void *dump_base;              /* device, n_subiter*n elements or NULL: the
                                   field each solve of the last step started
                                   its guess from (the previous solution, or
                                   the extrapolated pressure change before
                                   any network correction; zero where the
                                   solve had no guess) */
} les_step_opts;

typedef struct les_step_stats {
  int32_t steps, solves;
  int64_t sweeps_total;
  int32_t sweeps_max;
  int32_t not_converged;        /* solves that hit the cap */
  double res_rel_max;           /* max over solves of res_norm / rhs_norm */
  double seconds;               /* device time of the whole call */
  double poisson_seconds;       /* device time inside the solves */
  double sweep_seconds;         /* time_sweeps: device time of the timed sweeps */
  int64_t sweeps_timed;         /* time_sweeps: number of sweeps in sweep_seconds */
} les_step_stats;

typedef struct les_diag {
  double mass_thl;   /* sum rho0 thl dV  (kg K) */
  double mass_qt;    /* sum rho0 qt dV   (kg) */
  double div_l2;     /* ||div_c(rho0 u)||_2 */
  double div_max;    /* max |div_c(rho0 u)| */
  double cfl;        /* max (|u| dt/dx + |v| dt/dy + |w| dt/dz) */
  double ke;         /* sum rho0 |u|^2 / 2 dV (J) */
} les_diag;

#define LES_NPROFILES 9  /* thl, qt, ql, u, v, w, w^2, w^3, b (horizontal means) */

/* Fills Table 1 of the paper and defaults for the rest (a 32^3 grid). */
void les_default_config(les_config *cfg);

/* Bytes of workspace needed for cfg (0 if cfg is invalid). */
size_t les_workspace_bytes(const les_config *cfg);

/* Byte offset inside the workspace of an intermediate field (debug and
 * tests); returns LES_ERR_ARG for an unknown field id.  Field ids:
 * 0 u^n, 1 v^n, 2 w^n, 3 thl^{n+1/2}, 4 qt^{n+1/2}, 5 thl_mid, 6 qt_mid,
 * 7..9 u,v,w at n+1/2, 10 b^{n+1/2}, 11 b_mid, 12 ql_mid, 13 c_pm*Pi (mid),
 * 14 nu scalars, 15 nu momentum, 16 radiative heating, 17 Poisson rhs,
 * 18..21 Poisson iterate buffers 0..3, 22 pressure of the previous step,
 * 23 starting iterate of a guessed solve, 24 its defect right-hand side. */
int les_workspace_offset(const les_config *cfg, int32_t field, size_t *offset);

/* Validates cfg and buffers, computes the reference state (Sec. 2.1) and
 * uploads it into the workspace.  The prognostic fields are read, never
 * written, by les_init: the caller fills them with the initial state. */
int les_init(const les_config *cfg, const les_buffers *bufs, void *hip_stream,
             les_handle **out);

/* Advances the state in the caller's buffers by nsteps time steps
 * (Sec. 2.4).  opts and stats may be NULL.  Synchronizes the stream. */
int les_step(les_handle *h, int32_t nsteps, const les_step_opts *opts, les_step_stats *stats);

/* Solves L phi = rhs (compact 7-point Laplacian, periodic x/y, Neumann z;
 * the pressure-correction equation of Sec. 2.4) by the configured sweeps.
 * rhs: device, n elements, read only (its mean is removed internally).
 * phi: device, n elements; in = guess if opts->use_guess, out = zero-mean
 * solution (with LES_MEAN_LEVEL or LES_MEAN_EXACT its horizontally
 * uniform part, solved exactly in FP64, is added before rounding once).  The sweeps solve for a
 * guess's correction from zero.  Uses the handle's workspace.
 * Synchronizes the stream. */
int les_poisson_solve(les_handle *h, const void *rhs, void *phi, const les_poisson_opts *opts,
                      les_solve_stats *stats);

/* The whole pressure perturbation p' (Sec. 2.4: the sum of the pressure
 * corrections rho0 phi of the solves): p_out (device, n elements of the
 * storage type, nullable) = p + pbar(z), rounded once; pbar_host (host, nz
 * doubles, nullable) = the FP64 profile pbar kept by LES_MEAN_LEVEL and
 * LES_MEAN_EXACT (zero with LES_MEAN_SWEPT).  Synchronizes the stream. */
int les_pressure(les_handle *h, void *p_out, double *pbar_host);

/* Restart with LES_MEAN_LEVEL or LES_MEAN_EXACT: sets the FP64
 * horizontally uniform pressure pbar (host, nz doubles, finite) that p is
 * taken relative to, e.g. the pbar_host of les_pressure on an earlier run
 * (les_init starts it at zero).  LES_ERR_STATE with LES_MEAN_SWEPT.
 * Synchronizes the stream. */
int les_set_pressure_profile(les_handle *h, const double *pbar_host);

/* Thermodynamic state of arbitrary fields (Sec. 2.1-2.2): temperature T,
 * liquid water q_l and buoyancy b from thl, qt at the handle's levels.
 * Device arrays of n elements; outputs may be NULL. */
int les_thermo(les_handle *h, const void *thl, const void *qt, void *T, void *ql, void *b);

/* Diagnostics of the current state: scalars into *out (host) and, if
 * profiles is non-NULL, LES_NPROFILES x nz horizontal means (host, FP64,
 * profile-major): the mean-state profiles of theta_l, q_t and liquid water
 * and the variance and skewness moments of w the paper compares for its
 * stratocumulus case (Sec. 4, fidelity of the simulation), the domain
 * integrals of rho0 theta_l and rho0 q_t that the scheme conserves (Sec.
 * 2.4), the kinetic energy, the central divergence and the CFL number.
 * FP64 reductions.  Synchronizes the stream. */
int les_diagnostics(les_handle *h, les_diag *out, double *profiles);

/* State the library keeps between les_step calls, beyond the caller's
 * fields: the FP64 horizontally uniform pressure of LES_MEAN_LEVEL and
 * LES_MEAN_EXACT, the
 * previous step's pressure (LES_GUESS_EXTRAPOLATE), the previous step's
 * solutions of each sub-iteration and which of them are held
 * (LES_GUESS_PREVIOUS, LES_GUESS_LEARNED), and the count of steps taken.
 * Together with the caller's u, v, w, thl, qt, p it is the whole state of a
 * run (the host does input and output only, Sec. 2.5), so a run can stop
 * and continue in another handle, process or machine: les_step on an
 * imported state gives bit for bit what the exporting handle's next steps
 * would.  A bound network (les_bind_cnn) is not part of it.
 * les_state_bytes: size of the exported state (0 if h is NULL).
 * les_export_state: writes it to dst (device, 256-byte aligned,
 * les_state_bytes(h) bytes).  les_import_state: reads one from src (device)
 * into a handle of the same grid, precision, mean mode, guess mode and
 * n_subiter (else LES_ERR_ARG); the caller's fields are not touched.  Both
 * synchronize the stream.  les_steps_done: the count of steps (-1 if h is
 * NULL). */
size_t les_state_bytes(const les_handle *h);
int les_export_state(les_handle *h, void *dst);
int les_import_state(les_handle *h, const void *src);
int64_t les_steps_done(const les_handle *h);

void les_destroy(les_handle *h);

const char *les_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* LES_H */
