/*
 * Serial FP64 CPU oracle of one time step of the moist anelastic LES
 * (Chammas et al., "Accelerating large-eddy simulations of clouds with
 * Tensor Processing Units", Sec. 2).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header or table with the GPU library and the GPU library never calls it.
 *
 * Arrays are cell-centred, float64, index i + nx*(j + ny*k) (x fastest).
 * Momentum inside the oracle is U = rho0*u as in the paper's conservation
 * form; the interface exchanges primitive velocities.
 */
#ifndef LES_ORACLE_H
#define LES_ORACLE_H
#include <stdint.h>

typedef struct ocfg {
  int32_t nx, ny, nz, n_subiter;
  int32_t poisson_scheme;      /* 0 = weighted Jacobi, 1 = Chebyshev-weighted Jacobi */
  int32_t poisson_check_every; /* residual checked every m sweeps */
  int32_t poisson_max_sweeps;
  int32_t satadj_maxit;
  int32_t guess;               /* initial guess of the solves, see oracle_step */
  int32_t advection;           /* 0 QUICK, 1 WENO3 with Lax-Friedrichs flux */
  int32_t wall;                /* u, v at z = 0, H: 0 no-slip (odd mirror), 1 free-slip (even) */
  int32_t phase;               /* condensate partition: 0 Heaviside at T_f, 1 linear ramp T_ice..T_f */
  int32_t mean_mode;           /* parts of each solve solved exactly first (see
                                  oracle_poisson): 0 none, 1 the horizontally uniform
                                  part, 2 also the vertically uniform part */
  int32_t reserved;
  double dx, dy, dz, dt;
  double poisson_tol;          /* ||rhs - L phi||_2 <= tol * ||rhs||_2 */
  double jacobi_omega;         /* 0 = closed-form optimum */
  /* Table 1 */
  double p00, theta0, Rd, Rv, cpd, cpv, cl, ci, Lv0, Ls0, Tf, fcor, g, cs, Pr, Sc;
  /* forcing */
  double ug, vg, shf, lhf, wsub_div, sponge_frac, sponge_max, rad_F0, rad_kappa;
  /* saturation vapour pressure anchor and secant stopping */
  double e_tr, T_tr, satadj_tol;
  double nu_const;             /* > 0: uniform kinematic viscosity in place of the SGS model */
  double T_ice;                /* phase 1: all condensate is ice at and below T_ice (K) */
} ocfg;

typedef struct osolve {        /* one Poisson solve */
  int32_t sweeps;              /* sweeps performed */
  int32_t status;              /* 0 converged, 1 not converged, -3 non-finite */
  double rhs_norm;             /* ||rhs||_2 after mean removal */
  double res_norm;             /* ||rhs - L phi||_2 of the returned iterate */
  int32_t guess;               /* oracle_step: 0 zero start, 1 guess kept, 2 rejected,
                                  3 kept but the cap or its budget was reached, solved
                                  again from the zero start (sweeps count both passes) */
  int32_t guess_sweeps;        /* guess 3: sweeps of the dropped guess's pass */
} osolve;

/* Reference state (Sec. 2.1): p0, T0, rho0, alpha0 at cell centres. */
int oracle_reference_state(const ocfg *c, double *p0, double *T0, double *rho0, double *alpha0);

/* Pointwise thermodynamics (Sec. 2.1, 2.2). */
double oracle_exner(const ocfg *c, double p0, double qt, double ql, double qi);
double oracle_theta_l(const ocfg *c, double T, double ql, double qi, double qt, double p0);
double oracle_qv_sat(const ocfg *c, double T, double p0);      /* over liquid */
double oracle_qv_sat_ice(const ocfg *c, double T, double p0);  /* over ice */
double oracle_liquid_fraction(const ocfg *c, double T);        /* share of condensate that is liquid */
double oracle_qv_star(const ocfg *c, double T, double p0);     /* saturation humidity of the partition */
int oracle_satadj(const ocfg *c, double thl, double qt, double p0,
                  double *T, double *ql, double *qi);
/* Field thermodynamics: T, q_l, q_i, b (all optional except inputs). */
int oracle_thermo(const ocfg *c, const double *thl, const double *qt,
                  double *T, double *ql, double *qi, double *b);

/* Operators (Sec. 2.3, 2.4, App. A).  Velocities primitive unless noted. */
int oracle_sgs_nu(const ocfg *c, const double *u, const double *v, const double *w,
                  const double *b, double *nu);
/* out = -div(U q), flux form, face values by c->advection. */
int oracle_advect(const ocfg *c, const double *U, const double *V, const double *W,
                  const double *q, double zparity, double *out);
/* Face value of the upwind reconstruction from (q_{l-1}, q_l, q_{l+1}),
 * taken on the upwind side of face l+1/2 (scheme 0 QUICK uses q_{l+1}
 * as its downwind point, scheme 1 WENO3). */
double oracle_face_value(int scheme, double qm1, double q0, double q1);
int oracle_diffuse(const ocfg *c, const double *nu, double inv_prandtl,
                   const double *q, double *out);
int oracle_sgs_momentum(const ocfg *c, const double *nu, const double *u, const double *v,
                        const double *w, double *fx, double *fy, double *fz);
int oracle_laplacian(const ocfg *c, const double *phi, double *out);
int oracle_app_a(const ocfg *c, const double *phi, double *out);
int oracle_divergence(const ocfg *c, const double *U, const double *V, const double *W,
                      double *out);
int oracle_radiation(const ocfg *c, const double *ql, const double *cpm_pi, double *out);

/* Poisson solve (Sec. 2.4): phi in = guess, out = zero-mean solution.
 * fixed_sweeps > 0 performs exactly that many sweeps.  With mean_mode >= 1
 * the horizontal mean of the equation, a one-dimensional Neumann problem in
 * z, is solved exactly first; with mean_mode 2 also its vertical mean, a
 * two-dimensional periodic problem (oracle_vertical_mode_solve); the sweeps
 * start from those solutions plus the guess with the same parts removed. */
int oracle_poisson(const ocfg *c, const double *rhs, double *phi, int32_t fixed_sweeps,
                   osolve *st);
/* The same solve as the time step runs it for a guess: the guess is kept
 * only if its residual is below the zero start's, and a kept guess whose
 * sweeps reach the cap, or (budget > 0) the first residual check at or
 * beyond `budget` sweeps, is dropped and the sweeps repeated from the zero
 * start (no fixed count); st->guess as in oracle_step's records. */
int oracle_poisson_gated(const ocfg *c, const double *rhs, double *phi, int32_t fixed_sweeps,
                         int32_t budget, osolve *st);
/* The two-dimensional periodic problem of the vertical mean (mean_mode 2):
 * Lh pv = rv on nx x ny, Lh the x and y part of the compact Laplacian, rv
 * with zero mean; pv with zero mean. */
int oracle_vertical_mode_solve(const ocfg *c, const double *rv, double *pv);
/* Closed-form extreme eigenvalues of -D^{-1} L on zero-mean fields (with
 * mean_mode 2, on the modes the sweeps act on). */
int oracle_jacobi_bounds(const ocfg *c, double *mu_min, double *mu_max);

/* Debug intermediates of the last sub-iteration of the last step (optional). */
typedef struct odebug {
  double *b_half;   /* buoyancy from the step-start scalars */
  double *nu;       /* momentum viscosity of the last sub-iteration */
  double *rhs;      /* Poisson right-hand side (mean removed) */
  double *phi;      /* Poisson solution (zero mean) */
  double *uhat, *vhat, *what; /* predicted primitive velocity */
} odebug;

/* nsteps time steps in place.  replay (nullable) gives per-solve sweep counts;
 * rec (nullable) receives nsteps*n_subiter solve records.
 * Initial guess of each solve by c->guess:
 *   0  zero;
 *   1  first solve of a step: alpha0 (p^n - p^{n-1}), the pressure change of
 *      the last step (zero on the first step of the call); later solves zero;
 *   2  each sub-iteration: the zero-mean solution of the same sub-iteration
 *      of the last step (zero on the first step of the call).
 * A guess is kept only if ||rhs - L phi_0||_2 is below the residual of the
 * zero start (rhs with its mean removed; with mean_mode = 1, rhs minus its
 * horizontal mean per level); otherwise the solve starts from the zero
 * start.  A kept guess whose solve reaches the sweep cap, or needs more
 * sweeps than the last solve of the same sub-iteration that ran from the
 * zero start (its budget), is dropped and the solve repeated from the zero
 * start (not with replayed sweep counts).
 * The guess changes the sweep count only: the stopping test is relative to
 * ||rhs||, whatever the starting iterate. */
int oracle_step(const ocfg *c, double *u, double *v, double *w, double *thl, double *qt,
                double *p, int32_t nsteps, const int32_t *replay, osolve *rec, odebug *dbg);

/* Diagnostics: scalars[0..5] = sum rho0*thl*dV, sum rho0*qt*dV, ||div_c(rho0 u)||_2,
 * max|div_c(rho0 u)|, max CFL, sum rho0*|u|^2/2*dV.  profiles (nullable) gets
 * 9 x nz horizontal means: thl, qt, ql, u, v, w, w^2, w^3, b. */
int oracle_diagnostics(const ocfg *c, const double *u, const double *v, const double *w,
                       const double *thl, const double *qt, double *scalars, double *profiles);

#endif
